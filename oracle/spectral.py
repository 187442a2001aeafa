"""Bases diagonalising the pair (K, M) (oracle; test infrastructure only).

Section 2.1, eq. (2.7): L_h is defined by a(w, v) = (L_h w, v) on V_h, so in
nodal coordinates L_h = M^{-1} K.  With generalised eigenpairs K V = M V Lam,
V^T M V = I, every operator function is
    psi(-tau L_h) v = V psi(-tau Lam) V^T M v,
and for a load vector F (entries (f, phi_i)) the projection P_h f has nodal
values M^{-1} F, so psi(-tau L_h) P_h f = V psi(-tau Lam) V^T F.

Each basis exposes
    lam                 eigenvalues (array shaped like a nodal array)
    to_spectral(u)      V^T M u
    load_to_spectral(F) V^T F
    from_spectral(c)    V c
Three tiers compute the same thing by different routes:
    DenseBasis     dense generalised eigendecomposition of the assembled
                   matrices (the definition written out; small grids only)
    KroneckerBasis per-axis dense eigendecomposition of (B, A), applied as
                   tensor mode products (Section 4, eq. (4.2))
    SineBasis      the orthonormal type-I sine transform of a library FFT
                   with closed-form eigenvalues (Section 4, after the
                   printed formulas are corrected; see the tests)
Spectral coefficients are tier-specific (eigenvector signs and degenerate
eigenspaces differ); tiers are compared in nodal space.
"""
import numpy as np
import scipy.fft
import scipy.linalg

from . import fem


def _mode_product(mat, arr, axis, d):
    """(mat applied along grid axis `axis`) of an array with x fastest."""
    ax = d - 1 - axis
    out = np.tensordot(mat, arr, axes=([1], [ax]))
    return np.moveaxis(out, 0, ax)


class DenseBasis:
    """Tier A: scipy.linalg.eigh(K, M) on the assembled dense matrices."""

    def __init__(self, N, h, D):
        self.N, self.h, self.D = list(N), list(h), float(D)
        self.shape = tuple(N[a] - 1 for a in reversed(range(len(N))))
        M, K = fem.mass_stiffness(N, h, D)
        self.M = M.toarray()
        self.K = K.toarray()
        lam, V = scipy.linalg.eigh(self.K, self.M)
        self.lam = lam
        self.V = V

    def to_spectral(self, u):
        return self.V.T @ (self.M @ u.reshape(-1))

    def load_to_spectral(self, F):
        return self.V.T @ F.reshape(-1)

    def from_spectral(self, c):
        return (self.V @ c).reshape(self.shape)


class KroneckerBasis:
    """Tier B: per-axis generalised eigenpairs of (B_a, A_a), V = (x) V_a."""

    def __init__(self, N, h, D):
        self.N, self.h, self.D = list(N), list(h), float(D)
        d = len(N)
        self.d = d
        self.shape = tuple(N[a] - 1 for a in reversed(range(d)))
        self.A, self.V, mus = [], [], []
        for a in range(d):
            A, B = fem.assemble_1d(N[a], h[a])
            mu, V = scipy.linalg.eigh(B, A)
            self.A.append(A)
            self.V.append(V)
            mus.append(mu)
        lam = np.zeros(self.shape)
        for a in range(d):
            shp = [1] * d
            shp[d - 1 - a] = N[a] - 1
            lam = lam + mus[a].reshape(shp)
        self.lam = self.D * lam
        self.mus = mus

    def _apply(self, mats, arr):
        out = arr.reshape(self.shape)
        for a in range(self.d):
            out = _mode_product(mats[a], out, a, self.d)
        return out

    def to_spectral(self, u):
        return self._apply([self.V[a].T @ self.A[a] for a in range(self.d)], u)

    def load_to_spectral(self, F):
        return self._apply([self.V[a].T for a in range(self.d)], F)

    def from_spectral(self, c):
        return self._apply(self.V, c)


def sine_eigs(N, h):
    """Closed-form 1D eigenvalues of A and B in the sine basis.

    Section 4 prints lambda^A_i = (h/6)(6 - 4 sin(i pi/(2N))) and
    lambda^B_i = (4/h) sin^2(i pi/(2N)) with P_ij = sin(ij pi/N).  The mass
    eigenvalue needs the sine squared, (h/6)(6 - 4 sin^2) = (h/6)(4 + 2 cos(i pi/N)),
    and P must be scaled by sqrt(2/N) to be orthogonal; the tests check both
    readings against the assembled matrices.
    """
    k = np.arange(1, N)
    s2 = np.sin(k * np.pi / (2.0 * N)) ** 2
    lamA = (h / 6.0) * (6.0 - 4.0 * s2)
    lamB = (4.0 / h) * s2
    return lamA, lamB


class SineBasis:
    """Tier C: orthonormal DST-I (scipy.fft) with closed-form eigenvalues.

    With S the orthonormal sine matrix, A = S diag(lamA) S and B = S diag(lamB) S,
    so V_a = S diag(lamA)^{-1/2} satisfies V^T A V = I, V^T B V = diag(lamB/lamA).
    """

    def __init__(self, N, h, D, workers=-1):
        self.N, self.h, self.D = list(N), list(h), float(D)
        d = len(N)
        self.d = d
        self.shape = tuple(N[a] - 1 for a in reversed(range(d)))
        self.workers = workers
        lam = np.zeros(self.shape)
        self.sqA = np.ones(self.shape)
        for a in range(d):
            lamA, lamB = sine_eigs(N[a], h[a])
            shp = [1] * d
            shp[d - 1 - a] = N[a] - 1
            lam = lam + (lamB / lamA).reshape(shp)
            self.sqA = self.sqA * np.sqrt(lamA).reshape(shp)
        self.lam = self.D * lam

    def _dst(self, arr):
        return scipy.fft.dstn(arr, type=1, norm="ortho", workers=self.workers)

    def to_spectral(self, u):
        return self.sqA * self._dst(u.reshape(self.shape))

    def load_to_spectral(self, F):
        return self._dst(F.reshape(self.shape)) / self.sqA

    def from_spectral(self, c):
        return self._dst(c.reshape(self.shape) / self.sqA)


def make_basis(tier, N, h, D, **kw):
    return {"A": DenseBasis, "B": KroneckerBasis, "C": SineBasis}[tier](N, h, D, **kw)
