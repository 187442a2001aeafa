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
    FourierBasis   periodic boundary conditions: the real orthonormal
                   Fourier (cosine / sine) basis of a library real FFT with
                   closed-form eigenvalues of the circulant 1D matrices (the
                   end of Section 4 prints sine vectors there; see the tests)
Spectral coefficients are tier-specific (eigenvector signs and degenerate
eigenspaces differ); tiers are compared in nodal space.  Tiers A and B take
bc = "dirichlet" or "periodic".
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

    def __init__(self, N, h, D, bc="dirichlet"):
        self.N, self.h, self.D, self.bc = list(N), list(h), float(D), bc
        self.shape = tuple(fem.n_unknowns(N[a], bc) for a in reversed(range(len(N))))
        M, K = fem.mass_stiffness(N, h, D, bc)
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

    def __init__(self, N, h, D, bc="dirichlet"):
        self.N, self.h, self.D, self.bc = list(N), list(h), float(D), bc
        d = len(N)
        self.d = d
        self.shape = tuple(fem.n_unknowns(N[a], bc) for a in reversed(range(d)))
        self.A, self.V, mus = [], [], []
        for a in range(d):
            A, B = fem.assemble_1d(N[a], h[a], bc)
            mu, V = scipy.linalg.eigh(B, A)
            self.A.append(A)
            self.V.append(V)
            mus.append(mu)
        lam = np.zeros(self.shape)
        for a in range(d):
            shp = [1] * d
            shp[d - 1 - a] = fem.n_unknowns(N[a], bc)
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


def fourier_freq(N):
    """Frequency k(r) of position r of the real Fourier basis of length N.

    Positions r = 0 .. N//2 hold cosines of frequency r; positions
    r = N//2 + 1 .. N - 1 (N - 1 - N//2 of them) hold sines of frequency
    N - r.  For even N, r = N/2 is the alternating vector (-1)^j."""
    r = np.arange(N)
    return np.where(r <= N // 2, r, N - r)


def fourier_eigs(N, h):
    """Closed-form eigenvalues of the periodic 1D matrices at every position.

    A and B are circulant (A = (h/6) circ(4, 1, ..., 1), B = (1/h) G^P), so
    cos(2 pi j k / N) and sin(2 pi j k / N) are eigenvectors with
    lambda^A = (h/6)(4 + 2 cos(2 pi k/N)) and lambda^B = (2/h)(1 - cos(2 pi k/N)).
    The end of Section 4 prints sine vectors and (i-1) pi / (2N) arguments for
    this case; the tests pin the circulant reading against the assembled
    matrices."""
    c = np.cos(2.0 * np.pi * fourier_freq(N) / N)
    return (h / 6.0) * (4.0 + 2.0 * c), (2.0 / h) * (1.0 - c)


def real_fourier(x, axis, inverse=False):
    """Orthonormal real Fourier transform of length n = x.shape[axis] along `axis`.

    Forward: with X = rfft(x, norm="ortho"), position 0 holds X_0, positions
    1 .. (n-1)//2 hold sqrt(2) Re X_k and positions n - k hold -sqrt(2) Im X_k
    (the coefficients of sqrt(2/n) cos and sqrt(2/n) sin), and for even n
    position n/2 holds X_{n/2}.  The inverse rebuilds X and calls irfft."""
    x = np.moveaxis(np.asarray(x, dtype=np.float64), axis, -1)
    n = x.shape[-1]
    kmax = (n - 1) // 2  # frequencies with both a cosine and a sine
    ks = np.arange(1, kmax + 1)
    if not inverse:
        X = np.fft.rfft(x, axis=-1, norm="ortho")
        out = np.empty(x.shape)
        out[..., 0] = X[..., 0].real
        out[..., ks] = np.sqrt(2.0) * X[..., ks].real
        out[..., n - ks] = -np.sqrt(2.0) * X[..., ks].imag
        if n % 2 == 0:
            out[..., n // 2] = X[..., n // 2].real
    else:
        X = np.zeros(x.shape[:-1] + (n // 2 + 1,), dtype=np.complex128)
        X[..., 0] = x[..., 0]
        X[..., ks] = (x[..., ks] - 1j * x[..., n - ks]) / np.sqrt(2.0)
        if n % 2 == 0:
            X[..., n // 2] = x[..., n // 2]
        out = np.fft.irfft(X, n=n, axis=-1, norm="ortho")
    return np.moveaxis(out, -1, axis)


class FourierBasis:
    """Tier C for periodic grids: the real orthonormal Fourier transform R along
    every axis with the closed-form eigenvalues of fourier_eigs, so that
    V_a = R^T diag(lamA)^{-1/2} (V^T A V = I, V^T B V = diag(lamB / lamA))."""

    def __init__(self, N, h, D, bc="periodic"):
        if bc != "periodic":
            raise ValueError("FourierBasis is the periodic basis")
        self.N, self.h, self.D, self.bc = list(N), list(h), float(D), bc
        d = len(N)
        self.d = d
        self.shape = tuple(N[a] for a in reversed(range(d)))
        lam = np.zeros(self.shape)
        self.sqA = np.ones(self.shape)
        for a in range(d):
            lamA, lamB = fourier_eigs(N[a], h[a])
            shp = [1] * d
            shp[d - 1 - a] = N[a]
            lam = lam + (lamB / lamA).reshape(shp)
            self.sqA = self.sqA * np.sqrt(lamA).reshape(shp)
        self.lam = self.D * lam

    def _apply(self, arr, inverse):
        out = arr.reshape(self.shape)
        for a in range(self.d):
            out = real_fourier(out, self.d - 1 - a, inverse)
        return out

    def to_spectral(self, u):
        return self.sqA * self._apply(u, False)

    def load_to_spectral(self, F):
        return self._apply(F, False) / self.sqA

    def from_spectral(self, c):
        return self._apply(c.reshape(self.shape) / self.sqA, True)


def make_basis(tier, N, h, D, bc="dirichlet", **kw):
    if tier == "C":
        return (FourierBasis if bc == "periodic" else SineBasis)(N, h, D, **kw)
    return {"A": DenseBasis, "B": KroneckerBasis}[tier](N, h, D, bc=bc, **kw)
