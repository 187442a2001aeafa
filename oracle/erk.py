"""General s-stage explicit exponential Runge-Kutta steps (oracle; test infrastructure only).

Section 2.2, eq. (2.2): for nodes c_1 = 0 < ... (distinct, in [0, 1]) and
z = -tau L,
    U_i     = chi_i(z) u^n + tau sum_{j<i} a_ij(z) G_j,   G_i = P_h f(t_n + c_i tau, U_i),
    u^{n+1} = chi(z) u^n + tau sum_i b_i(z) G_i,
with chi = e^z, chi_i = e^{c_i z} and the interpolatory weights
    b_i(z)  = int_0^1 e^{(1-theta) z} l_i(theta) d theta,
    a_ij(z) = (1/tau) int_0^{c_i tau} e^{(c_i tau - sigma) z / tau} l_j^{(i)}(sigma / tau) d sigma.
b_i uses the Lagrange polynomials l_i of all s nodes.  For a_ij the paper
writes l_j as well, but its consistency conditions (eq. (2.3)) require
sum_{j<i} a_ij = c_i phi_1(c_i z), which holds only when the l_j^{(i)} are the
Lagrange polynomials of the nodes c_1 .. c_{i-1} that the sum runs over; that
is the reading taken here.

With l(theta) = sum_k beta_k theta^{k-1}, the integral definition of phi_k gives
    int_0^1 e^{(1-theta) z} theta^{k-1} d theta = (k-1)! phi_k(z),
so b_i(z) = sum_k beta_ik (k-1)! phi_k(z), and substituting sigma = c_i tau theta,
    a_ij(z) = sum_k alpha_ijk c_i^k (k-1)! phi_k(c_i z).
s = 1 is EIFE1 (eq. (2.13)); s = 2 with nodes (0, c2) is EIFE2 (eq. (2.14)).
"""
from math import factorial

import numpy as np

from . import fem
from .phi import phi
from .stepper import load_spectral


def lagrange_coefficients(nodes, j):
    """Coefficients beta_k (of theta^{k-1}, k = 1 .. len(nodes)) of the Lagrange
    polynomial that is 1 at nodes[j] and 0 at the other nodes."""
    others = [c for m, c in enumerate(nodes) if m != j]
    poly = np.array([1.0])  # ascending powers
    for c in others:
        poly = np.convolve(poly, np.array([-c, 1.0])) / (nodes[j] - c)
    return poly


def weights(nodes, z):
    """chi_i, a_ij and b_i of eq. (2.2) as arrays over z (a_ij for j < i only)."""
    s = len(nodes)
    b = []
    for i in range(s):
        beta = lagrange_coefficients(nodes, i)
        b.append(sum(beta[k - 1] * factorial(k - 1) * phi(k, z) for k in range(1, s + 1)))
    a = {}
    for i in range(1, s):
        ci = nodes[i]
        sub = list(nodes[:i])
        for j in range(i):
            alpha = lagrange_coefficients(sub, j)
            a[i, j] = sum(alpha[k - 1] * ci ** k * factorial(k - 1) * phi(k, ci * z) for k in range(1, i + 1))
    chi_i = [phi(0, c * z) for c in nodes]
    return chi_i, a, b, phi(0, z)


def run(basis, u0, f, tau, n_steps, nodes, t0=0.0, load="lumped", origin=None):
    """n_steps steps of the s-stage scheme with the given nodes (nodes[0] = 0).

    tau: one step size (t_n = t0 + n tau) or a sequence of n_steps sizes tau_n
    (t_{n+1} = t_n + tau_n, every weight formed with tau_n)."""
    nodes = [float(c) for c in nodes]
    if nodes[0] != 0.0 or len(set(nodes)) != len(nodes) or not all(0.0 <= c <= 1.0 for c in nodes):
        raise ValueError("nodes must be distinct, in [0, 1], the first one 0")
    X = fem.mesh(basis.N, basis.h, origin, getattr(basis, "bc", "dirichlet"))
    uniform = np.ndim(tau) == 0
    taus = np.full(n_steps, float(tau)) if uniform else np.asarray(tau, dtype=np.float64)
    if len(taus) != n_steps or np.any(taus <= 0.0):
        raise ValueError("need n_steps positive step sizes")
    s = len(nodes)
    U = np.array(u0, dtype=np.float64).reshape(basis.shape)
    c = basis.to_spectral(U)
    tn, cached = t0, (None, None)
    for n in range(n_steps):
        tau = float(taus[n])
        tn = t0 + n * tau if uniform else (tn + float(taus[n - 1]) if n > 0 else t0)
        if cached[0] != tau:
            cached = (tau, weights(nodes, -tau * basis.lam))
        chi_i, a, b, chi = cached[1]
        G = []
        for i in range(s):
            ci = chi_i[i] * c + tau * sum(a[i, j] * G[j] for j in range(i)) if i else c
            Ui = basis.from_spectral(ci) if i else U
            G.append(load_spectral(basis, f, tn + nodes[i] * tau, Ui, X, load))
        c = chi * c + tau * sum(b[i] * G[i] for i in range(s))
        U = basis.from_spectral(c)
    return U
