"""EIFE1 and EIFE2 time stepping (oracle; test infrastructure only).

Section 2.2.  With steps tau_n and t_{n+1} = t_n + tau_n (uniform: tau_n = tau),
the EIFE1 scheme (eq. (2.13)) is
    u^{n+1} = e^{-tau L} u^n + tau phi_1(-tau L) P_h f(t_n, u^n)
and the EIFE2 scheme (eq. (2.14)), with node c2 in (0, 1], is
    U2      = e^{-c2 tau L} u^n + c2 tau phi_1(-c2 tau L) P_h f(t_n, u^n)
    u^{n+1} = e^{-tau L} u^n
              + tau [ (phi_1(-tau L) - phi_2(-tau L)/c2) P_h f(t_n, u^n)
                      + (phi_2(-tau L)/c2) P_h f(t_n + c2 tau, U2) ].
All operator functions act through a basis of `spectral` (z = -tau Lam).

The load P_h f(t, u_h) is read in one of two ways (the paper writes the load
tensor with entries (f(t, u_ijk), phi_i phi_j phi_k) in Section 4 but the
projection of f(u_h) in Section 2):
    "lumped" (default): F_i = f(t, u_i) * int phi_i = f(t, u_i) * prod_a h_a,
                        so P_h f = M^{-1} F
    "nodal":            P_h f is the interpolant with nodal values f(t, u_i).
"""
import numpy as np

from . import fem
from .phi import phi


def load_spectral(basis, f, t, U, X, load):
    val = f(t, X, U)
    val = np.broadcast_to(val, U.shape).astype(np.float64)
    if load == "lumped":
        return basis.load_to_spectral(val * float(np.prod(basis.h)))
    if load == "nodal":
        return basis.to_spectral(val)
    raise ValueError(load)


def run(basis, u0, f, tau, n_steps, stages, c2=0.5, t0=0.0, load="lumped",
        origin=None, callback=None, boundary=None):
    """Advance nodal values u0 by n_steps EIFE steps; returns nodal u^n.

    tau: one step size, or a sequence of per-step sizes tau_n (Section 2.2
    lets the step vary; every operator function is then formed with tau_n)
    whose length must equal n_steps.

    f(t, X, U) is the reaction, X the coordinate arrays of the interior nodes.
    callback(n, t_n, U) is called after every step when given.
    boundary: None (homogeneous data) or a pair (g, g_t) of callables of
    (t, Xb) giving the Dirichlet values and their time derivative at the
    boundary nodes (coordinates Xb of fem.boundary_coupling).  Then the load
    gains -Mb g_t(t) - Kb g(t) (Dirichlet grids only): the boundary values
    enter as part of f, evaluated at the same times as f.
    """
    if stages not in (1, 2):
        raise ValueError("stages must be 1 or 2")
    if not (0.0 < c2 <= 1.0):
        raise ValueError("c2 must lie in (0, 1]")
    X = fem.mesh(basis.N, basis.h, origin, getattr(basis, "bc", "dirichlet"))
    if boundary is not None:
        if getattr(basis, "bc", "dirichlet") != "dirichlet":
            raise ValueError("boundary data need a Dirichlet grid")
        Mb, Kb, Xb = fem.boundary_coupling(basis.N, basis.h, basis.D, origin)
        g_b, g_bt = boundary

        def load_at(t, U):
            extra = -(Mb @ g_bt(t, Xb) + Kb @ g_b(t, Xb))
            return load_spectral(basis, f, t, U, X, load) + basis.load_to_spectral(extra.reshape(basis.shape))
    else:
        def load_at(t, U):
            return load_spectral(basis, f, t, U, X, load)
    uniform = np.ndim(tau) == 0
    taus = np.full(n_steps, float(tau)) if uniform else np.asarray(tau, dtype=np.float64)
    if len(taus) != n_steps or np.any(taus <= 0.0):
        raise ValueError("need n_steps positive step sizes")
    cached = [None]

    def factors(tau_n):
        if cached[0] is None or cached[0][0] != tau_n:
            z = -tau_n * basis.lam
            f2 = (phi(2, z), phi(0, c2 * z), phi(1, c2 * z)) if stages == 2 else (None, None, None)
            cached[0] = (tau_n, phi(0, z), phi(1, z)) + f2
        return cached[0][1:]

    U = np.array(u0, dtype=np.float64).reshape(basis.shape)
    c = basis.to_spectral(U)
    tn = t0
    for n in range(n_steps):
        tau = float(taus[n])
        # t_n = t0 + n tau (uniform) or the running sum t0 + tau_0 + ... + tau_{n-1}
        tn = t0 + n * tau if uniform else (tn + float(taus[n - 1]) if n > 0 else t0)
        E, P1, P2, Ec, P1c = factors(tau)
        G1 = load_at(tn, U)
        if stages == 1:
            c = E * c + tau * P1 * G1
        else:
            c_stage = Ec * c + c2 * tau * P1c * G1
            U2 = basis.from_spectral(c_stage)
            G2 = load_at(tn + c2 * tau, U2)
            c = E * c + tau * ((P1 - P2 / c2) * G1 + (P2 / c2) * G2)
        U = basis.from_spectral(c)
        if callback is not None:
            callback(n + 1, tn + tau, U)
    return U
