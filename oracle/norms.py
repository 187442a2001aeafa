"""Error norms and energy (oracle; test infrastructure only).

The paper reports ||u(t_n) - u_h^n||_0 and ||u(t_n) - u_h^n||_1 (Section 5.1)
without naming a quadrature.  Two versions are provided:
  * discrete: for a nodal error vector e, ||e||_0^2 = e^T M e and
    ||e||_1^2 = e^T M e + e^T K_1 e with K_1 the stiffness matrix for D = 1
    (the full H1 norm of the finite element function with those nodal values);
  * quadrature: the error between an exact solution and the Q1 function with
    the given nodal values (zero on the boundary), integrated with 4x4 Gauss
    points per element (2D only).
"""
import numpy as np

from . import fem


def discrete_norms(N, h, e, bc="dirichlet"):
    """Return (L2, H1, max) of the finite element function with nodal values e."""
    M, K1 = fem.mass_stiffness(N, h, 1.0, bc)
    v = np.asarray(e, dtype=np.float64).reshape(-1)
    m2 = float(v @ (M @ v))
    k2 = float(v @ (K1 @ v))
    return np.sqrt(m2), np.sqrt(m2 + k2), float(np.max(np.abs(v))) if v.size else 0.0


def allen_cahn_energy(N, h, D, U):
    """Discrete Allen-Cahn energy (D/2) U^T K_1 U + sum_i prod(h) (U_i^2 - 1)^2 / 4.

    The paper defines an energy only for its Flory-Huggins example; this is
    the double-well analogue with the gradient term taken from the stiffness
    matrix and the potential by nodal quadrature over interior nodes.
    """
    _, K1 = fem.mass_stiffness(N, h, 1.0)
    v = np.asarray(U, dtype=np.float64).reshape(-1)
    grad = 0.5 * D * float(v @ (K1 @ v))
    pot = float(np.prod(h)) * float(np.sum(0.25 * (v * v - 1.0) ** 2))
    return grad + pot


def flory_huggins_energy(N, h, D, U, theta, theta_c, bc="periodic"):
    """Discrete Example 5.3 energy: (D/2) U^T K_1 U + prod(h) sum_i F(U_i) with
    F(u) = (theta/2)((1 + u) ln(1 + u) + (1 - u) ln(1 - u)) - (theta_c/2) u^2,
    the gradient term from the stiffness matrix and the potential by nodal
    quadrature (Section 5.2 states the continuous functional)."""
    _, K1 = fem.mass_stiffness(N, h, 1.0, bc)
    v = np.asarray(U, dtype=np.float64).reshape(-1)
    grad = 0.5 * D * float(v @ (K1 @ v))
    F = 0.5 * theta * ((1.0 + v) * np.log1p(v) + (1.0 - v) * np.log1p(-v)) - 0.5 * theta_c * v * v
    return grad + float(np.prod(h)) * float(np.sum(F))


def quadrature_errors_2d(N, h, origin, U, exact, exact_grad, t, chunk_rows=64):
    """Continuous L2 and H1 errors between exact(t, .) and the Q1 function of U (2D).

    4x4 Gauss points per rectangle; the Q1 function takes nodal values U at
    interior nodes and 0 at boundary nodes.
    """
    Nx, Ny = N
    hx, hy = h
    ax, ay = origin
    full = np.zeros((Ny + 1, Nx + 1))
    full[1:Ny, 1:Nx] = np.asarray(U).reshape(Ny - 1, Nx - 1)
    g, w = np.polynomial.legendre.leggauss(4)
    g = (g + 1.0) / 2.0
    w = w / 2.0
    l2 = 0.0
    semi = 0.0
    for r0 in range(0, Ny, chunk_rows):
        r1 = min(Ny, r0 + chunk_rows)
        v00 = full[r0:r1, 0:Nx]
        v10 = full[r0:r1, 1:Nx + 1]
        v01 = full[r0 + 1:r1 + 1, 0:Nx]
        v11 = full[r0 + 1:r1 + 1, 1:Nx + 1]
        x0 = ax + hx * np.arange(Nx)[None, :]
        y0 = ay + hy * np.arange(r0, r1)[:, None]
        for i in range(4):
            for j in range(4):
                xi, eta = g[i], g[j]
                wt = w[i] * w[j] * hx * hy
                uh = ((1 - xi) * (1 - eta) * v00 + xi * (1 - eta) * v10
                      + (1 - xi) * eta * v01 + xi * eta * v11)
                dux = ((1 - eta) * (v10 - v00) + eta * (v11 - v01)) / hx
                duy = ((1 - xi) * (v01 - v00) + xi * (v11 - v10)) / hy
                X = (x0 + xi * hx, y0 + eta * hy)
                ue = exact(t, X)
                gx, gy = exact_grad(t, X)
                l2 += wt * float(np.sum((ue - uh) ** 2))
                semi += wt * float(np.sum((gx - dux) ** 2 + (gy - duy) ** 2))
    return np.sqrt(l2), np.sqrt(l2 + semi)


def quadrature_errors(N, h, origin, U, exact, exact_grad, t, npts=4):
    """Continuous L2 and H1 errors between exact(t, .) and the Q1 function whose
    interior nodal values are U and whose boundary nodal values are the exact
    solution's (nonhomogeneous Dirichlet data), any d.

    npts Gauss points per axis and element.  exact(t, X) and exact_grad(t, X)
    (a list with one array per axis) take coordinate arrays broadcast to the
    quadrature points.  Returns (L2, H1) with H1^2 = L2^2 + |grad error|^2.
    """
    d = len(N)
    origin = [0.0] * d if origin is None else list(origin)
    shape_all = tuple(N[a] + 1 for a in reversed(range(d)))
    coords = np.meshgrid(*[origin[a] + h[a] * np.arange(N[a] + 1) for a in reversed(range(d))], indexing="ij")
    Xall = [coords[d - 1 - a] for a in range(d)]
    full = np.array(exact(t, Xall), dtype=np.float64) * np.ones(shape_all)
    inner = tuple(slice(1, N[a]) for a in reversed(range(d)))
    full[inner] = np.asarray(U, dtype=np.float64).reshape(tuple(N[a] - 1 for a in reversed(range(d))))
    gq, wq = np.polynomial.legendre.leggauss(npts)
    gq = (gq + 1.0) / 2.0
    wq = wq / 2.0

    def at_points(deriv_axis):
        # value (or derivative along deriv_axis) of the Q1 function at every
        # quadrature point: shape = cells in array order (N_{d-1}, ..., N_0),
        # then one quadrature axis per mesh axis (0, 1, ..., d-1)
        arr = full
        for ax in range(d):
            k = d - 1 - ax
            lo = np.take(arr, np.arange(0, N[ax]), axis=k)
            hi = np.take(arr, np.arange(1, N[ax] + 1), axis=k)
            if ax == deriv_axis:
                arr = np.stack([(hi - lo) / h[ax]] * npts, axis=-1)
            else:
                arr = np.stack([lo * (1.0 - g) + hi * g for g in gq], axis=-1)
        return arr

    uh = at_points(-1)
    pts, w = [], 1.0
    for ax in range(d):
        xq = origin[ax] + h[ax] * (np.arange(N[ax])[:, None] + gq[None, :])  # (cells, q)
        shp = [1] * (2 * d)
        shp[d - 1 - ax] = N[ax]
        shp[d + ax] = npts
        pts.append(xq.reshape(shp))
        wshp = [1] * (2 * d)
        wshp[d + ax] = npts
        w = w * (wq * h[ax]).reshape(wshp)
    l2 = float(np.sum(w * (uh - exact(t, pts)) ** 2))
    grads = exact_grad(t, pts)
    semi = 0.0
    for ax in range(d):
        semi += float(np.sum(w * (at_points(ax) - grads[ax]) ** 2))
    return np.sqrt(l2), np.sqrt(l2 + semi)
