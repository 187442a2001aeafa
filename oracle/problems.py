"""Reaction terms and exact solutions of the test problems (oracle; test infrastructure only).

A reaction is a callable f(t, X, U): t the time, X the coordinate arrays of
the interior nodes (broadcastable to U), U the nodal values.
"""
import numpy as np


def zero():
    return lambda t, X, U: np.zeros_like(U)


def constant(c0):
    """u-independent, space- and time-constant forcing."""
    return lambda t, X, U: np.full_like(U, c0)


def affine_t(c0, c1):
    """u-independent forcing c0 + c1 t."""
    return lambda t, X, U: np.full_like(U, c0 + c1 * t)


def allen_cahn():
    """Allen-Cahn reaction u - u^3 (double-well potential; with D = eps^2)."""
    return lambda t, X, U: U - U ** 3


def flory_huggins(theta, theta_c):
    """Example 5.3 reaction (theta/2) ln((1 - u)/(1 + u)) + theta_c u, |u| < 1.

    Its positive root gamma (f(gamma) = 0) is the maximum bound of the
    solution; theta = 0.8, theta_c = 1.6 give gamma = 0.9575..."""
    return lambda t, X, U: 0.5 * theta * np.log((1.0 - U) / (1.0 + U)) + theta_c * U


def flory_huggins_bound(theta, theta_c):
    """Positive root of (theta/2) ln((1 - g)/(1 + g)) + theta_c g = 0 (bisection)."""
    lo, hi = 1e-12, 1.0 - 1e-15
    f = lambda g: 0.5 * theta * np.log((1.0 - g) / (1.0 + g)) + theta_c * g
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if f(mid) > 0.0:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


def _sine_product(X):
    s = 1.0
    for x in X:
        s = s * np.sin(np.pi * x)
    return s


def mms_u2(D):
    """Manufactured problem u_t = D Lap u + u^2 + g on (0,1)^d.

    Exact solution u = exp(-t) prod_a sin(pi x_a); substituting it gives
    g = (d pi^2 D - 1) e^{-t} s - e^{-2t} s^2 with s = prod_a sin(pi x_a).
    """
    def f(t, X, U):
        d = len(X)
        s = _sine_product(X)
        g = (d * np.pi ** 2 * D - 1.0) * np.exp(-t) * s - np.exp(-2.0 * t) * s * s
        return U * U + g
    return f


def mms_u2_exact(t, X):
    return np.exp(-t) * _sine_product(X)


def ex51():
    """Example 5.1 reaction: -pi^2/2 u + pi^2/2 e^{-pi^2 t} sin(pi x) sin(pi y), D = 1/2."""
    def f(t, X, U):
        x, y = X
        return (-0.5 * np.pi ** 2 * U
                + 0.5 * np.pi ** 2 * np.exp(-np.pi ** 2 * t) * np.sin(np.pi * x) * np.sin(np.pi * y))
    return f


def ex51_exact(t, X):
    """Example 5.1 exact solution e^{-pi^2 t} (sin(pi x) - 1) sin(pi y)."""
    x, y = X
    return np.exp(-np.pi ** 2 * t) * (np.sin(np.pi * x) - 1.0) * np.sin(np.pi * y)


def ex51_exact_grad(t, X):
    x, y = X
    e = np.exp(-np.pi ** 2 * t)
    return (e * np.pi * np.cos(np.pi * x) * np.sin(np.pi * y),
            e * (np.sin(np.pi * x) - 1.0) * np.pi * np.cos(np.pi * y))


EX51_ORIGIN = (0.5, 0.0)
EX51_D = 0.5


def traveling_wave(eps):
    """Example 5.2 reaction (u - u^3) / eps^2 (the equation u_t = Lap u + f, D = 1)."""
    return lambda t, X, U: (U - U ** 3) / (eps * eps)


def traveling_wave_solution(eps):
    """Example 5.2 exact solution and its derivatives, functions of (t, x):
    u = (1 - tanh(xi)) / 2 with xi = (x - s t) / (2 sqrt(2) eps), s = 3 / (sqrt(2) eps);
    u_t = s / (4 sqrt(2) eps) sech^2(xi), u_x = -1 / (4 sqrt(2) eps) sech^2(xi).
    It depends on x only; the Dirichlet data are its values on the boundary."""
    w = 2.0 * np.sqrt(2.0) * eps
    s = 3.0 / (np.sqrt(2.0) * eps)

    def u(t, x):
        return 0.5 * (1.0 - np.tanh((x - s * t) / w))

    def sech2(t, x):
        return 1.0 / np.cosh((x - s * t) / w) ** 2

    def u_t(t, x):
        return 0.5 * s / w * sech2(t, x)

    def u_x(t, x):
        return -0.5 / w * sech2(t, x)

    return u, u_t, u_x


def linear_in_time_data(coef):
    """Closed-form check of the boundary lifting: with l(x) = c_0 + sum_a c_{a+1} x_a,
    f = l(x) (independent of u and t) and Dirichlet data g = t l(x), the solution
    of u_t = D Lap u + f is u = t l(x) for every D (Lap l = 0)."""
    def l(X):
        v = coef[0]
        for a, x in enumerate(X):
            v = v + coef[a + 1] * x
        return v

    f = lambda t, X, U: np.broadcast_to(l(X), np.shape(U)).astype(np.float64)
    g = lambda t, Xb: t * l(Xb)
    g_t = lambda t, Xb: l(Xb) + 0.0 * Xb[0]
    return f, g, g_t, l
