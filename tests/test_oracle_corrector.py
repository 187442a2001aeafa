"""Pins of the FP64 corrector reference (CPU).

Forward: every layer rebuilt from scipy.signal.correlate2d (an independent
route to the same zero-padded 3x3 cross-correlations).  Gradients: central
finite differences of the loss.  Adam: the closed form under a constant
gradient.  Indicator: a hand-computed case.
"""
import numpy as np
import pytest
from scipy.signal import correlate2d

from oracle import corrector as cr


def _data(seed, B=2, ny=6, nx=7):
    rng = np.random.default_rng(seed)
    un = rng.uniform(-0.9, 0.9, (B, ny, nx))
    uc = un + 0.1 * rng.standard_normal((B, ny, nx))
    uf = uc + 0.01 * rng.standard_normal((B, ny, nx))
    return un, uc, uf


def _params(seed):
    rng = np.random.default_rng(seed)
    p = cr.init_params(seed)
    # nonzero biases, so that each term of the layout is exercised
    return p + 0.05 * rng.standard_normal(p.shape)


def test_layout():
    assert cr.N_PARAMS == 576 + 32 + 4 * (9216 + 32) + 288 + 1 == 37889
    p = _params(0)
    assert np.array_equal(cr.pack(cr.unpack(p)), p)


def _kernel(Wt):
    """[9] tap weights -> 3x3 correlation kernel K[dy + 1][dx + 1]."""
    return np.asarray(Wt).reshape(3, 3)


def test_forward_matches_scipy_correlate2d():
    un, uc, _ = _data(1)
    p = _params(2)
    o, acts = cr.forward(p, un, uc)
    L = cr.unpack(p)
    B = un.shape[0]
    c = np.sqrt(np.mean((uc - un) ** 2, axis=(1, 2))) + 1e-30
    X = np.stack([uc, (uc - un) / c[:, None, None]], -1)
    W1, b1 = L[0]
    Y = np.zeros(un.shape + (cr.C,))
    for b in range(B):
        for oc in range(cr.C):
            z = b1[oc] + sum(correlate2d(X[b, :, :, c], _kernel(W1[:, c, oc]), mode="same") for c in range(2))
            Y[b, :, :, oc] = np.maximum(z, 0)
    assert np.allclose(Y, acts[1], rtol=1e-12, atol=1e-12)
    for li in range(1, 1 + cr.N_MID):
        W, bias = L[li]
        Yn = np.zeros_like(Y)
        for b in range(B):
            for oc in range(cr.C):
                z = bias[oc] + sum(correlate2d(Y[b, :, :, ic], _kernel(W[:, oc, ic]), mode="same")
                                   for ic in range(cr.C))
                Yn[b, :, :, oc] = np.maximum(z, 0)
        assert np.allclose(Yn, acts[li + 1], rtol=1e-12, atol=1e-12)
        Y = Yn
    W6, b6 = L[-1]
    ref = np.stack([b6[0] + sum(correlate2d(Y[b, :, :, ic], _kernel(W6[:, ic]), mode="same") for ic in range(cr.C))
                    for b in range(B)])
    assert np.allclose(ref, o, rtol=1e-12, atol=1e-12)


def test_zero_weights_give_the_output_bias():
    un, uc, _ = _data(3)
    p = np.zeros(cr.N_PARAMS)
    p[-1] = 0.25
    o, _ = cr.forward(p, un, uc)
    assert np.all(o == 0.25)


def test_gradient_matches_central_differences():
    un, uc, uf = _data(4)
    p = _params(5)
    s = 0.05
    loss, g = cr.loss_and_grad(p, un, uc, uf, s)
    rng = np.random.default_rng(6)
    # indices spread over every layer's weights and biases
    bounds = np.cumsum([0] + cr.SIZES)
    idx = [int(rng.integers(lo, hi)) for lo, hi in zip(bounds[:-1], bounds[1:]) for _ in range(4)]
    eps = 1e-6
    for i in idx:
        pp, pm = p.copy(), p.copy()
        pp[i] += eps
        pm[i] -= eps
        fd = (cr.loss_and_grad(pp, un, uc, uf, s)[0] - cr.loss_and_grad(pm, un, uc, uf, s)[0]) / (2 * eps)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)) + 1e-9, (i, fd, g[i])


def test_adam_constant_gradient_closed_form():
    """With a constant gradient g the bias-corrected moments are g and g^2, so each
    step moves p by -lr g / (|g| + eps)."""
    g = np.array([0.3, -2.0, 1e-3])
    p = np.zeros(3)
    opt = cr.Adam(3)
    for k in range(1, 6):
        p = opt.step(p, g, 0.01)
        assert np.allclose(p, -0.01 * k * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=0)


def test_indicator_hand_case():
    un = np.zeros((2, 2))
    uc = np.array([[0.5, 0.0], [0.0, 0.0]])
    delta = np.array([[0.0, 0.1], [0.0, 0.0]])
    r, umax, crms = cr.indicator(un, uc, delta)
    assert r == pytest.approx(0.1 / 0.5, rel=1e-10)
    assert umax == 0.5
    assert crms == pytest.approx(0.25, rel=1e-12)


def test_output_is_relative_to_the_coarse_change():
    """Scaling the change u_c - u_n by k (same u_c) leaves the features but the
    scale c, so delta scales by k."""
    un, uc, _ = _data(9)
    p = _params(10)
    un2 = uc - 3.0 * (uc - un)
    d1 = cr.delta(p, un, uc, 0.1)
    d2 = cr.delta(p, un2, uc, 0.1)
    assert np.allclose(d2, 3.0 * d1, rtol=1e-12, atol=1e-15)
