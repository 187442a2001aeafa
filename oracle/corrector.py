"""Learned corrector network in plain FP64 NumPy: test infrastructure only.

The corrector is not part of the paper; it is an addition on top of the EIFE2
step (eq. (2.14)): one coarse step u_c from u_n, then a small convolutional
network predicts the residual delta towards the result of several fine steps,
u_{n+1} = u_c + delta.  This module is the slow, obviously correct reference
of that network, its MSE loss, its gradients and the Adam update, against which
the HIP kernels are checked.

Network: six 3x3 convolutions over the interior nodes of a 2D grid, channels
2 -> 32 -> 32 -> 32 -> 32 -> 32 -> 1, ReLU after the first five, zero padding
(the padded ring is the homogeneous Dirichlet boundary).  Per image, with the
RMS coarse change c = sqrt(mean((u_c - u_n)^2)) + 1e-30, the input channels
are (u_c, (u_c - u_n) / c) and the output o is scaled, delta = s_out c o: the
network sees the change at unit scale and answers relative to it.

Arrays are [B][ny][nx][C] (x fastest, channels innermost).  Tap t = 3 (dy + 1)
+ (dx + 1) reads the input at (y + dy, x + dx).  Parameter vector (float):
  W1 [9][2][32] (tap, input channel, output channel), b1 [32],
  then four times W [9][32][32] (tap, output channel, input channel), b [32],
  then W6 [9][32] (tap, input channel), b6 [1].
"""
import numpy as np

C = 32
TAPS = [(dy, dx) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]
N_MID = 4
SIZES = [9 * 2 * C, C] + [9 * C * C, C] * N_MID + [9 * C, 1]
N_PARAMS = int(sum(SIZES))


def unpack(p):
    """Split the flat parameter vector into [(W, b), ...] for the six layers."""
    p = np.asarray(p, dtype=np.float64)
    assert p.shape == (N_PARAMS,)
    out, o = [], 0
    shapes = [((9, 2, C), (C,))] + [((9, C, C), (C,))] * N_MID + [((9, C), (1,))]
    for ws, bs in shapes:
        nw, nb = int(np.prod(ws)), int(np.prod(bs))
        out.append((p[o:o + nw].reshape(ws), p[o + nw:o + nw + nb].reshape(bs)))
        o += nw + nb
    return out


def pack(layers):
    return np.concatenate([np.concatenate([W.reshape(-1), b.reshape(-1)]) for W, b in layers])


def shift(a, dy, dx):
    """s[:, y, x] = a[:, y + dy, x + dx], zero where that lies outside the grid."""
    B, ny, nx = a.shape[:3]
    s = np.zeros_like(a)
    ys, yd = (slice(dy, ny), slice(0, ny - dy)) if dy >= 0 else (slice(0, ny + dy), slice(-dy, ny))
    xs, xd = (slice(dx, nx), slice(0, nx - dx)) if dx >= 0 else (slice(0, nx + dx), slice(-dx, nx))
    s[:, yd, xd] = a[:, ys, xs]
    return s


def init_params(seed):
    """He-normal weights (fan-in 9 * C_in), zero biases, a small last layer."""
    rng = np.random.default_rng(seed)
    layers = [(rng.normal(0, np.sqrt(2.0 / 18), (9, 2, C)), np.zeros(C))]
    for _ in range(N_MID):
        layers.append((rng.normal(0, np.sqrt(2.0 / (9 * C)), (9, C, C)), np.zeros(C)))
    layers.append((rng.normal(0, 0.1 * np.sqrt(1.0 / (9 * C)), (9, C)), np.zeros(1)))
    return pack(layers)


def change_scale(un, uc):
    """Per image: c = sqrt(mean over nodes of (u_c - u_n)^2) + 1e-30, shape [B]."""
    d = np.asarray(uc, np.float64) - np.asarray(un, np.float64)
    return np.sqrt(np.mean(d * d, axis=(1, 2))) + 1e-30


def features(un, uc):
    """Input channels [B][ny][nx][2]: (u_c, (u_c - u_n) / c)."""
    un, uc = np.asarray(un, np.float64), np.asarray(uc, np.float64)
    c = change_scale(un, uc)
    return np.stack([uc, (uc - un) / c[:, None, None]], axis=-1)


def forward(p, un, uc):
    """Network output o [B][ny][nx] and the activations [X0, Y1, ..., Y5]."""
    L = unpack(p)
    X0 = features(un, uc)
    acts = [X0]
    W1, b1 = L[0]
    Z = b1 + sum(shift(X0, dy, dx) @ W1[t] for t, (dy, dx) in enumerate(TAPS))
    Y = np.maximum(Z, 0.0)
    acts.append(Y)
    for W, b in L[1:1 + N_MID]:
        Z = b + sum(shift(Y, dy, dx) @ W[t].T for t, (dy, dx) in enumerate(TAPS))
        Y = np.maximum(Z, 0.0)
        acts.append(Y)
    W6, b6 = L[-1]
    o = b6[0] + sum(shift(Y, dy, dx) @ W6[t] for t, (dy, dx) in enumerate(TAPS))
    return o, acts


def delta(p, un, uc, s_out):
    """The predicted residual delta = s_out c o."""
    o, _ = forward(p, un, uc)
    return s_out * change_scale(un, uc)[:, None, None] * o


def loss_and_grad(p, un, uc, uf, s_out):
    """MSE of o against the scaled residual (uf - uc) / (s_out c), and its gradient in p."""
    o, acts = forward(p, un, uc)
    L = unpack(p)
    c = change_scale(un, uc)[:, None, None]
    target = (np.asarray(uf, np.float64) - np.asarray(uc, np.float64)) / (s_out * c)
    e = o - target
    loss = float(np.mean(e * e))
    g = 2.0 * e / e.size  # dloss/do
    grads = [None] * len(L)
    # output layer: o = b6 + sum_t shift(Y5, t) . W6[t]
    Y5 = acts[-1]
    W6 = L[-1][0]
    dW6 = np.stack([np.einsum("byx,byxc->c", g, shift(Y5, dy, dx)) for dy, dx in TAPS])
    grads[-1] = (dW6, np.array([g.sum()]))
    # gradient reaching Y5: the transpose of a shift is the opposite shift
    dY = sum(shift(g[..., None] * W6[t], -dy, -dx) for t, (dy, dx) in enumerate(TAPS))
    for li in range(N_MID, 0, -1):
        Yout, Yin = acts[li + 1], acts[li]
        W = L[li][0]
        dZ = dY * (Yout > 0)
        dW = np.stack([np.einsum("byxo,byxi->oi", dZ, shift(Yin, dy, dx)) for dy, dx in TAPS])
        grads[li] = (dW, dZ.sum(axis=(0, 1, 2)))
        dY = sum(shift(dZ @ W[t], -dy, -dx) for t, (dy, dx) in enumerate(TAPS))
    dZ1 = dY * (acts[1] > 0)
    X0 = acts[0]
    dW1 = np.stack([np.einsum("byxc,byxo->co", shift(X0, dy, dx), dZ1) for dy, dx in TAPS])
    grads[0] = (dW1, dZ1.sum(axis=(0, 1, 2)))
    return loss, pack(grads)


class Adam:
    """Adam with bias correction (beta1 = 0.9, beta2 = 0.999, eps = 1e-8)."""

    def __init__(self, n, b1=0.9, b2=0.999, eps=1e-8):
        self.m = np.zeros(n)
        self.v = np.zeros(n)
        self.t = 0
        self.b1, self.b2, self.eps = b1, b2, eps

    def step(self, p, g, lr):
        self.t += 1
        self.m = self.b1 * self.m + (1 - self.b1) * g
        self.v = self.b2 * self.v + (1 - self.b2) * g * g
        mh = self.m / (1 - self.b1 ** self.t)
        vh = self.v / (1 - self.b2 ** self.t)
        return p - lr * mh / (np.sqrt(vh) + self.eps)


def indicator(un, uc, delta):
    """Acceptance data of one corrected step: (r, max|u_c + delta|, c_rms) with
    r = ||delta||_2 / (||u_c - u_n||_2 + 1e-12) over the nodal values (a mesh
    weight would cancel in the ratio) and c_rms the RMS coarse change."""
    d = np.asarray(uc, np.float64) - np.asarray(un, np.float64)
    nd = np.sqrt(np.sum(np.asarray(delta, np.float64) ** 2))
    ns = np.sqrt(np.sum(d ** 2))
    return nd / (ns + 1e-12), float(np.max(np.abs(np.asarray(uc, np.float64) + delta))), \
        float(np.sqrt(np.mean(d ** 2)))
