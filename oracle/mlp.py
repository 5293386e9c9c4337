"""FP64 reference of the learned beam -- TEST INFRASTRUCTURE ONLY.

Only the test suite, the package smoke check and the benchmark's CPU-baseline
leg may import this module; the product path never does.

The learned beam is not part of the paper: it stands in for the beam step of
Alg. 2 (Sec. 3.4 gives the beam's role, a complex 2 x 2 Jones matrix per
direction and channel).  The network, as the library documents it:

    x   = (u, v, w) = (az / 2 pi, za / (pi / 2), (nu - nu_min) / (nu_max - nu_min))
    phi = (sin 2 pi B (u, v), cos 2 pi B (u, v))        B [128][2], fixed
    h1  = SiLU(W1 phi + b1); h_{l+1} = SiLU(W_{l+1} h_l + b_{l+1}), l = 1..3
    g   = W5 h4 + b5                                     [64] = 8 outputs x 8 coefficients
    out_o = sum_k T_k(2 w - 1) g[8 o + k],  o = 0..7     (re, im) of J[0][0], J[0][1], J[1][0], J[1][1]

with T_k the Chebyshev polynomials of the first kind (T_0 = 1, T_1 = t,
T_{k+1} = 2 t T_k - T_{k-1}): the direction enters through the features and
the frequency only through a degree-7 polynomial per output.  SiLU(z) =
z / (1 + e^-z); the loss L = mean over rows and the 8 outputs of
(out - y)^2.  The parameter vector stores B, W1, b1, ..., W5, b5 in that
order, weights row-major [out][in].

``forward`` is the definition in float64; with ``bf16=True`` the operands of
the four hidden-layer products (features, activations, W1..W4) are first
rounded to bfloat16 (round to nearest, ties to even), which is what the
library's MFMA products compute before accumulating.  ``loss_grad`` is
reverse-mode differentiation of the float64 definition, written out layer by
layer.
"""
from __future__ import annotations

import math

import numpy as np

N_FREQ, N_FEAT, N_HID, N_OUT, N_BASIS = 128, 256, 128, 8, 8
N_NET = N_OUT * N_BASIS  # network outputs: the basis coefficients of every output
_SHAPES = (("B", (N_FREQ, 2)), ("W1", (N_HID, N_FEAT)), ("b1", (N_HID,)), ("W2", (N_HID, N_HID)), ("b2", (N_HID,)),
           ("W3", (N_HID, N_HID)), ("b3", (N_HID,)), ("W4", (N_HID, N_HID)), ("b4", (N_HID,)), ("W5", (N_NET, N_HID)),
           ("b5", (N_NET,)))
N_PARAMS = sum(int(np.prod(s)) for _, s in _SHAPES)


def unpack(p) -> dict:
    """Views of the named parameters inside the flat vector p (float64 copy)."""
    p = np.asarray(p, dtype=np.float64)
    if p.shape != (N_PARAMS,):
        raise ValueError(f"expected {N_PARAMS} parameters, got {p.shape}")
    out, o = {}, 0
    for name, shape in _SHAPES:
        k = int(np.prod(shape))
        out[name] = p[o:o + k].reshape(shape)
        o += k
    return out


def pack(d: dict) -> np.ndarray:
    """Inverse of unpack."""
    return np.concatenate([np.asarray(d[name], dtype=np.float64).ravel() for name, _ in _SHAPES])


def round_bf16(a) -> np.ndarray:
    """Round to the nearest bfloat16 (ties to even), returned as float64.

    bfloat16 keeps the sign, the 8 exponent bits and the top 7 mantissa bits
    of an IEEE float32; the value is first rounded to float32, then the low 16
    bits are rounded off.
    """
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    u = ((u + 0x7FFF + lsb) & 0xFFFF0000).astype(np.uint32)
    return u.view(np.float32).astype(np.float64)


def normalise(za, az, nu, nu_min: float, nu_max: float) -> np.ndarray:
    """Network inputs x [n][3] from (za, az) in radians and nu in Hz."""
    za, az, nu = (np.asarray(v, dtype=np.float64) for v in (za, az, nu))
    za, az, nu = np.broadcast_arrays(za, az, nu)
    return np.stack([az / (2.0 * math.pi), za / (0.5 * math.pi), (nu - nu_min) / (nu_max - nu_min)], axis=-1)


def _silu(z):
    return z / (1.0 + np.exp(-z))


def features(P: dict, x) -> np.ndarray:
    """phi [n][256]: sines then cosines of 2 pi B (u, v)."""
    arg = 2.0 * math.pi * (np.asarray(x, dtype=np.float64)[:, :2] @ P["B"].T)
    return np.concatenate([np.sin(arg), np.cos(arg)], axis=1)


def chebyshev(x) -> np.ndarray:
    """T [n][N_BASIS]: T_k(2 w - 1) of the frequency input w = x[:, 2], by the three-term recurrence."""
    t = 2.0 * np.asarray(x, dtype=np.float64)[:, 2] - 1.0
    T = np.empty((t.shape[0], N_BASIS))
    T[:, 0] = 1.0
    T[:, 1] = t
    for k in range(2, N_BASIS):
        T[:, k] = 2.0 * t * T[:, k - 1] - T[:, k - 2]
    return T


def combine(g, x) -> np.ndarray:
    """out [n][8]: out_o = sum_k T_k(2 w - 1) g[8 o + k]."""
    g = np.asarray(g, dtype=np.float64).reshape(-1, N_OUT, N_BASIS)
    return np.einsum("nok,nk->no", g, chebyshev(x))


def forward(p, x, bf16: bool = False, keep: bool = False):
    """Network outputs [n][8] (and, with keep, the coefficients g, the pre-activations and activations)."""
    P = unpack(p)
    r = round_bf16 if bf16 else (lambda a: a)
    h = features(P, x)
    zs, hs = [], [h]
    for l in range(1, 5):
        z = r(h) @ r(P[f"W{l}"]).T + P[f"b{l}"]
        h = _silu(z)
        zs.append(z)
        hs.append(h)
    g = h @ P["W5"].T + P["b5"]
    out = combine(g, x)
    return (out, g, zs, hs) if keep else out


def loss(p, x, y, bf16: bool = False) -> float:
    d = forward(p, x, bf16) - np.asarray(y, dtype=np.float64)
    return float(np.mean(d * d))


def loss_grad(p, x, y):
    """(gradient [N_PARAMS], loss) of the float64 network; B gets a zero gradient (it is not trained)."""
    P = unpack(p)
    y = np.asarray(y, dtype=np.float64)
    out, _, zs, hs = forward(p, x, keep=True)
    n = out.shape[0]
    d = out - y
    L = float(np.mean(d * d))
    g = {"B": np.zeros_like(P["B"])}
    dout = 2.0 * d / (N_OUT * n)            # dL/dout
    dg = (dout[:, :, None] * chebyshev(x)[:, None, :]).reshape(n, N_NET)  # dL/dg[8 o + k] = T_k dL/dout_o
    g["W5"] = dg.T @ hs[4]
    g["b5"] = dg.sum(axis=0)
    dh = dg @ P["W5"]                       # dL/dh4
    for l in range(4, 0, -1):
        z = zs[l - 1]
        s = 1.0 / (1.0 + np.exp(-z))
        dz = dh * s * (1.0 + z * (1.0 - s))  # SiLU'(z) = s + z s (1 - s)
        g[f"W{l}"] = dz.T @ hs[l - 1]
        g[f"b{l}"] = dz.sum(axis=0)
        dh = dz @ P[f"W{l}"]
    return pack(g), L


def adam_step(p, g, m1, m2, step: int, lr: float, b1: float = 0.9, b2: float = 0.999, eps: float = 1e-8):
    """One Adam update (Kingma and Ba, 2015, Algorithm 1) of every trained parameter.

    m1 and m2 (first and second moments) are updated in place; returns the new
    parameter vector.  The Fourier matrix B (the first 256 entries) is fixed.
    """
    p = np.array(p, dtype=np.float64)
    g = np.asarray(g, dtype=np.float64)
    t = slice(N_FREQ * 2, None)
    m1[t] = b1 * m1[t] + (1.0 - b1) * g[t]
    m2[t] = b2 * m2[t] + (1.0 - b2) * g[t] * g[t]
    mh = m1[t] / (1.0 - b1 ** step)
    vh = m2[t] / (1.0 - b2 ** step)
    p[t] -= lr * mh / (np.sqrt(vh) + eps)
    return p
