"""Pins of the learned-beam reference (oracle/mlp.py) on the CPU.

The learned beam is not in the paper, so the pins are mathematical: central
finite differences and an independent reverse-mode engine (torch autograd in
float64) for the gradient, closed forms for degenerate networks, the
frequency head against numpy's Chebyshev series and hand values, periodicity
in azimuth, and bfloat16 rounding against torch's own conversion and hand
values.
"""
import math

import numpy as np
import pytest
import torch

from oracle import mlp as om
from paper_2312_09763_amd import synth


def _params(seed=0, scale=1.0):
    p = synth.surrogate_init(seed).astype(np.float64)
    P = om.unpack(p)
    d = {k: v.copy() for k, v in P.items()}
    for k in d:
        if k != "B":
            d[k] = d[k] * scale
    return om.pack(d)


def _data(n, seed=1):
    rng = np.random.Generator(np.random.PCG64(seed))
    x = np.stack([rng.random(n), rng.random(n), rng.random(n)], axis=1)
    y = rng.normal(0.0, 0.5, (n, 8))
    return x, y


def test_layout_size_matches_documented_count():
    assert om.N_PARAMS == 90944
    assert synth.SURROGATE_N_PARAMS == om.N_PARAMS


def test_gradient_matches_central_differences():
    p = _params(0, scale=2.0)
    x, y = _data(16)
    g, L = om.loss_grad(p, x, y)
    assert L == pytest.approx(om.loss(p, x, y), rel=1e-14)
    rng = np.random.Generator(np.random.PCG64(5))
    # a sample of parameters from every trained block (skip the fixed B)
    idx = rng.choice(np.arange(256, om.N_PARAMS), 60, replace=False)
    idx = np.concatenate([idx, [256, 256 + 128 * 256, om.N_PARAMS - 1, om.N_PARAMS - 9, om.N_PARAMS - 64 - 1]])
    for i in idx:
        h = 1e-5 * max(1.0, abs(p[i]))
        pp, pm = p.copy(), p.copy()
        pp[i] += h
        pm[i] -= h
        fd = (om.loss(pp, x, y) - om.loss(pm, x, y)) / (2 * h)
        assert g[i] == pytest.approx(fd, rel=1e-6, abs=1e-10), i


def test_gradient_matches_torch_autograd():
    p = _params(3, scale=1.5)
    x, y = _data(32, seed=4)
    g, L = om.loss_grad(p, x, y)
    P = om.unpack(p)
    T = {k: torch.tensor(v, dtype=torch.float64, requires_grad=(k != "B")) for k, v in P.items()}
    xt = torch.tensor(x)
    arg = 2 * math.pi * xt[:, :2] @ T["B"].T
    h = torch.cat([torch.sin(arg), torch.cos(arg)], dim=1)
    for l in range(1, 5):
        h = torch.nn.functional.silu(torch.nn.functional.linear(h, T[f"W{l}"], T[f"b{l}"]))
    coef = torch.nn.functional.linear(h, T["W5"], T["b5"]).reshape(-1, 8, 8)
    # Chebyshev basis from the trigonometric definition T_k(cos th) = cos(k th)
    th = torch.arccos(2 * xt[:, 2] - 1)
    basis = torch.cos(torch.arange(8, dtype=torch.float64)[None, :] * th[:, None])
    out = (coef * basis[:, None, :]).sum(dim=2)
    lt = torch.nn.functional.mse_loss(out, torch.tensor(y))
    lt.backward()
    assert L == pytest.approx(lt.item(), rel=1e-13)
    G = om.unpack(g)
    for k, v in T.items():
        if k == "B":
            assert np.all(G["B"] == 0)
            continue
        np.testing.assert_allclose(G[k], v.grad.numpy(), rtol=1e-10, atol=1e-14)


def test_zero_hidden_weights_closed_form():
    # all weights zero: h_l = SiLU(b_l) whatever the input, g = W5 SiLU(b4) + b5,
    # and each output a Chebyshev series in 2 w - 1 with coefficients g[8 o .. 8 o + 7]
    P = {k: v.copy() for k, v in om.unpack(_params(1)).items()}
    for l in range(1, 5):
        P[f"W{l}"][:] = 0.0
    p = om.pack(P)
    x, _ = _data(7)
    b4 = P["b4"]
    g = P["W5"] @ (b4 / (1 + np.exp(-b4))) + P["b5"]
    expect = np.stack([np.polynomial.chebyshev.chebval(2 * x[:, 2] - 1, g[8 * o:8 * o + 8]) for o in range(8)],
                      axis=1)
    np.testing.assert_allclose(om.forward(p, x), expect, rtol=1e-13, atol=1e-14)


def test_single_path_network():
    # one feature -> one unit per layer -> one output through the constant
    # basis term (T_0 = 1): out = silu^4 applied to sin(2 pi (u + 0.3 v))
    P = {k: np.zeros_like(v) for k, v in om.unpack(_params(0)).items()}
    P["B"][0] = [1.0, 0.3]
    P["W1"][5, 0] = 1.0
    for l in (2, 3, 4):
        P[f"W{l}"][5, 5] = 1.0
    P["W5"][8 * 2, 5] = 1.0
    x, _ = _data(9)
    t = np.sin(2 * math.pi * (x[:, 0] + 0.3 * x[:, 1]))
    for _ in range(4):
        t = t / (1 + np.exp(-t))
    out = om.forward(om.pack(P), x)
    np.testing.assert_allclose(out[:, 2], t, rtol=1e-14, atol=1e-15)
    assert np.all(out[:, [0, 1, 3, 4, 5, 6, 7]] == 0)


def test_frequency_head_hand_values():
    # g = b5 alone (all weights zero, h4 = SiLU(0) = 0): output o is the series
    # sum_k b5[8 o + k] T_k(t), t = 2 w - 1; hand values at w = 0, 1/2, 3/4, 1
    # (t = -1, 0, 1/2, 1) for T_2 = 2 t^2 - 1, T_3 = 4 t^3 - 3 t and T_7
    P = {k: np.zeros_like(v) for k, v in om.unpack(_params(0)).items()}
    P["b5"][8 * 0 + 2] = 1.0   # output 0: T_2
    P["b5"][8 * 5 + 3] = -2.0  # output 5: -2 T_3
    P["b5"][8 * 7 + 7] = 0.5   # output 7: T_7 / 2
    x = np.array([[0.3, 0.4, 0.0], [0.1, 0.9, 0.5], [0.7, 0.2, 0.75], [0.5, 0.5, 1.0]])
    out = om.forward(om.pack(P), x)
    np.testing.assert_allclose(out[:, 0], [1.0, -1.0, -0.5, 1.0], atol=1e-15)
    np.testing.assert_allclose(out[:, 5], [2.0, 0.0, 2.0, -2.0], atol=1e-15)
    # T_7(cos th) = cos 7 th: t = 1/2 (th = pi / 3) gives cos(7 pi / 3) = 1/2
    np.testing.assert_allclose(out[:, 7], [-0.5, 0.0, 0.25, 0.5], atol=1e-14)
    assert np.all(out[:, [1, 2, 3, 4, 6]] == 0)


def test_periodic_in_azimuth():
    p = _params(2)
    x, _ = _data(20)
    x2 = x.copy()
    x2[:, 0] += 1.0  # az + 2 pi
    np.testing.assert_allclose(om.forward(p, x2), om.forward(p, x), rtol=0, atol=1e-11)


def test_normalise():
    x = om.normalise([0.0, math.pi / 2], [math.pi, 0.0], [100e6, 200e6], 100e6, 200e6)
    np.testing.assert_allclose(x, [[0.5, 0.0, 0.0], [0.0, 1.0, 1.0]], atol=1e-15)


def test_round_bf16_values():
    e = 2.0 ** -8
    vals = np.array([1.0, 1 + e, 1 + 3 * e, 1 + 1.01 * e, -2.5, 3.0e-3, 65504.0])
    exp = np.array([1.0, 1.0, 1 + 4 * e, 1 + 2 * e, -2.5, None, 65536.0], dtype=object)
    got = om.round_bf16(vals)
    for g, v, x in zip(got, vals, exp):
        if x is not None:
            assert g == x, v
    ref = torch.tensor(vals, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(got, ref)
    r = np.random.Generator(np.random.PCG64(9)).normal(0, 10, 10000)
    ref = torch.tensor(r, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(om.round_bf16(r), ref)


def test_bf16_forward_close_to_exact():
    # rounding the product operands is a small perturbation of the exact network
    p = _params(0)
    x, _ = _data(64)
    a, b = om.forward(p, x), om.forward(p, x, bf16=True)
    assert np.linalg.norm(a - b) / np.linalg.norm(a) < 2e-2
    assert not np.array_equal(a, b)


def test_adam_first_step_is_signed_learning_rate():
    # after one step from zero moments, m_hat = g and v_hat = g^2, so each trained
    # parameter moves by lr * g / (|g| + eps) ~ lr * sign(g); B does not move
    rng = np.random.Generator(np.random.PCG64(2))
    p = rng.normal(size=om.N_PARAMS)
    g = rng.normal(size=om.N_PARAMS)
    g[1000] = 0.0
    m1, m2 = np.zeros(om.N_PARAMS), np.zeros(om.N_PARAMS)
    q = om.adam_step(p, g, m1, m2, 1, 1e-2)
    np.testing.assert_array_equal(q[:256], p[:256])
    d = (p - q)[256:]
    gs = g[256:]
    np.testing.assert_allclose(d, 1e-2 * gs / (np.abs(gs) + 1e-8), rtol=1e-12, atol=1e-18)
    assert d[1000 - 256] == 0.0
    # a constant gradient keeps the step at lr (bias correction exact)
    for t in range(2, 6):
        q2 = om.adam_step(q, g, m1, m2, t, 1e-2)
        np.testing.assert_allclose((q - q2)[256:], 1e-2 * gs / (np.abs(gs) + 1e-8), rtol=1e-9, atol=1e-15)
        q = q2
