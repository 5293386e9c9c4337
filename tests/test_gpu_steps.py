"""Each hot-path kernel on its own, through the C ABI step entry points,
against the FP64 oracle on the same seeded inputs."""
import math

import numpy as np
import pytest

from paper_2312_09763_amd import matvis as mv
from paper_2312_09763_amd import synth

from helpers import say

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


# ---------------------------------------------------------------- step (i)
@pytest.mark.parametrize("n_src", [1, 255, 4999, 70001])
def test_sky_rotation_and_compaction(orc, n_src):
    torch = _torch()
    wl = synth.workload(2, n_src=n_src, n_time=5, n_freq=1)
    say(f"sky n_src={n_src}")
    cfg = mv.config_for(wl, "fp64", src_chunk=max(1, n_src // 3))
    with mv.Context(cfg) as ctx:
        d = mv.device_inputs(wl, "fp64")
        idx, count, s_hat, za_az = ctx.step_sky(d["lsts"], d["src_radec"])
        torch.cuda.synchronize()
        idx, count, s_hat, za_az = (x.cpu().numpy() for x in (idx, count, s_hat, za_az))
    xeq = orc.xeq(wl.ra, wl.dec)
    for t in range(wl.n_time):
        xh = orc.topocentric(orc.rotation(wl.lsts[t], wl.latitude), xeq)
        want = orc.visible(xh)
        m = int(count[t])
        got = idx[t, :m]
        if not np.array_equal(got, want):
            # only sources on the horizon to rounding may differ (strict U > 0 cut)
            diff = np.setxor1d(got, want)
            assert np.all(np.abs(xh[diff, 2]) < 1e-12), diff
            continue
        # FMA contraction and the device sincos may differ from the host by an ulp or two
        np.testing.assert_allclose(s_hat[t, :, :m].T, xh[want], rtol=0, atol=1e-15)
        az, za = orc.azza(xh[want])
        np.testing.assert_allclose(za_az[t, 0, :m], za, rtol=0, atol=4e-15)
        # azimuth is ill-conditioned near the zenith: compare the arc length it spans
        daz = np.angle(np.exp(1j * (za_az[t, 1, :m] - az)))
        assert (np.abs(daz) * np.hypot(xh[want, 0], xh[want, 1])).max(initial=0.0) < 4e-15
        assert np.all((za_az[t, 1, :m] >= 0) & (za_az[t, 1, :m] < 2 * math.pi))


# ---------------------------------------------------------------- step (ii)
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("mode", ["bilinear", "bicubic"])
def test_beam_interpolation(orc, precision, mode):
    torch = _torch()
    say(f"interp {precision} {mode}")
    wl = synth.workload(2, n_src=10, n_time=1, n_freq=1)
    grid = wl.beam[:, 0]  # [n_beam][p][k][za][az]
    if precision != "fp64":
        grid = grid.astype(np.complex64)
    rng = np.random.default_rng(11)
    n = 20011
    za = rng.uniform(0, math.pi / 2, n)
    az = rng.uniform(0, 2 * math.pi, n)
    # grid nodes, the zenith, the horizon cell and both sides of the az seam
    za[:6] = [0.0, 0.0, wl.dza * 3, math.pi / 2 - 1e-9, wl.dza * 0.5, math.pi / 2 - wl.dza * 0.3]
    az[:6] = [0.0, 2 * math.pi - 1e-12, wl.daz * 7, 1.0, 2 * math.pi - wl.daz * 0.25, wl.daz * 0.1]
    cfg = mv.config_for(wl, precision, beam_mode=mode)
    with mv.Context(cfg) as ctx:
        gd = torch.from_numpy(np.ascontiguousarray(grid)).cuda()
        zaz = torch.from_numpy(np.stack([za, az])).cuda()
        A = ctx.step_interp(zaz, gd).cpu().numpy().astype(np.complex128)
    scale = np.abs(grid).max()
    tol = 1e-13 if precision == "fp64" else 2e-6
    for p in range(2):
        for k in range(2):
            want = orc.interp(mode, grid[0, p, k].astype(np.complex128), wl.dza, wl.daz, za, az)
            err = np.abs(A[0, p, k] - want).max() / scale
            assert err < tol, (p, k, err)


# ---------------------------------------------------------------- step (v)
@pytest.mark.parametrize("precision,tol", [("fp64", 1e-13), ("fp32", 4e-6), ("bf16x3", 1e-5)])
@pytest.mark.parametrize("n_row,n_col", [(37, 1000), (130, 4113), (256, 10000), (300, 777)])
def test_herk_against_definition(orc, precision, tol, n_row, n_col):
    torch = _torch()
    say(f"herk {precision} {n_row}x{n_col}")
    rng = np.random.default_rng(n_row * 7 + n_col)
    Z = (rng.normal(size=(n_row, n_col)) + 1j * rng.normal(size=(n_row, n_col))) * rng.uniform(0.1, 3, (n_row, 1))
    if precision != "fp64":
        Z = Z.astype(np.complex64)
    cfg = mv.Config(n_ant=n_row, n_feed=1, n_ax=1, max_src=n_col, precision=precision)
    with mv.Context(cfg) as ctx:
        V = ctx.step_herk(torch.from_numpy(Z).cuda()).cpu().numpy()
    ref = orc.gram(Z.astype(np.complex128))
    d = np.sqrt(np.abs(np.diag(ref)))
    err = (np.abs(V.astype(np.complex128) - ref) / np.outer(d, d)).max()
    say(f"  err_cs={err:.3e}")
    assert err < tol
    # exactly Hermitian with a real diagonal
    np.testing.assert_array_equal(V, V.conj().T)
    assert np.all(np.diag(V).imag == 0)


@pytest.mark.parametrize("precision", ["fp64", "fp32", "bf16x3"])
def test_herk_rank_one_and_orthogonal_rows(precision):
    torch = _torch()
    n_col = 4096 * 3 + 5
    z = np.exp(2j * math.pi * np.arange(n_col) / 17.0)
    Z = np.outer([1.0, 2.0, -0.5j, 0.25 + 0.25j], z)
    if precision != "fp64":
        Z = Z.astype(np.complex64)
    cfg = mv.Config(n_ant=4, max_src=n_col, precision=precision)
    with mv.Context(cfg) as ctx:
        V = ctx.step_herk(torch.from_numpy(Z).cuda()).cpu().numpy().astype(np.complex128)
        a = np.array([1.0, 2.0, -0.5j, 0.25 + 0.25j])
        want = np.outer(a, a.conj()) * n_col
        tol = 1e-12 if precision == "fp64" else 1e-5
        assert np.abs(V - want).max() / np.abs(want).max() < tol
        # orthogonal rows (distinct Fourier modes over a full period) give a diagonal V
        n = 64 * 50
        k = np.arange(n)
        F = np.stack([np.exp(2j * math.pi * f * k / n) for f in (0, 1, 5, 9)])
        if precision != "fp64":
            F = F.astype(np.complex64)
        W = ctx.step_herk(torch.from_numpy(F).cuda()).cpu().numpy().astype(np.complex128)
        off = W - np.diag(np.diag(W))
        assert np.abs(off).max() < (1e-9 if precision == "fp64" else 2e-3 if precision == "fp32" else 2e-2)
        np.testing.assert_allclose(np.diag(W).real, n, rtol=1e-5)
