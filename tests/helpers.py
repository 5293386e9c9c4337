"""Shared helpers for the GPU tests (run the HIP path, run the oracle)."""
from __future__ import annotations

import sys

import numpy as np

from oracle import metrics

TOL = {"fp64": 1e-10, "fp32": 1e-5, "bf16x3": 1e-3, "fp32-unfused": 1e-5, "bf16x3-unfused": 1e-3}
ALL_PATHS = ["fp64", "fp32", "bf16x3", "fp32-unfused", "bf16x3-unfused"]


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def gpu_simulate(wl, precision, **cfgkw):
    """Run matvis_simulate on the GPU for every (t, f) of a workload; V as [inst][a][b][p][q] c128.

    ``precision`` may carry a "-unfused" suffix: Z then goes through device
    memory in its own step instead of being formed inside the product."""
    import torch
    from paper_2312_09763_amd import matvis as mv
    if precision.endswith("-unfused"):
        precision = precision[:-len("-unfused")]
        cfgkw["unfused"] = True
    beam_idx = cfgkw.pop("beam_idx", None)
    cfg = mv.config_for(wl, precision, **cfgkw)
    d = mv.device_inputs(wl, precision)
    with mv.Context(cfg) as ctx:
        vis = ctx.simulate(**d, beam_idx=beam_idx)
        ctx.finish()
        torch.cuda.synchronize()
        V = vis.cpu().numpy().astype(np.complex128)
    return V.reshape((-1,) + V.shape[2:])


def oracle_vis(wl, instances=None, grid=None):
    import oracle
    g = wl.beam if grid is None else grid
    return oracle.simulate(wl.antpos, wl.freqs, wl.lsts, wl.ra, wl.dec, wl.flux, g, wl.latitude, wl.dza, wl.daz,
                           wl.interp, instances=instances)


def grid_as_used(wl, precision):
    """The beam grid values the device sees (complex64 unless FP64), upcast for the oracle."""
    if precision.startswith("fp64"):
        return wl.beam
    return wl.beam.astype(np.complex64).astype(np.complex128)


def errors(V, Vref):
    return float(metrics.err_f(V, Vref).max()), float(metrics.err_cs(V, Vref).max())


def sample_pairs(n_ant, n, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    a = rng.integers(0, n_ant, n)
    b = rng.integers(0, n_ant, n)
    pairs = sorted(set(zip(a.tolist(), b.tolist())))
    ants = sorted(set(a.tolist()) | set(b.tolist()))
    return pairs + [(x, x) for x in ants]


def sampled_err_cs(V, wl, prec, instances, pairs, grid=None):
    """err_CS and err_F over sampled entries (each the max over the instances): V is the
    full device result [t][f][a][b][p][q]; the oracle gives the listed pairs only."""
    import oracle
    ref = oracle.simulate_pairs(wl.antpos, wl.freqs, wl.lsts, wl.ra, wl.dec, wl.flux, grid_as_used(wl, prec) if grid is None else grid,
                                wl.latitude, wl.dza, wl.daz, wl.interp, instances=instances, pairs=pairs)
    pa = np.array([a for a, _ in pairs])
    pb = np.array([b for _, b in pairs])
    Vp = np.stack([V[t, f][pa, pb] for (t, f) in instances])  # [inst][pair][p][q]
    return float(metrics.err_cs_pairs(Vp, ref, pairs).max()), float(metrics.err_f_pairs(Vp, ref).max())
