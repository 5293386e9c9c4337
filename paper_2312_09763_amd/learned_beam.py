"""The learned beam's training recipe, run on the GPU by the library's own kernels.

The network (include/matvis.h, "Learned beam") is fitted to the method's own
beam interpolant (Sec. 3.4): 2^20 points uniform by solid angle over the
visible hemisphere and uniform over the 16 channels (100-200 MHz) of the
polarised dipole beam on its 0.5 deg grid, targets from Keys bicubic
interpolation of that grid (matvis_beam_samples), then mini-batch Adam
(matvis_train_surrogate).  Everything is seeded, so the trained parameters are
reproducible; arithmetic runs in the library, this module only marshals.
"""
from __future__ import annotations

import numpy as np

from . import matvis as mv
from . import synth

NU0, NU1 = 100e6, 200e6  # the frequency range that normalises the network's third input


def training_beam():
    """The 16-channel polarised dipole beam the network learns (a workload-2 grid)."""
    return synth.workload(2, n_ant=4, n_src=10, n_time=1)


def samples(wl, grid, freqs, n: int, seed: int):
    """(targets [n][8], inputs [n][3]) device tensors from the bicubic interpolant."""
    import torch
    dev = lambda a, dt: torch.from_numpy(np.ascontiguousarray(a, dtype=dt)).cuda()
    rng = np.random.Generator(np.random.PCG64(seed))
    za, az = synth.hemisphere_points(rng, n)
    chan = rng.integers(0, wl.n_freq, n).astype(np.int32)
    return mv.beam_samples(grid, wl.dza, wl.daz, dev(za, np.float64), dev(az, np.float64), dev(chan, np.int32),
                           bicubic=True, chan_freq=freqs, nu_range=(NU0, NU1))


def train(epochs: int = 60, n_samples: int = 1 << 20, batch: int = 1024, seed: int = 1):
    """Train one network; returns (params [MLP_N_PARAMS] float32 device tensor,
    per-epoch mean loss list, training beam workload, its device grid)."""
    import torch
    wl = training_beam()
    grid = torch.from_numpy(np.ascontiguousarray(wl.beam[0], dtype=np.complex64)).cuda()
    freqs = torch.from_numpy(np.ascontiguousarray(wl.freqs, dtype=np.float64)).cuda()
    y, x = samples(wl, grid, freqs, n_samples, seed)
    P = torch.from_numpy(synth.surrogate_init(0, sigma_v=1.0, az_max=4)).cuda()
    hist = mv.train_surrogate(P, x, y, batch=batch, epochs=epochs, lr0=3e-3, lr1=3e-5, seed=seed)
    return P, hist, wl, grid
