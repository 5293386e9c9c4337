"""Error metrics between a simulated visibility set and the FP64 reference.

Test infrastructure (imported by the tests and the benchmark's CPU-baseline
leg).  Full V arrays are [inst][a][b][p][q] complex.

* err_F  = ||V - V_ref||_F / ||V_ref||_F per instance;
* err_CS = max_{a,b,p,q} |V - V_ref| / sqrt(|V_ref[a,a,p,p]| |V_ref[b,b,q,q]|),
  the error scaled by the Cauchy-Schwarz bound of each entry, which is the
  natural size of the rounding in a sum of products and stays well defined
  where |V| itself is small.

The paper defines no error metric on V itself (its validation compares delay
spectra); these two are the ones the parity tests state their tolerances in.
For problems too large for the full reference, the ``*_pairs`` forms take the
reference on a list of antenna pairs (which must include (a, a) and (b, b)
for every listed (a, b), so the Cauchy-Schwarz scale is known) and give the
same two numbers over the listed entries only, still per instance.
"""
from __future__ import annotations

import numpy as np


def err_f(V, Vref) -> np.ndarray:
    V = np.asarray(V, dtype=np.complex128)
    Vref = np.asarray(Vref, dtype=np.complex128)
    n = V.shape[0]
    d = (V - Vref).reshape(n, -1)
    r = Vref.reshape(n, -1)
    return np.linalg.norm(d, axis=1) / np.maximum(np.linalg.norm(r, axis=1), 1e-300)


def err_cs(V, Vref) -> np.ndarray:
    V = np.asarray(V, dtype=np.complex128)
    Vref = np.asarray(Vref, dtype=np.complex128)
    n, na, _, nf, _ = Vref.shape
    diag = np.abs(np.einsum("iaapp->iap", Vref))  # [inst][a][p]
    scale = np.sqrt(diag[:, :, None, :, None] * diag[:, None, :, None, :])
    out = np.abs(V - Vref) / np.maximum(scale, 1e-300)
    return out.reshape(n, -1).max(axis=1)


def _pair_index(pairs):
    idx = {}
    for k, (a, b) in enumerate(pairs):
        idx[(int(a), int(b))] = k
    for a, b in idx:
        if (a, a) not in idx or (b, b) not in idx:
            raise ValueError(f"pair ({a}, {b}) listed without both autocorrelations")
    return idx


def err_cs_pairs(Vp, Vref_p, pairs) -> np.ndarray:
    """err_CS over listed entries: Vp, Vref_p are [inst][pair][p][q], pairs [(a, b), ...]."""
    Vp = np.asarray(Vp, dtype=np.complex128)
    Vref_p = np.asarray(Vref_p, dtype=np.complex128)
    idx = _pair_index(pairs)
    out = np.zeros(Vref_p.shape[0])
    for (a, b), k in idx.items():
        da = np.abs(np.diagonal(Vref_p[:, idx[(a, a)]], axis1=1, axis2=2))  # [inst][p]
        db = np.abs(np.diagonal(Vref_p[:, idx[(b, b)]], axis1=1, axis2=2))  # [inst][q]
        scale = np.sqrt(da[:, :, None] * db[:, None, :])
        e = np.abs(Vp[:, k] - Vref_p[:, k]) / np.maximum(scale, 1e-300)
        out = np.maximum(out, e.reshape(e.shape[0], -1).max(axis=1))
    return out


def err_f_pairs(Vp, Vref_p) -> np.ndarray:
    """err_F over listed entries, per instance: Vp, Vref_p are [inst][pair][p][q]."""
    return err_f(Vp, Vref_p)
