"""Error metrics between a simulated visibility set and the FP64 reference.

Test infrastructure (imported by the tests and the benchmark's CPU-baseline
leg).  V arrays are [inst][a][b][p][q] complex.

* err_F  = ||V - V_ref||_F / ||V_ref||_F per instance;
* err_CS = max_{a,b,p,q} |V - V_ref| / sqrt(|V_ref[a,a,p,p]| |V_ref[b,b,q,q]|),
  the error scaled by the Cauchy-Schwarz bound of each entry, which is the
  natural size of the rounding in a sum of products and stays well defined
  where |V| itself is small.
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
