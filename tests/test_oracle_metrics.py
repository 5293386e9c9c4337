"""Pins of the error metrics every parity assertion goes through (oracle/metrics.py).

The expected numbers are worked out by hand below, not by re-running the
formula: a one-instance, two-antenna, two-feed reference with unequal
autocorrelations per antenna and feed, a dominant off-diagonal error, an error
on a zero reference entry and a complex error, then a second instance at a
different scale so that a norm or maximum pooled across instances shows.
"""
import math

import numpy as np
import pytest

from oracle import metrics


def _ref_one():
    """V_ref[a][b][p][q] of the hand example (entries listed in the comments)."""
    R = np.zeros((2, 2, 2, 2), dtype=np.complex128)
    R[0, 0] = [[4, 1 + 1j], [1 - 1j, 9]]     # |.|^2: 16 + 2 + 2 + 81 = 101
    R[1, 1] = [[16, 2j], [-2j, 1]]           # 256 + 4 + 4 + 1 = 265
    R[0, 1] = [[2, 3j], [1, 0]]              # 4 + 9 + 1 + 0 = 14  (a zero entry at p = q = 1)
    R[1, 0] = [[2, 1], [-3j, 0]]             # 4 + 1 + 9 + 0 = 14
    return R                                 # ||R||_F^2 = 394


def _err_one():
    """The error D = V - V_ref of the hand example."""
    D = np.zeros((2, 2, 2, 2), dtype=np.complex128)
    D[0, 1, 1, 0] = 0.48        # scale sqrt(|R[0,0,1,1]| |R[1,1,0,0]|) = sqrt(9 * 16) = 12 -> 0.04
    D[1, 0, 0, 1] = 0.03 + 0.04j  # |.| = 0.05, scale sqrt(16 * 9) = 12 -> 0.0041667
    D[0, 0, 0, 0] = 0.12        # scale sqrt(4 * 4) = 4 -> 0.03
    D[0, 1, 1, 1] = 0.06        # on the zero reference entry: scale sqrt(9 * 1) = 3 -> 0.02
    return D                    # ||D||_F^2 = 0.2304 + 0.0025 + 0.0144 + 0.0036 = 0.2509


def test_err_cs_hand_example():
    R, D = _ref_one(), _err_one()
    got = metrics.err_cs((R + D)[None], R[None])
    assert got.shape == (1,)
    assert got[0] == pytest.approx(0.04, rel=1e-12)
    # a metric that paired the feeds the other way round (|R[a,a,q,q]| |R[b,b,p,p]|)
    # would give 0.48 / sqrt(4 * 1) = 0.24 for the dominant entry
    assert abs(got[0] - 0.24) > 0.1


def test_err_f_hand_example():
    R, D = _ref_one(), _err_one()
    got = metrics.err_f((R + D)[None], R[None])
    assert got[0] == pytest.approx(math.sqrt(0.2509 / 394.0), rel=1e-12)


def test_metrics_are_per_instance():
    R, D = _ref_one(), _err_one()
    R2 = 100.0 * R
    D2 = np.zeros_like(D)
    D2[0, 0, 1, 1] = 1.0        # scale sqrt(900 * 900) = 900
    V = np.stack([R + D, R2 + D2])
    Vref = np.stack([R, R2])
    cs = metrics.err_cs(V, Vref)
    f = metrics.err_f(V, Vref)
    assert cs[0] == pytest.approx(0.04, rel=1e-12)
    assert cs[1] == pytest.approx(1.0 / 900.0, rel=1e-12)
    assert f[0] == pytest.approx(math.sqrt(0.2509 / 394.0), rel=1e-12)
    assert f[1] == pytest.approx(1.0 / (100.0 * math.sqrt(394.0)), rel=1e-12)
    # pooled over both instances the Frobenius ratio would be sqrt(1.2509 / (394 + 3 940 000))
    assert abs(f.max() - math.sqrt(1.2509 / 3940394.0)) > 1e-3


def test_exact_result_scores_zero_and_is_scale_free():
    R = _ref_one()
    assert metrics.err_cs(R[None], R[None])[0] == 0.0
    assert metrics.err_f(R[None], R[None])[0] == 0.0
    D = _err_one()
    for s in (1e-6, 1e6):  # both metrics are relative
        assert metrics.err_cs((s * (R + D))[None], (s * R)[None])[0] == pytest.approx(0.04, rel=1e-12)


def test_pair_forms_hand_example():
    R, D = _ref_one(), _err_one()
    V = R + D
    # listed pairs: (0, 1) with its two autocorrelations; (1, 0) is not listed
    pairs = [(0, 0), (0, 1), (1, 1)]
    Vp = np.stack([V[a, b] for a, b in pairs])[None]
    Rp = np.stack([R[a, b] for a, b in pairs])[None]
    assert metrics.err_cs_pairs(Vp, Rp, pairs)[0] == pytest.approx(0.04, rel=1e-12)
    # listed entries only: ||D||^2 without the (1, 0) entry, over 101 + 14 + 265
    assert metrics.err_f_pairs(Vp, Rp)[0] == pytest.approx(math.sqrt((0.2509 - 0.0025) / 380.0), rel=1e-12)
    # all four pairs listed: the pair forms agree with the full ones
    allp = [(0, 0), (0, 1), (1, 0), (1, 1)]
    Vp = np.stack([V[a, b] for a, b in allp])[None]
    Rp = np.stack([R[a, b] for a, b in allp])[None]
    assert metrics.err_cs_pairs(Vp, Rp, allp)[0] == pytest.approx(metrics.err_cs(V[None], R[None])[0], rel=1e-14)
    assert metrics.err_f_pairs(Vp, Rp)[0] == pytest.approx(metrics.err_f(V[None], R[None])[0], rel=1e-14)


def test_pair_forms_need_the_autocorrelations():
    R = _ref_one()
    pairs = [(0, 0), (0, 1)]  # (1, 1) missing
    Rp = np.stack([R[a, b] for a, b in pairs])[None]
    with pytest.raises(ValueError):
        metrics.err_cs_pairs(Rp, Rp, pairs)
