"""The library's host-side redundancy code (App. A) against the oracle, exactly.

matvis_redundant_groups and matvis_submatrix_plan run on the host only, so
these run without a GPU: group ids, representatives, the alpha order, the
sub-matrix sizes and their densities must all be identical to the plain
references in oracle/submat.py.
"""
import numpy as np
import pytest

from oracle import submat
from paper_2312_09763_amd import matvis as mv
from paper_2312_09763_amd import synth


def _arrays():
    rng = np.random.Generator(np.random.PCG64(5))
    hex61 = synth.hex_array(61)
    jitter = hex61 + rng.normal(0.0, 2e-4, hex61.shape)     # around a 1 mm tolerance
    sparse = rng.uniform(-200, 200, (40, 3)) * np.array([1, 1, 0.01])
    line = np.array([[0.0, 0, 0], [14.6, 0, 0], [29.2, 0, 0], [58.4, 0, 0]])
    return [("hex37", synth.hex_array(37), None, 1e-6),
            ("hex61_jitter", jitter, None, 1e-3),
            ("hex61_beams", hex61, (np.arange(61) % 3).astype(np.int32), 1e-6),
            ("random", sparse, None, 1e-3),
            ("line", line, None, 1e-3)]


@pytest.mark.parametrize("name,x,bi,tol", _arrays(), ids=[a[0] for a in _arrays()])
def test_groups_match_oracle(name, x, bi, tol):
    g_lib, reps_lib = mv.redundant_groups(x, bi, tol)
    g_orc, reps_orc = submat.redundant_groups(x, bi, tol)
    np.testing.assert_array_equal(g_lib, g_orc)
    assert reps_lib == reps_orc


@pytest.mark.parametrize("n_sub", [1, 2, 3, 4])
@pytest.mark.parametrize("reverse", [False, True])
def test_plan_matches_oracle(n_sub, reverse):
    for name, x, bi, tol in _arrays():
        _, reps = submat.redundant_groups(x, bi, tol)
        if reverse:
            reps = [(b, a) for a, b in reps]
        alpha_o, sizes_o, subs_o = submat.submatrix_plan(reps, n_sub)
        alpha_l, sizes_l, dens_l = mv.submatrix_plan(reps, x.shape[0], n_sub)
        assert alpha_l == alpha_o, name
        assert sizes_l == sizes_o, name
        assert dens_l == [d for _, _, d in subs_o], name


def test_compression_on_a_redundant_hexagon():
    # App. A reports a compression of more than 15 for HERA-like arrays with three
    # sub-matrices; a plain 127-antenna hexagon is at least as redundant
    x = synth.hex_array(127)
    _, reps = mv.redundant_groups(x, None, 1e-6)
    for n_sub, at_least in ((2, 2.5), (3, 5.0)):
        _, _, subs = submat.submatrix_plan(reps, n_sub)
        size = sum(len(A) * len(B) for A, B, _ in subs)
        assert 127 * 127 / size > at_least, (n_sub, size)


def test_argument_errors():
    x = synth.hex_array(7)
    with pytest.raises(mv.MatvisError):
        mv.redundant_groups(x, None, 0.0)
    with pytest.raises(mv.MatvisError):
        mv.submatrix_plan([(0, 9)], 7, 2)
