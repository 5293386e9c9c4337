"""Pins for the redundancy references (App. A), worked by hand from the appendix.

* baseline grouping: three antennas on a line (the two unit-spacing baselines
  share a group, the autocorrelations share one), the same line with a
  different beam in the middle (beams split groups), and invariants on a hex
  array (group members agree within tol, representatives differ beyond it,
  representatives are the first pairs of their groups, every pair is grouped);
* the sub-matrix heuristic on a four-antenna example whose threshold rounds
  are followed by hand in the comments, N_sub = 1 (the full alpha x beta
  product), and coverage of every unique pair on a hex array.
"""
import numpy as np

from oracle import submat
from paper_2312_09763_amd import synth


def test_line_of_three():
    x = np.array([[0.0, 0, 0], [14.6, 0, 0], [29.2, 0, 0]])
    g, reps = submat.redundant_groups(x, None, 1e-3)
    # pairs (0,0) (0,1) (0,2) (1,1) (1,2) (2,2): vectors 0, -d, -2d, 0, -d, 0
    assert g.tolist() == [0, 1, 2, 0, 1, 0]
    assert reps == [(0, 0), (0, 1), (0, 2)]


def test_beams_split_groups():
    x = np.array([[0.0, 0, 0], [14.6, 0, 0], [29.2, 0, 0]])
    g, reps = submat.redundant_groups(x, [0, 1, 0], 1e-3)
    # (1,1) has beams (1,1); (1,2) has beams (1,0) != (0,1) of (0,1)
    assert g.tolist() == [0, 1, 2, 3, 4, 0]
    assert reps == [(0, 0), (0, 1), (0, 2), (1, 1), (1, 2)]


def test_tolerance_is_respected():
    x = np.array([[0.0, 0, 0], [10.0, 0, 0], [20.0005, 0, 0]])
    assert submat.redundant_groups(x, None, 1e-3)[0].tolist() == [0, 1, 2, 0, 1, 0]
    assert submat.redundant_groups(x, None, 1e-4)[0].tolist() == [0, 1, 2, 0, 3, 0]


def test_hex_invariants():
    x = synth.hex_array(37)
    tol = 1e-6
    g, reps = submat.redundant_groups(x, None, tol)
    pairs = submat.pair_list(37)
    assert len(g) == 37 * 38 // 2
    for p, gi in zip(pairs, g):
        k, l = reps[gi]
        assert np.abs((x[p[0]] - x[p[1]]) - (x[k] - x[l])).max() <= tol
    # representatives: the first member of their group, pairwise distinct vectors
    first = {}
    for p, gi in zip(pairs, g):
        first.setdefault(gi, p)
    assert [first[i] for i in range(len(reps))] == reps
    vec = np.array([x[a] - x[b] for a, b in reps])
    d = np.abs(vec[:, None, :] - vec[None, :, :]).max(axis=2)
    np.fill_diagonal(d, 1.0)
    assert d.min() > tol
    # a 37-antenna hexagon is highly redundant
    assert len(reps) < 0.2 * len(pairs)


def test_heuristic_hand_example():
    U = [(0, 1), (0, 2), (0, 3), (1, 2), (2, 3), (3, 3)]
    alpha, sizes, subs = submat.submatrix_plan(U, 2)
    # multiplicities 0:3, 1:1, 2:1, 3:1 -> alpha' = [0, 1, 2, 3].  For tau > 2/3 the
    # first cut stays at {0} (D = 3/3; {0,1} gives 4/6), leaving {1,2,3} x {2,3} at
    # D = 3/6 < tau; the first tau_k = 1 - 0.01 k at or below 2/3 is 0.66: the cut
    # grows to {0,1} (D = 4/6 >= 0.66; {0,1,2} gives 5/9), leaving {2,3} x {3} at
    # D = 2/2 > 0.66.
    assert alpha == [0, 1, 2, 3]
    assert sizes == [2, 2]
    assert subs[0][0] == [0, 1] and subs[0][1] == [1, 2, 3] and abs(subs[0][2] - 4 / 6) < 1e-15
    assert subs[1][0] == [2, 3] and subs[1][1] == [3] and subs[1][2] == 1.0


def test_single_submatrix_is_the_full_product():
    U = [(0, 1), (0, 2), (0, 3), (1, 2), (2, 3), (3, 3)]
    alpha, sizes, subs = submat.submatrix_plan(U, 1)
    assert sizes == [4] and subs[0][0] == [0, 1, 2, 3] and subs[0][1] == [1, 2, 3]


def test_plan_covers_every_unique_pair():
    x = synth.hex_array(61)
    _, reps = submat.redundant_groups(x, None, 1e-6)
    for n_sub in (1, 2, 3):
        _, sizes, subs = submat.submatrix_plan(reps, n_sub)
        assert sum(sizes) == len({a for a, _ in reps})
        for a, b in reps:
            assert any(a in A and b in B for A, B, _ in subs)
        total = sum(len(A) * len(B) for A, B, _ in subs)
        if n_sub > 1:
            # fewer products than the single alpha x beta block
            _, _, one = submat.submatrix_plan(reps, 1)
            assert total <= len(one[0][0]) * len(one[0][1])
