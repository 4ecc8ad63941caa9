"""Pins for the oracle's label windows and hierarchical approximation
(Sec. 4.5): brute force over windowed labellings, the paper's statement that
block size 1 is the exact minimisation, hand-worked delegate costs, and the
bound E(approximate) >= E(exact)."""
import numpy as np
import pytest

from paper_1803_01516_amd import scenegen as sg


def test_full_windows_equal_exact(orc):
    p = sg.make_pair(sg.TINY, (1, 0))
    cost = orc.cost_volume(p.left, p.right, 8, 20)
    lo = np.zeros((48, 64), np.int32)
    hi = np.full((48, 64), 7, np.int32)
    l1, f1, e1 = orc.solve(cost, 1, 1023)
    l2, f2, e2 = orc.solve_window(cost, lo, hi, 1, 1023)
    assert (l1 == l2).all() and f1 == f2 and e1 == e2


@pytest.mark.parametrize("seed", range(6))
def test_windowed_solve_matches_brute_force(orc, seed):
    rng = np.random.default_rng(100 + seed)
    w, h, m = (3, 3, 6) if seed % 2 == 0 else (4, 2, 7)
    cost = rng.integers(0, 25, (m, h, w)).astype(np.int32)
    lo = rng.integers(0, m - 1, (h, w)).astype(np.int32)
    hi = np.minimum(m - 1, lo + rng.integers(1, 4, (h, w))).astype(np.int32)
    params = [(1, 1023), (2, 5), (0, 3)][seed % 3]
    emin, canon = orc.brute_force_window(cost, lo, hi, *params)
    for algo in ("dinic", "pushrelabel"):
        lab, flow, e = orc.solve_window(cost, lo, hi, *params, algo=algo)
        assert e == emin == flow
        assert (lab == canon).all()
        assert (lab >= lo).all() and (lab <= hi).all()


def test_coarse_cost_hand_example(orc):
    # 2x2 sites, m = 4, b = 2: one delegate site, two label groups {0,1}, {2,3}.
    # site (x=0,y=0): g = [5, 2, 7, 1] -> group mins 2, 1
    # site (x=1,y=0): g = [0, 9, 3, 4] -> 0, 3
    # site (x=0,y=1): g = [6, 6, 6, 2] -> 6, 2
    # site (x=1,y=1): g = [1, 3, 8, 8] -> 1, 8
    # delegate costs: group 0: 2+0+6+1 = 9, group 1: 1+3+2+8 = 14
    g = {(0, 0): [5, 2, 7, 1], (1, 0): [0, 9, 3, 4], (0, 1): [6, 6, 6, 2], (1, 1): [1, 3, 8, 8]}
    cost = np.zeros((4, 2, 2), np.int32)
    for (x, y), v in g.items():
        cost[:, y, x] = v
    cc = orc.coarse_cost(cost, 2)
    assert cc.shape == (2, 1, 1)
    assert cc[0, 0, 0] == 9 and cc[1, 0, 0] == 14
    # ragged edges: 3x3 sites with b = 2 -> 2x2 delegate sites, last group one label
    rng = np.random.default_rng(3)
    c3 = rng.integers(0, 30, (5, 3, 3)).astype(np.int32)
    cc3 = orc.coarse_cost(c3, 2)
    assert cc3.shape == (3, 2, 2)
    assert cc3[2, 1, 1] == c3[4, 2, 2]                       # one site, one label
    assert cc3[0, 0, 1] == min(c3[0, 0, 2], c3[1, 0, 2]) + min(c3[0, 1, 2], c3[1, 1, 2])


def test_block_size_one_is_exact(orc):
    """Sec. 4.5: with block size 1 the first cut already finds the real
    cross points, i.e. the procedure is the exact minimisation."""
    for spec, seed in [(sg.TINY, (1, 0)), (sg.spec_like(sg.MID, 96, 64, 16), (2, 1))]:
        p = sg.make_pair(spec, seed)
        cost = orc.cost_volume(p.left, p.right, spec.m, spec.cap)
        lab_e, f, e = orc.solve(cost, 1, 1023)
        lab_a, e_a, cl = orc.approx_level1(cost, 1, 1, 1023)
        assert e_a == e and (lab_a == lab_e).all() and (cl == lab_e).all()


@pytest.mark.parametrize("b", [2, 3])
def test_approximation_never_beats_exact(orc, b):
    spec = sg.spec_like(sg.MID, 120, 90, 16)
    p = sg.make_pair(spec, (2, 7))
    cost = orc.cost_volume(p.left, p.right, spec.m, spec.cap)
    _, f, e = orc.solve(cost, 1, 1023)
    lab, e_a, cl = orc.approx_level1(cost, b, 1, 1023)
    assert e_a >= e
    assert e_a == orc.energy(cost, lab, 1, 1023)
    # labels stay inside the skin of their delegate point
    lo, hi = orc.skin_windows(cl, spec.w, spec.h, spec.m, b)
    assert (lab >= lo).all() and (lab <= hi).all()


@pytest.mark.parametrize("b", [1, 2, 3])
def test_level2_is_a_labelling_in_the_skin(orc, b):
    """Level 2 cuts blocks separately, so it is no better than the exact cut;
    its labels stay inside the thin skin and its energy is recomputed from
    the definition."""
    spec = sg.spec_like(sg.MID, 96, 72, 16)
    p = sg.make_pair(spec, (2, 9))
    cost = orc.cost_volume(p.left, p.right, spec.m, spec.cap)
    _, _, opt = orc.solve(cost, 1, 1023)
    lab, e2, cl = orc.approx_level2(cost, b, 1, 1023)
    assert e2 >= opt and e2 == orc.energy(cost, lab, 1, 1023)
    lo, hi = orc.skin_windows(cl, spec.w, spec.h, spec.m, b)
    assert (lab >= lo).all() and (lab <= hi).all()
    # the first cut is the same as level 1's
    _, _, cl1 = orc.approx_level1(cost, b, 1, 1023)
    assert (cl == cl1).all()


def test_level2_single_block_is_exact(orc):
    """When one block covers the whole skin no arc is left unused, so the
    block cut is the exact restricted cut: here 3x3 sites, 3 node levels
    (m = 4) and b = 3 give a single block whose window is every label."""
    rng = np.random.default_rng(11)
    for _ in range(5):
        cost = rng.integers(0, 20, (4, 3, 3)).astype(np.int32)
        lab, e2, cl = orc.approx_level2(cost, 3, 1, 5)
        emin, _, lo, _ = orc.brute_force(cost, 1, 5)
        assert e2 == emin and (lab == lo).all()
