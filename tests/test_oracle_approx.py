"""Pins for the oracle's label windows and hierarchical approximations
(Sec. 4.5): brute force over windowed labellings, the paper's statement that
block size 1 is the exact minimisation, hand-worked delegate costs, skin
windows and a coarse cut that only the b^2 penalty scale gives, hand-worked
states of the level-2 wave, and level 2 against an unrelated exact solver
(Dinic's maximal source side) wherever its state must be a maximum preflow."""
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


def test_skin_windows_hand_example(orc):
    """Windows of Sec. 4.5's thin skin: the delegate group and the groups
    directly above and below, clipped to [0, m-1]; ragged delegate sites."""
    cl = np.array([[0, 2], [5, 1]], np.int32)          # [Y][X], b = 3
    lo, hi = orc.skin_windows(cl, 5, 4, 16, 3)
    want = {0: (0, 5), 2: (3, 11), 5: (12, 15), 1: (0, 8)}
    for y in range(4):
        for x in range(5):
            assert (lo[y, x], hi[y, x]) == want[int(cl[y // 3, x // 3])], (x, y)


def _b2_example():
    # 4x2 sites, m = 4, b = 2: delegate sites A (x 0..1) and B (x 2..3).
    # A: group {0,1} costs min 0 per site, group {2,3} mins 3, 3, 2, 2 -> (0, 10)
    # B: group {0,1} mins 1, 1, 1, 0, group {2,3} mins 0 -> (3, 0)
    cost = np.zeros((4, 2, 4), np.int32)
    col = {(0, 0): [0, 9, 3, 9], (1, 0): [0, 9, 3, 9], (0, 1): [0, 9, 2, 9], (1, 1): [0, 9, 2, 9],
           (2, 0): [1, 9, 0, 9], (3, 0): [1, 9, 0, 9], (2, 1): [1, 9, 0, 9], (3, 1): [9, 0, 0, 9]}
    for (x, y), g in col.items():
        cost[:, y, x] = g
    return cost


def test_level1_coarse_penalty_scales_with_b_squared(orc):
    """Coarse energies of the hand example (one horizontal delegate pair,
    two coarse labels, coarse penalty c): (0,0) = 3, (0,1) = c, (1,0) =
    13 + c, (1,1) = 10.  With c = b^2 * penalty = 4 the optimum is (0,0);
    a scale of b (c = 2) or 1 would give (0,1)."""
    cost = _b2_example()
    cc = orc.coarse_cost(cost, 2)
    assert cc.shape == (2, 1, 2)
    assert cc[:, 0, 0].tolist() == [0, 10] and cc[:, 0, 1].tolist() == [3, 0]
    lab, e, cl = orc.approx_level1(cost, 2, 1, 1023)
    assert cl.tolist() == [[0, 0]]
    # the same delegate problem with the other scales picks (0, 1)
    for c in (1, 2):
        l, _, _ = orc.solve(cc, c, 1023)
        assert l.tolist() == [[0, 1]]
    l, _, _ = orc.solve(cc, 4, 1023)
    assert l.tolist() == [[0, 0]]
    assert e == orc.energy(cost, lab, 1, 1023)


INF = 1 << 52


def test_level2_wave_single_column_hand_example(orc):
    """One site, m = 5, g = [6, 4, 9, 2, 7], full window.  Balances start
    at v1 = +6 (source arc), v4 = -7 (sink arc); chain residuals 4, 9, 2.
    Distances to the deficit: 4, 3, 2, 1.  Worked by hand, step by step:
      1: v1 pushes 4 to v2; v1 keeps 2 with no residual arc -> height inf
      2: v2 pushes 4 to v3
      3: v3 pushes 2 to v4 (arc saturated); v3 relabels to 1 + h(v2) = 4
      4: v3 pushes its 2 back up to v2; v2 relabels to 1 + h(v3) = 5
      5: v2 pushes 2 down to v3; v3 relabels to 6
    The maximal source side is every level above the saturated arc v3->v4
    once step 3 has run (label 3, the cheapest label g = 2); before, it ends
    above the first saturated arc."""
    cost = np.array([6, 4, 9, 2, 7], np.int32).reshape(5, 1, 1)
    lo = np.zeros((1, 1), np.int32)
    hi = np.full((1, 1), 4, np.int32)
    want = {0: ([6, 0, 0, -7], [4, 3, 2, 1], 0),
            1: ([2, 4, 0, -7], [INF, 3, 2, 1], 1),
            2: ([2, 0, 4, -7], [INF, 3, 2, 1], 1),
            3: ([2, 0, 2, -5], [INF, 3, 4, 1], 3),
            4: ([2, 2, 0, -5], [INF, 5, 4, 1], 3),
            5: ([2, 0, 2, -5], [INF, 5, 6, 1], 3)}
    for steps, (ex, ht, label) in want.items():
        lab, e, h, _ = orc.level2_skin(cost, lo, hi, 2, steps, 0, 0, blocks=False)
        assert e.ravel().tolist() == ex, steps
        assert [min(int(v), INF) for v in h.ravel()] == ht, steps
        assert lab[0, 0] == label, steps


def test_level2_wave_lateral_hand_example(orc):
    """Two sites a (x=0), b (x=1), m = 3, penalty 1, inhibit 5.
    g_a = [5, 1, 6], g_b = [2, 7, 3].  Balances a1 = +5, a2 = -6, b1 = +2,
    b2 = -3; residuals a1->a2 1, b1->b2 7, a1<->b1 and a2<->b2 1 each way,
    a2->b1 and b2->a1 5 (inhibit), a1->b2 and b1->a2 0.  Distances 2, 1, 2, 1.
      1: a1 pushes 1 down; b1 pushes 2 down.  a1 (4 left) relabels to
         1 + h(b1) = 3.
      2: a1 pushes 1 to b1 (same level); a1 has no residual arc left ->
         height inf.  b1 keeps height 2 (its chain arc is admissible).
      3: b1 pushes 1 down; b2's deficit is filled.
    Then only a2 has a deficit; b1 and b2 reach it (b2 -> a2 has residual 1),
    a1 does not: labels (1, 0), the unique minimum E = 4 of this problem."""
    cost = np.zeros((3, 1, 2), np.int32)
    cost[:, 0, 0] = [5, 1, 6]
    cost[:, 0, 1] = [2, 7, 3]
    lo = np.zeros((1, 2), np.int32)
    hi = np.full((1, 2), 2, np.int32)
    # arrays are [level][y][x]: [[a1, b1]], [[a2, b2]]
    want = {1: ([4, 0, -5, -1], [3, 2, 1, 1]),
            2: ([3, 1, -5, -1], [INF, 2, 1, 1]),
            3: ([3, 0, -5, 0], [INF, 2, 1, 1])}
    for steps, (ex, ht) in want.items():
        lab, e, h, _ = orc.level2_skin(cost, lo, hi, 2, steps, 1, 5, blocks=False)
        assert e.ravel().tolist() == ex, steps
        assert [min(int(v), INF) for v in h.ravel()] == ht, steps
    lab, _, _, _ = orc.level2_skin(cost, lo, hi, 2, 3, 1, 5)
    assert lab.tolist() == [[1, 0]]
    emin, _, canon, _ = orc.brute_force(cost, 1, 5)
    assert emin == 4 and canon.tolist() == [[1, 0]]


def _random_windows(rng, h, w, m, b):
    Sc = rng.integers(0, -(-m // b), (-(-h // b), -(-w // b))).astype(np.int32)
    return Sc


@pytest.mark.parametrize("seed", range(6))
def test_level2_without_pairwise_terms_is_the_windowed_max_side(orc, seed):
    """Penalty and inhibit 0: columns are independent, the wave carries
    every column's flow down its chain, and the read-out must be the
    back-most minimum inside the windows (Dinic, maximal source side)."""
    rng = np.random.default_rng(300 + seed)
    b = 2 + seed % 2
    w, h, m = 7 + seed, 5 + seed % 3, 9 + 2 * seed
    cost = rng.integers(0, 20, (m, h, w)).astype(np.int32)
    cl = _random_windows(rng, h, w, m, b)
    lo, hi = orc.skin_windows(cl, w, h, m, b)
    lab, *_ = orc.level2_skin(cost, lo, hi, b, 4 * (3 * b - 1), 0, 0)
    want, _ = orc.solve_window_max_side(cost, lo, hi, 0, 0)
    assert (lab == want).all()


@pytest.mark.parametrize("seed", range(6))
def test_level2_long_wave_is_the_windowed_max_side(orc, seed):
    """With pairwise terms and a wave long enough to reach a maximum
    preflow of the skin, the maximal source side is the back-most
    windowed minimum: checked against Dinic on the windowed graph."""
    rng = np.random.default_rng(400 + seed)
    b = 2 + seed % 2
    w, h, m = 6 + seed % 3, 5, 8 + seed
    cost = rng.integers(0, 25, (m, h, w)).astype(np.int32)
    params = [(1, 1023, 1, 1023), (2, 5, 2, 5), (1, 7, 3, 0)][seed % 3]
    cl = _random_windows(rng, h, w, m, b)
    lo, hi = orc.skin_windows(cl, w, h, m, b)
    want, flow = orc.solve_window_max_side(cost, lo, hi, *params)
    lab, *_ = orc.level2_skin(cost, lo, hi, b, 600, *params)
    assert (lab == want).all()
    assert orc.energy(cost, lab, *params) == flow


@pytest.mark.parametrize("b", [2, 3])
def test_level2_blocks_alone_cut_a_skin_they_cover(orc, b):
    """No wave step: the blocks do all the work.  With m <= b every level
    falls in one label group, so w = h = b makes the skin one block and the
    block's push-relabel loop must reach the exact (back-most) cut; with
    h = 2b and no vertical pair terms the two blocks are independent
    problems and must each reach theirs."""
    rng = np.random.default_rng(50 + b)
    m = b
    for w, h, pv, iv in ((b, b, 1, 1023), (b, 2 * b, 0, 0)):
        for _ in range(4):
            cost = rng.integers(0, 20, (m, h, w)).astype(np.int32)
            lo = np.zeros((h, w), np.int32)
            hi = np.full((h, w), m - 1, np.int32)
            lab, _, _, rounds = orc.level2_skin(cost, lo, hi, b, 0, 2, 1023, pv, iv)
            want, flow = orc.solve_window_max_side(cost, lo, hi, 2, 1023, pv, iv)
            assert (lab == want).all()
            assert orc.energy(cost, lab, 2, 1023, pv, iv) == flow
            if w * h <= 9:                # brute force: every labelling
                emin, _, _, back = orc.brute_force(cost, 2, 1023, pv, iv)
                assert flow == emin and (want == back).all()


@pytest.mark.parametrize("b", [2, 3])
def test_level2_is_a_labelling_in_the_skin(orc, b):
    """Level 2 is no better than level 1 (the exact minimum inside the same
    windows), which is no better than the exact cut; its labels stay inside
    the thin skin, its energy is recomputed from the definition and its
    first cut is level 1's."""
    spec = sg.spec_like(sg.MID, 96, 72, 16)
    p = sg.make_pair(spec, (2, 9))
    cost = orc.cost_volume(p.left, p.right, spec.m, spec.cap)
    _, _, opt = orc.solve(cost, 1, 1023)
    _, e1, cl1 = orc.approx_level1(cost, b, 1, 1023)
    lab, e2, cl = orc.approx_level2(cost, b, 1, 1023)
    assert e2 >= e1 >= opt and e2 == orc.energy(cost, lab, 1, 1023)
    lo, hi = orc.skin_windows(cl, spec.w, spec.h, spec.m, b)
    assert (lab >= lo).all() and (lab <= hi).all()
    assert (cl == cl1).all()
