"""Pins of the CPU reference against facts fixed outside it.

Each check ties the oracle to something it does not compute itself: hand
derivations from the paper's rules (tests/golden), brute-force Eq. (1),
closed forms, invariants of NCC and of the split-and-merge partition, and a
full sort.  The last group plants plausible mistakes in the oracle (on the CPU,
through monkeypatching) and shows that some pin catches each one.
"""

import inspect
import json
import math
import os
import textwrap
from fractions import Fraction

import numpy as np
import pytest

import oracle as O
from oracle import ncc as ONCC
from oracle import segmentation as OSEG
from oracle import select as OSEL

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _load(name):
    with open(os.path.join(GOLDEN, name)) as fh:
        return json.load(fh)


def _expr(e):
    # closed forms of the golden derivations: numbers, + - * / and sqrt only
    return float(eval(e, {"__builtins__": {}}, {"sqrt": math.sqrt}))


def _segs(ta):
    return [list(s.as_tuple()) for s in ta.segments]


# ----------------------------------------------------------------- golden files
@pytest.mark.parametrize("name", ["split_two_blocks.json", "split_merge_3x3.json"])
def test_golden_segmentation(name):
    d = _load(name)
    t = np.array(d["template"], dtype=np.uint8)
    ta = O.precompute_template_approximation(t, d["sigma_max"], d["k_max"])
    assert _segs(ta) == d["segments"]
    assert ta.k_before_merge == d["k_before_merge"]
    assert ta.sigma_used == d["sigma_used"]
    assert ta.q_k == pytest.approx(d["q_k"], rel=1e-12)
    assert ta.q_t == pytest.approx(d["q_t"], rel=1e-12)
    assert ta.rho_max == pytest.approx(d["rho_max"], abs=1e-12)


def test_golden_row_template_scores():
    d = _load("row_template_scores.json")
    t = np.array(d["template"], dtype=np.uint8)
    f = np.array(d["image"], dtype=np.uint8)
    s, s2 = O.sum_tables(f)
    for case in d["cases"]:
        ta = O.precompute_template_approximation(t, case["sigma_max"], case["k_max"])
        assert _segs(ta) == case["segments"]
        assert ta.sigma_used == case["sigma_used"]
        assert ta.q_k == pytest.approx(case["q_k"], rel=1e-13)
        assert ta.q_t == pytest.approx(case["q_t"], rel=1e-13)
        rho = O.rho_map(f, ta)
        exp_rho = np.array([[_expr(e) for e in row] for row in case["rho"]])
        np.testing.assert_allclose(rho, exp_rho, rtol=0, atol=1e-13)
        assert ta.rho_max == pytest.approx(_expr(case["rho"][0][0]), abs=1e-13)
        # energy of Eq. (16) as V / n
        _, _, V = O.window_sums(s, s2, ta.W, ta.H, np.arange(3), np.zeros(3, int))
        exp_e = [_expr(e) for e in case["energy"][0]]
        np.testing.assert_allclose(V / (ta.W * ta.H), exp_e, atol=1e-13)


# ------------------------------------------------------------------- sum tables
def test_sum_tables_closed_forms():
    # constant image c: s(x, y) = c (x+1)(y+1) on the padded grid
    N, M, c = 7, 11, 9
    s, s2 = O.sum_tables(np.full((N, M), c, np.uint8))
    yy, xx = np.mgrid[0:N + 1, 0:M + 1]
    assert (s == c * xx * yy).all()
    assert (s2 == c * c * xx * yy).all()
    # f(x, y) = x: s = y * x (x - 1) / 2 on the padded grid (x = count of columns)
    f = np.tile(np.arange(M, dtype=np.uint8), (N, 1))
    s, s2 = O.sum_tables(f)
    assert (s == yy * xx * (xx - 1) // 2).all()
    assert (s2 == yy * (xx - 1) * xx * (2 * xx - 1) // 6).all()


def test_sum_tables_recurrence_eq10():
    rng = np.random.default_rng(5)
    f = rng.integers(0, 256, (9, 13)).astype(np.uint8)
    s, s2 = O.sum_tables(f)
    fi = f.astype(np.int64)
    for y in range(9):
        for x in range(13):
            # Eq. (10) / (14) with the padded indexing
            assert s[y + 1, x + 1] == fi[y, x] + s[y + 1, x] + s[y, x + 1] - s[y, x]
            assert s2[y + 1, x + 1] == fi[y, x] ** 2 + s2[y + 1, x] + s2[y, x + 1] - s2[y, x]
    assert (s[0] == 0).all() and (s[:, 0] == 0).all()


def test_window_sums_brute():
    rng = np.random.default_rng(6)
    f = rng.integers(0, 256, (10, 12)).astype(np.uint8)
    s, s2 = O.sum_tables(f)
    W, H = 4, 3
    for v in range(10 - H + 1):
        for u in range(12 - W + 1):
            win = f[v:v + H, u:u + W].astype(np.int64)
            sf, sf2, V = O.window_sums(s, s2, W, H, u, v)
            assert sf == win.sum() and sf2 == (win * win).sum()
            assert V == W * H * (win * win).sum() - win.sum() ** 2


# --------------------------------------------------------------------- NCC pins
def _rand_case(seed, M=14, N=11, W=5, H=4, smooth=False):
    rng = np.random.default_rng(seed)
    if smooth:
        base = rng.integers(0, 256, (N // 2 + 2, M // 2 + 2))
        f = np.kron(base, np.ones((2, 2)))[:N, :M]
        f = np.clip(f + rng.integers(-3, 4, (N, M)), 0, 255).astype(np.uint8)
    else:
        f = rng.integers(0, 256, (N, M)).astype(np.uint8)
    x = int(rng.integers(0, M - W + 1))
    y = int(rng.integers(0, N - H + 1))
    t = np.clip(f[y:y + H, x:x + W].astype(int) + rng.integers(-2, 3, (H, W)), 0, 255)
    return f, t.astype(np.uint8), x, y


@pytest.mark.parametrize("seed", range(6))
def test_p1_zero_threshold_is_exact_ncc(seed):
    f, t, _, _ = _rand_case(seed, W=3 + seed % 3, H=2 + seed % 4)
    ta = O.precompute_template_approximation(t, 0)
    np.testing.assert_allclose(O.rho_map(f, ta), O.brute_ncc_map(f, t), atol=1e-12)


@pytest.mark.parametrize("seed", range(8))
def test_p2_segmented_equals_ncc_of_approximation(seed):
    f, t, _, _ = _rand_case(100 + seed, smooth=seed % 2 == 0)
    sigma = [3, 7, 15, 40][seed % 4]
    ta = O.precompute_template_approximation(t, sigma)
    k = O.approximation_image(ta.W, ta.H, ta.segments)
    assert not np.isnan(k).any()
    np.testing.assert_allclose(O.rho_map(f, ta), O.brute_ncc_map(f, k), atol=1e-12)


@pytest.mark.parametrize("seed", range(5))
def test_p3_planted_copy_gives_rho_max(seed):
    rng = np.random.default_rng(200 + seed)
    f = rng.integers(0, 256, (30, 40)).astype(np.uint8)
    t = rng.integers(0, 256, (7, 9)).astype(np.uint8)
    u, v = int(rng.integers(0, 32)), int(rng.integers(0, 24))
    f[v:v + 7, u:u + 9] = t
    ta = O.precompute_template_approximation(t, [10, 30, 45, 60, 5][seed])
    rho = O.rho_map(f, ta)
    assert rho[v, u] == pytest.approx(math.sqrt(ta.q_k / ta.q_t), abs=1e-12)
    assert ta.rho_max == pytest.approx(math.sqrt(ta.q_k / ta.q_t), abs=1e-12)


def test_p4_piecewise_constant_template_scores_one():
    rng = np.random.default_rng(7)
    t = np.zeros((12, 16), np.uint8)
    for _ in range(6):
        x, y = rng.integers(0, 12), rng.integers(0, 8)
        t[y:y + rng.integers(1, 5), x:x + rng.integers(1, 5)] = rng.integers(0, 256)
    f = rng.integers(0, 256, (40, 50)).astype(np.uint8)
    f[20:32, 5:21] = t
    ta = O.precompute_template_approximation(t, 0.5)
    k = O.approximation_image(ta.W, ta.H, ta.segments)
    assert (k == t).all()
    rho = O.rho_map(f, ta)
    assert rho[20, 5] == pytest.approx(1.0, abs=1e-12)
    assert O.argmax(rho)[:2] == (5, 20)


def test_p5_affine_invariance():
    rng = np.random.default_rng(8)
    f = rng.integers(0, 100, (20, 24)).astype(np.uint8)
    t = rng.integers(0, 100, (6, 5)).astype(np.uint8)
    ta = O.precompute_template_approximation(t, 12)
    r = O.rho_map(f, ta)
    f2 = (2 * f.astype(int) + 17).astype(np.uint8)
    np.testing.assert_allclose(O.rho_map(f2, ta), r, atol=1e-12)
    np.testing.assert_allclose(O.rho_map(255 - f, ta), -r, atol=1e-12)
    # template: t' = 2 t + 9 with sigma' = 2 sigma gives the same rectangles
    t2 = (2 * t.astype(int) + 9).astype(np.uint8)
    ta2 = O.precompute_template_approximation(t2, 24)
    assert [s.as_tuple()[:4] for s in ta2.segments] == [s.as_tuple()[:4] for s in ta.segments]
    np.testing.assert_allclose(O.rho_map(f, ta2), r, atol=1e-12)


@pytest.mark.parametrize("seed", range(4))
def test_p6_bounds_and_identities(seed):
    f, t, _, _ = _rand_case(300 + seed, M=30, N=25, W=9, H=8, smooth=True)
    ta = O.precompute_template_approximation(t, [2, 5, 9, 20][seed])
    rho = O.rho_map(f, ta)
    assert np.abs(rho).max() <= 1 + 1e-12
    assert abs(float((ta.area * ta.c).sum())) <= 1e-9 * float((ta.area * np.abs(ta.c)).sum())
    assert ta.kbar == pytest.approx(t.astype(float).mean(), abs=1e-12)
    # Eq. (12) equals sum_i box_i c_i because sum_i A_i c_i = 0
    s, s2 = O.sum_tables(f)
    vv, uu = np.meshgrid(np.arange(25 - 8 + 1), np.arange(30 - 9 + 1), indexing="ij")
    alt = np.zeros(vv.shape)
    for seg, c in zip(ta.segments, ta.c):
        alt += ONCC._box(s, uu, vv, seg.x, seg.y, seg.w, seg.h) * c
    sf, _, V = O.window_sums(s, s2, 9, 8, uu, vv)
    alt = alt / np.sqrt(V / 72.0 * ta.q_k)
    np.testing.assert_allclose(alt, rho, atol=1e-9)


# --------------------------------------------------------- segmentation invariants
def _split_path_ok(t, sigma, seg):
    """Walk from the whole template down to ``seg`` by the halving rule of
    split_segment; every rectangle above the leaf must fail Eq. (2)."""
    x, y, w, h = 0, 0, t.shape[1], t.shape[0]
    while (x, y, w, h) != (seg[0], seg[1], seg[2], seg[3]):
        blk = t[y:y + h, x:x + w].astype(np.float64)
        if w * h == 1 or blk.std() < sigma - 1e-9:
            return False            # an ancestor that should have been a leaf
        if w > h:
            a = (w + 1) // 2
            if seg[0] < x + a:
                w = a
            else:
                x, w = x + a, w // 2
        else:
            a = (h + 1) // 2
            if seg[1] < y + a:
                h = a
            else:
                y, h = y + a, h // 2
        if w == 0 or h == 0:
            return False
    return True


def _check_partition(t, ta, sigma):
    H, W = t.shape
    cover = np.zeros((H, W), int)
    for s in ta.segments:
        cover[s.y:s.y + s.h, s.x:s.x + s.w] += 1
        blk = t[s.y:s.y + s.h, s.x:s.x + s.w].astype(np.int64)
        assert s.total == blk.sum() and s.area == s.w * s.h
    assert (cover == 1).all()
    for leaf in ta.extra["leaves"]:
        blk = t[leaf.y:leaf.y + leaf.h, leaf.x:leaf.x + leaf.w].astype(np.float64)
        assert leaf.w * leaf.h == 1 or blk.std() < sigma + 1e-9
        assert _split_path_ok(t, sigma, leaf.as_tuple())
    # merge fixpoint: no aligned neighbours with equal means remain
    segs = ta.segments
    for a in segs:
        for b in segs:
            if a is b or Fraction(a.total, a.area) != Fraction(b.total, b.area):
                continue
            assert not (a.x == b.x and a.w == b.w and a.y + a.h == b.y)
            assert not (a.y == b.y and a.h == b.h and a.x + a.w == b.x)


@pytest.mark.parametrize("seed", range(20))
def test_p7_partition_invariants(seed):
    rng = np.random.default_rng(400 + seed)
    H, W = int(rng.integers(1, 14)), int(rng.integers(1, 14))
    levels = int(rng.integers(2, 6))
    t = (rng.integers(0, levels, (H, W)) * (255 // levels)).astype(np.uint8)
    if seed % 3 == 0:
        t = rng.integers(0, 256, (H, W)).astype(np.uint8)
    sigma = float(rng.choice([0.5, 3, 10, 40]))
    try:
        ta = O.precompute_template_approximation(t, sigma, k_max=10_000)
    except ValueError:
        # only a uniform approximation is rejected: all segment means equal
        leaves = []
        O.split_segment(t, sigma, 0, 0, W, H, leaves)
        means = {Fraction(s.total, s.area) for s in O.merge_redundant_segments(leaves)}
        assert len(means) == 1
        return
    _check_partition(t, ta, ta.sigma_used)
    assert ta.k_before_merge == len(ta.extra["leaves"])


def test_kmax_loop_raises_threshold_by_one():
    rng = np.random.default_rng(9)
    t = rng.integers(0, 256, (16, 16)).astype(np.uint8)
    ta = O.precompute_template_approximation(t, 4, k_max=60)
    assert ta.k_before_merge <= 60
    # one below the accepted threshold still gave too many leaves
    leaves = []
    O.split_segment(t, ta.sigma_used - 1, 0, 0, 16, 16, leaves)
    assert len(leaves) > 60
    assert (ta.sigma_used - 4) == int(ta.sigma_used - 4)


def test_std_test_is_strict_and_exact():
    # two pixels 0 and 16: population std exactly 8 -> not below 8, below 8.0001
    assert not OSEG.std_below(16, 256, 2, 8)
    assert OSEG.std_below(16, 256, 2, 8.0001)
    assert not OSEG.std_below(0, 0, 4, 0)        # sigma 0 never accepts


# ------------------------------------------------------------------- selection
def test_p9_topk_matches_full_sort():
    rng = np.random.default_rng(10)
    rho = np.round(rng.uniform(-1, 1, (6, 7)), 1)       # many ties
    entries = [(-rho[v, u], v, u) for v in range(6) for u in range(7)]
    entries.sort()
    want = [(u, v, -r) for (r, v, u) in entries[:9]]
    got = O.topk(rho, 9)
    assert [(a, b) for a, b, _ in got] == [(a, b) for a, b, _ in want]
    assert O.argmax(rho)[:2] == want[0][:2]


# ----------------------------------- coarse-to-fine selection (Sec. 5, 7f-i)
def test_top2_margin_hand_values():
    # best 0.9 twice: the margin of a tie is 0
    assert O.top2_margin(np.array([[0.5, 0.9], [0.9, 0.1]])) == 0.0
    # NaN (a map entry that was never scored) is never selected: 0.7 - 0.2
    assert O.top2_margin(np.array([[np.nan, 0.2], [0.7, 0.1]])) == pytest.approx(0.5, abs=1e-15)
    # a single offset has no runner-up
    assert O.top2_margin(np.array([[0.3]])) == float("inf")
    # negative scores: -0.1 - (-0.4)
    assert O.top2_margin(np.array([[-0.4, -0.1, -0.9]])) == pytest.approx(0.3, abs=1e-15)


@pytest.mark.parametrize("seed", range(3))
def test_top2_margin_full_sort(seed):
    rng = np.random.default_rng(20 + seed)
    rho = np.round(rng.uniform(-1, 1, (5, 9)), 1 + seed)     # ties on the first seeds
    vals = sorted(rho.ravel().tolist(), reverse=True)
    assert O.top2_margin(rho) == pytest.approx(vals[0] - vals[1], abs=1e-15)


@pytest.mark.parametrize("case", range(4))
def test_golden_neighbourhood_union(case):
    d = _load("neighbourhood_union.json")["cases"][case]
    cands = [(u, v, 0.0) for u, v in d["cands"]]
    cu, cv = OSEL.neighbourhood(cands, d["radius"], d["nu"], d["nv"])
    assert len(cu) == d["count"]
    assert [[int(v), int(u)] for u, v in zip(cu, cv)] == d["sorted_vu"]


def _brute_coarse_fine(f, coarse, fine, k, radius):
    """Steps 7f-i from brute-force Eq. (1) maps of both approximation images:
    the k best coarse offsets by a full sort, the set of offsets within
    Chebyshev distance radius of one of them, and the best fine offset there
    (ties to smaller v, then u)."""
    bc = O.brute_ncc_map(f, O.approximation_image(coarse.W, coarse.H, coarse.segments))
    bf = O.brute_ncc_map(f, O.approximation_image(fine.W, fine.H, fine.segments))
    nv, nu = bc.shape
    allc = sorted((-bc[v, u], v, u) for v in range(nv) for u in range(nu))
    cands = [(u, v) for _, v, u in allc[:k]]
    gap = allc[k - 1][0] - allc[k][0] if k < len(allc) else -np.inf
    inset = [(v, u) for v in range(nv) for u in range(nu)
             if min(max(abs(u - a), abs(v - b)) for a, b in cands) <= radius]
    ranked = sorted((-bf[v, u], v, u) for v, u in inset)
    return cands, -gap, inset, ranked, bf


@pytest.mark.parametrize("seed,k,radius", [(0, 1, 2), (1, 3, 1), (2, 5, 2), (3, 2, 0)])
def test_coarse_fine_equals_brute_force(seed, k, radius):
    f, t, _, _ = _rand_case(700 + seed, M=26, N=19, W=6, H=5, smooth=seed % 2 == 0)
    coarse = O.precompute_template_approximation(t, 30)
    fine = O.precompute_template_approximation(t, 4)
    N, M = f.shape
    s, s2 = O.sum_tables(f)
    res = O.coarse_fine(s, s2, coarse, fine, M, N, k=k, radius=radius)
    cands, gap, inset, ranked, bf = _brute_coarse_fine(f, coarse, fine, k, radius)
    assert gap > 1e-9                      # the candidate set is unique at these seeds
    assert [(u, v) for u, v, _ in res["coarse"]] == cands
    assert [(int(v), int(u)) for u, v in zip(res["fine_u"], res["fine_v"])] == inset
    np.testing.assert_allclose(res["fine_rho"], [bf[v, u] for v, u in inset], atol=1e-12)
    assert len(ranked) == 1 or ranked[1][0] - ranked[0][0] > 1e-9
    (_, bv, bu) = ranked[0]
    assert res["best"][:2] == (bu, bv)
    assert res["best"][2] == pytest.approx(bf[bv, bu], abs=1e-12)


def test_coarse_fine_ties_go_to_smaller_v_then_u():
    """Two exact copies of the template score the same rho bit for bit with
    either approximation; the result is the copy with the smaller v even
    though its u is larger."""
    rng = np.random.default_rng(77)
    f = rng.integers(0, 256, (24, 30)).astype(np.uint8)
    t = rng.integers(0, 256, (5, 6)).astype(np.uint8)
    f[3:8, 12:18] = t                      # (u, v) = (12, 3)
    f[9:14, 2:8] = t                       # (u, v) = (2, 9)
    coarse = O.precompute_template_approximation(t, 60)
    fine = O.precompute_template_approximation(t, 20)
    N, M = f.shape
    s, s2 = O.sum_tables(f)
    res = O.coarse_fine(s, s2, coarse, fine, M, N, k=2, radius=1)
    assert [(u, v) for u, v, _ in res["coarse"]] == [(12, 3), (2, 9)]
    fr = dict(zip(zip(res["fine_u"].tolist(), res["fine_v"].tolist()), res["fine_rho"]))
    assert fr[(12, 3)] == fr[(2, 9)] == max(fr.values())
    assert res["best"][:2] == (12, 3)
    assert res["best"][2] == pytest.approx(fine.rho_max, abs=1e-12)
    # the same holds with the copies in one row: the smaller u wins
    g = rng.integers(0, 256, (24, 30)).astype(np.uint8)
    g[10:15, 20:26] = t
    g[10:15, 4:10] = t
    res = O.coarse_fine(*O.sum_tables(g), coarse, fine, M, N, k=2, radius=1)
    assert res["best"][:2] == (4, 10)


# ------------------------------------------------------------------ degenerate
def test_p10_uniform_window_and_template():
    f = np.full((10, 10), 77, np.uint8)
    f[0, 0] = 3
    t = np.array([[1, 2], [3, 9]], np.uint8)
    ta = O.precompute_template_approximation(t, 0.1)
    rho, flag = O.rho_map(f, ta, return_flag=True)
    assert flag[5, 5] and rho[5, 5] == 0.0 and not flag[0, 0]
    with pytest.raises(ValueError):
        O.precompute_template_approximation(np.full((4, 4), 9, np.uint8), 1)
    with pytest.raises(ValueError):
        # sigma above the template's own deviation: one segment, uniform k
        O.precompute_template_approximation(t, 100)


def test_z1_unweighted_denominator_breaks_the_ncc_bound():
    """The printed Eq. (17) without W_i H_i would give |rho| > 1: evidence
    for the area-weighted reading."""
    t = np.array([[0, 0, 0, 0, 0, 0, 200, 0]], np.uint8)
    ta = O.precompute_template_approximation(t, 1)
    q_unweighted = float((ta.c ** 2).sum())
    assert q_unweighted < ta.q_k
    f = t.copy()
    rho_w = O.rho_map(f, ta)[0, 0]
    rho_unw = rho_w * math.sqrt(ta.q_k / q_unweighted)
    assert rho_w == pytest.approx(1.0, abs=1e-12) and rho_unw > 1.0


# ------------------------------------ the paper's two-threshold search (Sec. 5)
def test_paper_sigmas_population_std():
    t = (np.indices((6, 8)).sum(0) % 2 * 2).astype(np.uint8)   # 0/2 checker: std 1
    sf, ss = O.paper_sigmas(t)
    assert sf == pytest.approx(0.99, abs=1e-15) and ss == pytest.approx(0.1, abs=1e-15)


def _threshold_case(seed):
    rng = np.random.default_rng(500 + seed)
    f, t, x, y = _rand_case(500 + seed, M=34, N=26, W=7, H=6, smooth=seed % 2 == 1)
    f[y:y + 6, x:x + 7] = t                    # an exact copy of t at (x, y)
    sf, ss = O.paper_sigmas(t)
    fast = O.precompute_template_approximation(t, sf)
    slow = O.precompute_template_approximation(t, ss)
    return f, t, x, y, fast, slow


@pytest.mark.parametrize("seed", range(4))
def test_threshold_match_equals_brute_force(seed):
    """Survivors and matches equal the offsets where brute-force Eq. (1) with
    the fast and slow approximation images clears both thresholds."""
    f, t, x, y, fast, slow = _threshold_case(seed)
    N, M = f.shape
    s, s2 = O.sum_tables(f)
    for precision in (0.9, 0.5):
        res = O.threshold_match(s, s2, fast, slow, M, N, precision=precision)
        bf = O.brute_ncc_map(f, O.approximation_image(fast.W, fast.H, fast.segments))
        bs = O.brute_ncc_map(f, O.approximation_image(slow.W, slow.H, slow.segments))
        bf, bs = np.nan_to_num(bf, nan=0.0), np.nan_to_num(bs, nan=0.0)
        tf, ts = precision * fast.rho_max, precision * slow.rho_max
        assert res["thr_fast"] == tf and res["thr_slow"] == ts
        clear = (np.abs(bf - tf) > 1e-9) & (np.abs(bs - ts) > 1e-9)
        want_c = {(u, v) for v, u in zip(*np.nonzero((bf >= tf) & clear))}
        got_c = {(int(u), int(v)) for u, v in zip(res["cand_u"], res["cand_v"])
                 if clear[v, u]}
        assert got_c == want_c
        want_m = {(u, v) for v, u in zip(*np.nonzero((bf >= tf) & (bs >= ts) & clear))}
        got = {(u, v): r for u, v, r in res["matches"]}
        assert {k for k in got if clear[k[1], k[0]]} == want_m
        for (u, v), r in got.items():
            assert r == pytest.approx(bs[v, u], abs=1e-12)
        assert (x, y) in got                   # the copy is always found


@pytest.mark.parametrize("seed", range(3))
def test_threshold_match_planted_copy(seed):
    f, t, x, y, fast, slow = _threshold_case(10 + seed)
    N, M = f.shape
    s, s2 = O.sum_tables(f)
    res = O.threshold_match(s, s2, fast, slow, M, N)
    i = [k for k, (u, v) in enumerate(zip(res["cand_u"], res["cand_v"])) if (u, v) == (x, y)]
    assert len(i) == 1
    assert res["cand_rho"][i[0]] == pytest.approx(math.sqrt(fast.q_k / fast.q_t), abs=1e-12)
    got = {(u, v): r for u, v, r in res["matches"]}
    assert got[(x, y)] == pytest.approx(math.sqrt(slow.q_k / slow.q_t), abs=1e-12)
    # matches are a subset of the survivors, in row-major order
    keys = [(v, u) for u, v, _ in res["matches"]]
    assert keys == sorted(keys)


# ----------------------------------------------- planted mistakes are caught
def _pins_pass():
    """A compact run of the pins above; returns False on the first failure."""
    try:
        test_golden_row_template_scores()
        for name in ["split_two_blocks.json", "split_merge_3x3.json"]:
            test_golden_segmentation(name)
        for seed in range(3):
            test_p1_zero_threshold_is_exact_ncc(seed)
            test_p2_segmented_equals_ncc_of_approximation(seed)
        test_p3_planted_copy_gives_rho_max(0)
        test_p4_piecewise_constant_template_scores_one()
        for seed in range(6):
            test_p7_partition_invariants(seed)
        test_threshold_match_equals_brute_force(0)
        test_threshold_match_planted_copy(0)
        test_top2_margin_hand_values()
        test_top2_margin_full_sort(0)
        for case in range(4):
            test_golden_neighbourhood_union(case)
        test_coarse_fine_equals_brute_force(1, 3, 1)
        test_coarse_fine_ties_go_to_smaller_v_then_u()
    except (AssertionError, ValueError, IndexError, KeyError):
        return False
    return True


def test_pins_pass_unmodified():
    assert _pins_pass()


def _mutant(module, name, old, new):
    """A copy of ``module.name`` with one source fragment replaced."""
    src = textwrap.dedent(inspect.getsource(getattr(module, name)))
    assert old in src, (name, old)
    ns = dict(module.__dict__)
    exec(compile(src.replace(old, new), f"<mutant {name}>", "exec"), ns)
    return ns[name]


MUTANTS = {
    "dropped_area_weight": (OSEG, "template_constants",
                            "q_k = float((area * c * c).sum())",
                            "q_k = float((c * c).sum())"),
    "shifted_corner_row": (ONCC, "rho_map",
                           "- t[y:y + nv, x + w:x + w + nu]",
                           "- t[y + 1:y + 1 + nv, x + w:x + w + nu]"),
    "energy_sign": (ONCC, "_rho",
                    "V = n * sf2 - sf * sf", "V = n * sf2 + sf * sf"),
    "floor_first_half": (OSEG, "split_segment",
                         "first = (w + 1) // 2", "first = w // 2"),
    "split_wide_on_ties": (OSEG, "split_segment", "if w > h:", "if w >= h:"),
    "merge_ignores_width": (OSEG, "merge_redundant_segments",
                            "a.x == b.x and a.w == b.w and a.y + a.h == b.y",
                            "a.x == b.x and a.y + a.h == b.y"),
    "merge_ignores_adjacency": (OSEG, "merge_redundant_segments",
                                "a.y == b.y and a.h == b.h and a.x + a.w == b.x",
                                "a.y == b.y and a.h == b.h"),
    "mean_term_uses_wrong_area": (ONCC, "_rho",
                                  "b -= fbar * seg.area", "b -= fbar * seg.w"),
    "fast_test_inverted": (OSEL, "threshold_match",
                           "keep = np.asarray(fast_map) >= tf",
                           "keep = np.asarray(fast_map) > -tf"),
    "slow_rescored_with_fast": (OSEL, "threshold_match",
                                "rs = rho_at(s, s2, slow, cu, cv)",
                                "rs = rho_at(s, s2, fast, cu, cv)"),
    "thresholds_swapped": (OSEL, "threshold_match",
                           "tf = precision * fast.rho_max", "tf = precision * slow.rho_max"),
    "neighbourhood_radius_short": (OSEL, "neighbourhood",
                                   "for dv in range(-radius, radius + 1):",
                                   "for dv in range(-radius, radius):"),
    "neighbourhood_clip_inclusive": (OSEL, "neighbourhood",
                                     "if 0 <= uu < nu and 0 <= vv < nv:",
                                     "if 0 <= uu <= nu and 0 <= vv < nv:"),
    "fine_ties_by_u_first": (OSEL, "coarse_fine",
                             "key=lambda i: (-fr[i], cv[i], cu[i])",
                             "key=lambda i: (-fr[i], cu[i], cv[i])"),
    "fine_scored_with_coarse": (OSEL, "coarse_fine",
                                "fr = rho_at(s, s2, fine, cu, cv)",
                                "fr = rho_at(s, s2, coarse, cu, cv)"),
    "margin_of_single_offset_zero": (OSEL, "top2_margin",
                                     'if len(best) > 1 else float("inf")',
                                     "if len(best) > 1 else 0.0"),
    "margin_sign_flipped": (OSEL, "top2_margin",
                            "best = topk(rho, 2)", "best = topk(rho, 2)[::-1]"),
}


@pytest.mark.parametrize("which", sorted(MUTANTS))
def test_planted_mistake_is_caught(monkeypatch, which):
    module, name, old, new = MUTANTS[which]
    bad = _mutant(module, name, old, new)
    monkeypatch.setattr(module, name, bad)
    if hasattr(O, name):
        monkeypatch.setattr(O, name, bad)
    # a mutant may give a negative energy; its sqrt warning is expected noise
    with np.errstate(invalid="ignore"):
        assert not _pins_pass()
