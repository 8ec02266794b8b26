"""HIP path against the oracle, element by element (MI355X).

Tolerances: sum tables, window sums and window energies are bit-exact
(integer work); FP32-compensated rho within 1e-5 (the bound the matching
method is held to); FP64 rho within 1e-9 (FP64 rounding of a sum of at most
a few thousand terms, each bounded by the NCC denominator, stays orders of
magnitude below this).  Argmax positions must match wherever the oracle's
top-2 margin exceeds 1e-4.
"""

import numpy as np
import pytest

import oracle as O
from oracle import select as OSEL
from workloads import synth

from gpu_util import build_sats, lib_templates, oracle_templates, topk_ok

pytestmark = pytest.mark.gpu

TOL32 = 1e-5
TOL64 = 1e-9


@pytest.fixture(scope="module")
def S():
    import paper_2502_01286_amd as S
    return S


@pytest.fixture(scope="module")
def ctx(S):
    import torch
    torch.cuda.init()
    c = S.sncc_ctx_create(0)
    yield c
    S.sncc_ctx_destroy(c)


def _u32(t):
    return t.cpu().numpy().view(np.uint32)


# ------------------------------------------------------------------ tables
@pytest.mark.parametrize("shape", [(3, 37, 29), (2, 130, 301), (1, 64, 256), (1, 1, 1),
                                   (2, 300, 517), (3, 150, 1028), (2, 720, 1280)])
def test_sat_bit_exact(S, ctx, shape):
    B, N, M = shape
    rng = np.random.default_rng(B * 1000 + N + M)
    frames = [rng.integers(0, 256, (N, M)).astype(np.uint8) for _ in range(B)]
    print("case", shape, flush=True)
    _, s, s2 = build_sats(S, ctx, frames)
    S.sncc_sync(ctx)
    P = s.shape[-1]
    gs, gs2 = _u32(s), _u32(s2)
    for b in range(B):
        os_, os2 = O.sum_tables(frames[b])
        want = np.zeros((N + 1, P), np.uint64)
        want[:, :M + 1] = os_ % (1 << 32)
        assert (gs[b].astype(np.uint64) == want).all()
        want[:, :M + 1] = os2 % (1 << 32)
        assert (gs2[b].astype(np.uint64) == want).all()


@pytest.mark.parametrize("M", [1, 3, 4, 5, 63, 64, 65, 252, 255, 256, 257, 511, 512, 640,
                               1280, 1281])
def test_sat_every_entry_written(S, ctx, M):
    """Tables pre-filled with a sentinel: every entry of every row, the zero
    column, the row total at column M and the padding columns up to the
    pitch, is written (widths at and around multiples of the 256-column tile
    and of the 64-word pitch)."""
    import torch
    N = 67
    rng = np.random.default_rng(M)
    frames = [rng.integers(0, 256, (N, M)).astype(np.uint8) for _ in range(2)]
    f = torch.from_numpy(np.stack(frames)).cuda()
    P = S.sncc_sat_pitch(M)
    print("case", M, P, flush=True)
    s = torch.full((2, N + 1, P), -0x21524111, dtype=torch.int32, device="cuda")
    s2 = torch.full_like(s, -0x21524111)
    S.sncc_build_sats(ctx, f, s, s2)
    S.sncc_sync(ctx)
    gs, gs2 = _u32(s), _u32(s2)
    for b in range(2):
        os_, os2 = O.sum_tables(frames[b])
        want = np.zeros((N + 1, P), np.uint64)
        want[:, :M + 1] = os_ % (1 << 32)
        assert (gs[b].astype(np.uint64) == want).all()
        want[:, :M + 1] = os2 % (1 << 32)
        assert (gs2[b].astype(np.uint64) == want).all()


def test_sat_wraps_modulo_2_32_and_windows_stay_exact(S, ctx):
    # all-255 frame: s^2 exceeds 2^32 many times over; 256x256 windows of f^2
    # (the largest template of the workloads) are still exact
    N, M = 700, 900
    f = np.full((N, M), 255, np.uint8)
    f[::7, ::5] = 3
    _, s, s2 = build_sats(S, ctx, [f])
    S.sncc_sync(ctx)
    gs, gs2 = _u32(s)[0].astype(np.int64), _u32(s2)[0].astype(np.int64)
    os_, os2 = O.sum_tables(f)
    assert (gs[:, :M + 1] == os_ % (1 << 32)).all()
    assert (gs2[:, :M + 1] == os2 % (1 << 32)).all()
    rng = np.random.default_rng(1)
    for _ in range(200):
        u, v = int(rng.integers(0, M - 256 + 1)), int(rng.integers(0, N - 256 + 1))
        box = lambda t: (t[v + 256, u + 256] - t[v + 256, u] - t[v, u + 256] + t[v, u]) % (1 << 32)
        sf, sf2, V = O.window_sums(os_, os2, 256, 256, u, v)
        assert box(gs) == sf and box(gs2) == sf2
        assert sf2 < (1 << 32)


# ------------------------------------------------------------------- maps
def _case(seed, M, N, W, H, sigma, flat_region=False):
    f = synth.scene(seed, M, N)
    if flat_region:
        f[10:10 + H + 20, 20:20 + W + 30] = 77          # uniform windows
    rng = np.random.default_rng(seed + 1)
    t, x, y = synth.crop_template(rng, f, W, H, sigma_max=sigma)
    return f, t


MAP_CASES = [
    # seed, M, N, W, H, sigma
    (1, 200, 150, 17, 13, 8),
    (2, 203, 131, 32, 32, 4),
    (3, 260, 170, 64, 40, 16),
    (4, 96, 80, 96, 80, 8),      # template = image: one offset
    (5, 300, 90, 7, 60, 4),
    (6, 400, 300, 150, 150, 4),  # several LDS passes
    (7, 333, 222, 200, 31, 12),
]


def _special_template(kind, rng):
    """Templates whose segmentations stress the record layout: long runs of
    segments with equal rows (stripes), one-pixel-wide or one-row templates,
    and a 2 x 2 template."""
    if kind == "stripes":     # 40 x 24: 8 bands of rows, columns of width 3
        t = (np.indices((24, 40))[1] // 3 % 2) * 90 + (np.indices((24, 40))[0] // 3) * 12 + 20
        return np.clip(t + rng.integers(0, 2, (24, 40)), 0, 255).astype(np.uint8), 1.5
    if kind == "column":      # W = 1
        return rng.integers(0, 256, (20, 1)).astype(np.uint8), 30.0
    if kind == "row":         # H = 1
        return rng.integers(0, 256, (1, 25)).astype(np.uint8), 30.0
    return np.array([[10, 200], [90, 30]], np.uint8), 0.5   # 2 x 2


@pytest.mark.parametrize("kind", ["stripes", "column", "row", "tiny"])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_map_parity_special_templates(S, ctx, kind, precision):
    import torch
    rng = np.random.default_rng(["stripes", "column", "row", "tiny"].index(kind) + 500)
    t, sigma = _special_template(kind, rng)
    H, W = t.shape
    M, N = 170, 120
    f = synth.scene(77, M, N)
    f[30:30 + H, 40:40 + W] = t                     # an exact copy
    print("template", kind, t.shape, precision, flush=True)
    _, s, s2 = build_sats(S, ctx, [f])
    tm = lib_templates(S, ctx, [t], [sigma])
    ta = oracle_templates([t], [sigma])[0]
    if kind == "stripes":
        hz = {}
        for g in ta.segments:
            hz.setdefault((g.y, g.h), []).append(g.x)
        assert max(len(v) for v in hz.values()) > 4    # chains longer than one piece
    nu, nv = M - W + 1, N - H + 1
    prec = S.SNCC_FP64 if precision == "fp64" else S.SNCC_FP32_KAHAN
    dt = torch.float64 if precision == "fp64" else torch.float32
    rho = torch.empty((nv, nu), dtype=dt, device="cuda")
    S.sncc_score(ctx, tm, 0, s, s2, M, N, prec, rho)
    S.sncc_sync(ctx)
    got = rho.cpu().numpy().astype(np.float64)
    want = O.rho_map(f, ta)
    tol = TOL64 if precision == "fp64" else TOL32
    assert np.abs(got - want).max() <= tol
    assert abs(got[30, 40] - ta.rho_max) <= tol       # the copy scores rho_max
    S.sncc_tmpl_destroy(tm)


@pytest.mark.parametrize("case", MAP_CASES)
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_map_parity(S, ctx, case, precision):
    import torch
    seed, M, N, W, H, sigma = case
    print("case", case, precision, flush=True)
    f, t = _case(seed, M, N, W, H, sigma, flat_region=(seed == 1))
    _, s, s2 = build_sats(S, ctx, [f])
    tm = lib_templates(S, ctx, [t], [sigma])
    nu, nv = M - W + 1, N - H + 1
    prec = S.SNCC_FP64 if precision == "fp64" else S.SNCC_FP32_KAHAN
    dt = torch.float64 if precision == "fp64" else torch.float32
    pitch = nu + 3
    rho = torch.full((nv, pitch), float("nan"), dtype=dt, device="cuda")
    deg = torch.full((nv, pitch), 7, dtype=torch.uint8, device="cuda")
    S.sncc_score(ctx, tm, 0, s, s2, M, N, prec, rho, deg)
    S.sncc_sync(ctx)
    got = rho.cpu().numpy()[:, :nu].astype(np.float64)
    gdeg = deg.cpu().numpy()[:, :nu]
    ta = oracle_templates([t], [sigma])[0]
    want, flat = O.rho_map(f, ta, return_flag=True)
    tol = TOL64 if precision == "fp64" else TOL32
    err = np.abs(got - want)
    assert np.isfinite(got).all()
    assert err.max() <= tol, (err.max(), np.unravel_index(err.argmax(), err.shape))
    assert (gdeg == flat.astype(np.uint8)).all()
    assert (rho.cpu().numpy()[:, nu:] != rho.cpu().numpy()[:, nu:]).all()  # pad untouched
    if O.top2_margin(want) > 1e-4:
        gi = np.unravel_index(np.argmax(got), got.shape)
        assert O.argmax(want)[:2] == (gi[1], gi[0])
    S.sncc_tmpl_destroy(tm)


def test_fp32_map_deterministic(S, ctx):
    import torch
    f, t = _case(11, 300, 200, 48, 40, 4)
    _, s, s2 = build_sats(S, ctx, [f])
    tm = lib_templates(S, ctx, [t], [4])
    nu, nv = 300 - 48 + 1, 200 - 40 + 1
    a = torch.empty((nv, nu), dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    S.sncc_score(ctx, tm, 0, s, s2, 300, 200, S.SNCC_FP32_KAHAN, a)
    S.sncc_score(ctx, tm, 0, s, s2, 300, 200, S.SNCC_FP32_KAHAN, b)
    S.sncc_sync(ctx)
    assert torch.equal(a.view(torch.int32), b.view(torch.int32))


# ------------------------------------------------------------------- top-k
def _multi(seed, B=3, M=240, N=180, sides=((24, 30), (40, 33), (17, 64), (64, 20)),
           sigmas=(16, 8, 4, 12)):
    frames = [synth.scene(seed + i, M, N) for i in range(B)]
    rng = np.random.default_rng(seed)
    temps = []
    for (W, H), sg in zip(sides, sigmas):
        fi = int(rng.integers(0, B))
        t, _, _ = synth.crop_template(rng, frames[fi], W, H, sigma_max=sg)
        temps.append(t)
    pairs = [(b, t) for b in range(B) for t in range(len(temps))]
    return frames, temps, list(sigmas), pairs


@pytest.mark.parametrize("k", [1, 5, 32, 64])
@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_topk_parity(S, ctx, k, precision):
    import torch
    frames, temps, sigmas, pairs = _multi(50 + k)
    B, N, M = len(frames), frames[0].shape[0], frames[0].shape[1]
    print("case k", k, precision, flush=True)
    _, s, s2 = build_sats(S, ctx, frames)
    tm = lib_templates(S, ctx, temps, sigmas)
    out = torch.zeros((len(pairs), k, 3), dtype=torch.int32, device="cuda")
    prec = S.SNCC_FP64 if precision == "fp64" else S.SNCC_FP32_KAHAN
    S.sncc_topk(ctx, tm, s, s2, B, M, N, pairs, k, prec, out)
    S.sncc_sync(ctx)
    got = S.decode_matches(out)
    tas = oracle_templates(temps, sigmas)
    tables = [O.sum_tables(f) for f in frames]
    for p, (b, ti) in enumerate(pairs):
        want_map = O.rho_map(frames[b], tas[ti], tables=tables[b])
        errs = topk_ok(want_map, got[p], k, TOL32)
        assert not errs, (p, errs[:5])


def test_fp64_topk_orders_by_the_double_value(S, ctx):
    """Two copies of the template, the second with one pixel raised and one
    lowered by a grey level (chosen so that its rho exceeds the first copy's by
    about 1.2e-8, below float resolution at 0.9999): the FP64 top-k ranks by the
    double value, so the second copy (larger offset index) comes first, and
    the whole list is the order of a full sort of the FP64 map with key
    (rho desc, v, u).  A float key would tie the two and put the first copy
    first."""
    import torch
    rng = np.random.default_rng(123)
    M, N, W, H = 300, 200, 20, 16
    f = rng.integers(0, 200, (N, M)).astype(np.uint8)
    t = rng.integers(10, 200, (H, W)).astype(np.uint8)
    (x1, y1), (x2, y2) = (40, 20), (200, 150)
    f[y1:y1 + H, x1:x1 + W] = t
    f[y2:y2 + H, x2:x2 + W] = t
    f[y2 + 7, x2 + 15] += 1
    f[y2 + 14, x2 + 19] -= 1
    ta = O.precompute_template_approximation(t, 6)
    s_o, s2_o = O.sum_tables(f)
    r1 = float(O.rho_at(s_o, s2_o, ta, x1, y1))
    r2 = float(O.rho_at(s_o, s2_o, ta, x2, y2))
    assert 1e-9 < r2 - r1 < 3e-8 and np.float32(r1) == np.float32(r2)
    _, s, s2 = build_sats(S, ctx, [f])
    tm = lib_templates(S, ctx, [t], [6])
    nu, nv = M - W + 1, N - H + 1
    r64 = torch.empty((nv, nu), dtype=torch.float64, device="cuda")
    out = torch.zeros((1, 8, 3), dtype=torch.int32, device="cuda")
    S.sncc_score(ctx, tm, 0, s, s2, M, N, S.SNCC_FP64, r64)
    S.sncc_topk(ctx, tm, s, s2, 1, M, N, [(0, 0)], 8, S.SNCC_FP64, out)
    S.sncc_sync(ctx)
    S.sncc_tmpl_destroy(tm)
    m = r64.cpu().numpy()
    flat = [(-m[v, u], v, u) for v in range(nv) for u in range(nu)]
    flat.sort()
    want = [(u, v) for _, v, u in flat[:8]]
    got = S.decode_matches(out)[0]
    order = [(int(a), int(b)) for a, b in zip(got["u"], got["v"])]
    assert order == want
    assert np.array_equal(got["rho"], np.float32([-x for x, _, _ in flat[:8]]))
    assert order[:2] == [(x2, y2), (x1, y1)]


def test_topk_more_slots_than_offsets(S, ctx):
    import torch
    f = synth.scene(9, 40, 30)
    rng = np.random.default_rng(2)
    t, _, _ = synth.crop_template(rng, f, 36, 27, sigma_max=4)
    _, s, s2 = build_sats(S, ctx, [f])
    tm = lib_templates(S, ctx, [t], [4])
    out = torch.zeros((1, 32, 3), dtype=torch.int32, device="cuda")
    S.sncc_topk(ctx, tm, s, s2, 1, 40, 30, [(0, 0)], 32, S.SNCC_FP32_KAHAN, out)
    S.sncc_sync(ctx)
    got = S.decode_matches(out)[0]
    n_off = (40 - 36 + 1) * (30 - 27 + 1)
    assert (got["u"][:n_off] >= 0).all()
    assert (got["u"][n_off:] == -1).all() and np.isneginf(got["rho"][n_off:]).all()
    want = O.rho_map(f, oracle_templates([t], [4])[0])
    assert not topk_ok(want, got, n_off, TOL32)


def test_topk_repeated_calls_match_fresh_contexts(S, ctx):
    """A context keeps the plan of its last top-k call and reuses it when the
    call repeats; each change of what the plan depends on (k, the pair list,
    the template set) and each change of the tables (not part of the plan)
    must give exactly what a fresh context gives."""
    import torch
    frames, temps, sigmas, pairs = _multi(90)
    B, N, M = len(frames), frames[0].shape[0], frames[0].shape[1]
    _, s, s2 = build_sats(S, ctx, frames)
    _, r, r2 = build_sats(S, ctx, [synth.scene(990 + i, M, N) for i in range(B)])
    tm = lib_templates(S, ctx, temps, sigmas)
    tm2 = lib_templates(S, ctx, temps[::-1], sigmas[::-1])

    def run(c, t, tabs, pr, k):
        out = torch.zeros((len(pr), k, 3), dtype=torch.int32, device="cuda")
        S.sncc_topk(c, t, tabs[0], tabs[1], B, M, N, pr, k, S.SNCC_FP32_KAHAN, out)
        S.sncc_sync(c)
        return out.cpu().numpy()

    calls = [(tm, (s, s2), pairs, 8), (tm, (s, s2), pairs, 8), (tm, (r, r2), pairs, 8),
             (tm, (r, r2), pairs, 3), (tm, (r, r2), pairs[::-1], 3), (tm2, (r, r2), pairs[::-1], 3),
             (tm, (s, s2), pairs, 8)]
    got = [run(ctx, *c) for c in calls]
    for i, (c, g) in enumerate(zip(calls, got)):
        fresh = S.sncc_ctx_create(0)
        try:
            want = run(fresh, *c)
        finally:
            S.sncc_ctx_destroy(fresh)
        assert np.array_equal(g, want), i
    assert np.array_equal(got[0], got[1]) and np.array_equal(got[0], got[-1])
    assert not np.array_equal(got[1], got[2])
    for h in (tm, tm2):
        S.sncc_tmpl_destroy(h)


def test_one_item_per_workgroup_matches_the_queues(S, ctx, monkeypatch):
    """Small launches run one workgroup per item without queue counters or
    pair floors; the same calls through the work queues (forced by the
    library's SNCC_TEST_QUEUES hook) must give the same maps bit for bit and
    the same top-k lists."""
    import torch
    frames, temps, sigmas, pairs = _multi(91)
    B, N, M = len(frames), frames[0].shape[0], frames[0].shape[1]
    _, s, s2 = build_sats(S, ctx, frames)
    tm = lib_templates(S, ctx, temps, sigmas)
    W, H, _, _ = S.sncc_tmpl_info(tm, 2)

    def run():
        out = {}
        for k in (1, 5, 32):
            o = torch.zeros((len(pairs), k, 3), dtype=torch.int32, device="cuda")
            S.sncc_topk(ctx, tm, s, s2, B, M, N, pairs, k, S.SNCC_FP32_KAHAN, o)
            out[k] = o
        rho = torch.zeros((N - H + 1, M - W + 1), dtype=torch.float32, device="cuda")
        S.sncc_score(ctx, tm, 2, s[1], s2[1], M, N, S.SNCC_FP32_KAHAN, rho)
        S.sncc_sync(ctx)
        return {k: v.cpu().numpy() for k, v in out.items()}, rho.cpu().numpy()

    monkeypatch.delenv("SNCC_TEST_QUEUES", raising=False)
    lists, rho = run()
    monkeypatch.setenv("SNCC_TEST_QUEUES", "1")
    lists_q, rho_q = run()
    monkeypatch.delenv("SNCC_TEST_QUEUES")
    assert np.array_equal(rho.view(np.uint32), rho_q.view(np.uint32))
    for k in lists:
        assert np.array_equal(lists[k], lists_q[k]), k
    S.sncc_tmpl_destroy(tm)


def test_map_repeated_calls_match_fresh_contexts(S, ctx):
    """A context keeps the plan of its last FP32 map call; calls that change
    the template index, the template set or the tables must give exactly what
    a fresh context gives."""
    import torch
    frames, temps, sigmas, _ = _multi(95, B=2)
    N, M = frames[0].shape
    _, s, s2 = build_sats(S, ctx, frames[:1])
    _, r, r2 = build_sats(S, ctx, frames[1:])
    tm = lib_templates(S, ctx, temps, sigmas)
    tm2 = lib_templates(S, ctx, temps[::-1], sigmas[::-1])

    def run(c, t, i, tabs):
        W, H, _, _ = S.sncc_tmpl_info(t, i)
        out = torch.full((N - H + 1, M - W + 1), 7.0, dtype=torch.float32, device="cuda")
        S.sncc_score(c, t, i, tabs[0], tabs[1], M, N, S.SNCC_FP32_KAHAN, out)
        S.sncc_sync(c)
        return out.cpu().numpy()

    calls = [(tm, 0, (s, s2)), (tm, 0, (s, s2)), (tm, 1, (s, s2)), (tm, 1, (r, r2)),
             (tm2, 2, (r, r2)), (tm, 0, (s, s2))]
    got = [run(ctx, *c) for c in calls]
    for i, (c, g) in enumerate(zip(calls, got)):
        fresh = S.sncc_ctx_create(0)
        try:
            want = run(fresh, *c)
        finally:
            S.sncc_ctx_destroy(fresh)
        assert np.array_equal(g, want), i
    assert np.array_equal(got[0], got[1]) and np.array_equal(got[0], got[-1])
    for h in (tm, tm2):
        S.sncc_tmpl_destroy(h)


# ------------------------------------------------------------------ refine
@pytest.mark.parametrize("case", ["default", "large_fine", "radius3", "wide_frame", "two_classes"])
def test_refine_parity(S, ctx, case):
    """FP64 refine against the oracle's coarse-fine.  `large_fine` adds a
    130 x 100 template, whose chunk region exceeds the LDS budget (scored from
    the global tables); `radius3` uses +-3 px neighbourhoods; `wide_frame` is
    an 8300-wide frame, where a 64-tall template's staged regions are made
    row-relative (255 H P >= 2^27) and a 20-tall one's are not; `two_classes`
    pairs a small template with a 90 x 95 one whose chunk region (43 KB)
    is too large for four workgroups per CU, so the refine runs in two
    launches."""
    import torch
    if case == "large_fine":
        frames, temps, _, pairs = _multi(71, B=2, M=300, N=220, sides=((24, 30), (130, 100)),
                                         sigmas=(16, 16))
    elif case == "two_classes":
        frames, temps, _, pairs = _multi(74, B=2, M=320, N=240, sides=((24, 30), (90, 95)),
                                         sigmas=(16, 16))
    elif case == "wide_frame":
        frames, temps, _, pairs = _multi(73, B=1, M=8300, N=90, sides=((24, 64), (30, 20)),
                                         sigmas=(16, 16))
    else:
        frames, temps, _, pairs = _multi(70, sigmas=(16, 16, 16, 16))
    print("case", case, flush=True)
    B, N, M = len(frames), frames[0].shape[0], frames[0].shape[1]
    coarse_s, fine_s = [16] * len(temps), [4] * len(temps)
    _, s, s2 = build_sats(S, ctx, frames)
    fine = lib_templates(S, ctx, temps, fine_s)
    tas_c = oracle_templates(temps, coarse_s)
    tas_f = oracle_templates(temps, fine_s)
    tables = [O.sum_tables(f) for f in frames]
    k, radius = 8, (3 if case == "radius3" else 2)
    # candidates from the oracle's coarse pass, given to both sides as input
    cand = np.zeros((len(pairs), k, 3), np.int32)
    expected = []
    for p, (b, ti) in enumerate(pairs):
        res = O.coarse_fine(*tables[b], tas_c[ti], tas_f[ti], M, N, k=k, radius=radius)
        for j, (u, v, r) in enumerate(res["coarse"]):
            cand[p, j] = (u, v, np.float32(r).view(np.int32))
        expected.append(res)
    cand[0, k - 1] = (-1, -1, 0)          # an empty slot is ignored
    expected[0] = O.coarse_fine(*tables[pairs[0][0]], tas_c[pairs[0][1]], tas_f[pairs[0][1]],
                                M, N, k=k - 1, radius=radius)
    dcand = torch.from_numpy(cand).cuda()
    out = torch.zeros((len(pairs), 4), dtype=torch.int32, device="cuda")
    cnt = torch.zeros(len(pairs), dtype=torch.int32, device="cuda")
    S.sncc_refine(ctx, fine, s, s2, B, M, N, pairs, dcand, radius, out, cnt)
    S.sncc_sync(ctx)
    got = S.decode_matches64(out)
    counts = cnt.cpu().numpy()
    for p in range(len(pairs)):
        res = expected[p]
        assert counts[p] == len(res["fine_u"])
        assert (int(got[p]["u"]), int(got[p]["v"])) == res["best"][:2], p
        assert abs(float(got[p]["rho"]) - res["best"][2]) <= TOL64


@pytest.mark.parametrize("n_cand,radius", [(96, 1), (300, 0), (64, 2), (65, 2)])
def test_refine_many_candidates(S, ctx, n_cand, radius):
    """Candidate lists longer than a wavefront (up to n_cand (2 radius + 1)^2 =
    4096 entries are allowed): clustered and scattered offsets, duplicates and
    empty slots.  Count = the oracle's neighbourhood union, best = the
    oracle's FP64 argmax over it (rho desc, then v, then u)."""
    import torch
    frames, temps, _, pairs = _multi(72, sigmas=(16, 16, 16, 16))
    print("case", n_cand, radius, flush=True)
    B, N, M = len(frames), frames[0].shape[0], frames[0].shape[1]
    _, s, s2 = build_sats(S, ctx, frames)
    fine = lib_templates(S, ctx, temps, [4] * len(temps))
    tas_f = oracle_templates(temps, [4] * len(temps))
    tables = [O.sum_tables(f) for f in frames]
    rng = np.random.default_rng(n_cand * 10 + radius)
    cand = np.zeros((len(pairs), n_cand, 3), np.int32)
    for p, (b, ti) in enumerate(pairs):
        nu, nv = M - temps[ti].shape[1] + 1, N - temps[ti].shape[0] + 1
        cu, cv = int(rng.integers(0, nu)), int(rng.integers(0, nv))
        for j in range(n_cand):
            if j % 3 == 0:      # scattered
                u, v = int(rng.integers(0, nu)), int(rng.integers(0, nv))
            else:               # a cluster, reaching past the edges
                u = int(np.clip(cu + rng.integers(-6, 7), -2, nu + 1))
                v = int(np.clip(cv + rng.integers(-6, 7), -2, nv + 1))
                u, v = min(max(u, 0), nu - 1), min(max(v, 0), nv - 1)
            cand[p, j] = (u, v, 0)
        cand[p, 5] = cand[p, 2]              # a duplicate
        cand[p, n_cand - 1] = (-1, -1, 0)    # an empty slot
    dcand = torch.from_numpy(cand).cuda()
    out = torch.zeros((len(pairs), 4), dtype=torch.int32, device="cuda")
    cnt = torch.zeros(len(pairs), dtype=torch.int32, device="cuda")
    S.sncc_refine(ctx, fine, s, s2, B, M, N, pairs, dcand, radius, out, cnt)
    S.sncc_sync(ctx)
    got = S.decode_matches64(out)
    counts = cnt.cpu().numpy()
    for p, (b, ti) in enumerate(pairs):
        nu, nv = M - temps[ti].shape[1] + 1, N - temps[ti].shape[0] + 1
        valid = [(int(u), int(v), 0.0) for u, v, _ in cand[p] if u >= 0]
        us, vs = OSEL.neighbourhood(valid, radius, nu, nv)
        assert counts[p] == len(us), (p, counts[p], len(us))
        rho = np.array([float(O.rho_at(*tables[b], tas_f[ti], int(u), int(v)))
                        for u, v in zip(us, vs)])
        order = sorted(range(len(us)), key=lambda i: (-rho[i], vs[i], us[i]))
        best = order[0]
        assert (int(got[p]["u"]), int(got[p]["v"])) == (int(us[best]), int(vs[best])), p
        assert abs(float(got[p]["rho"]) - rho[best]) <= TOL64


# ------------------------------------------------------------------ batches
@pytest.mark.parametrize("case", ["mixed", "narrow"])
def test_batch_graph_parity_and_replays(S, ctx, case):
    """One graph-captured batch replayed three times, against the oracle.
    Both cases have pairs whose last column of 128-wide tiles holds at most
    64 offsets (scored by the second launch); in `narrow` a 150 px template
    on 200 px frames leaves 51 offset columns, so its pairs have no tiles in
    the main launch at all (and k = 64, radius 1)."""
    import torch
    if case == "narrow":
        frames, temps, _, pairs = _multi(91, B=3, M=200, N=150,
                                         sides=((150, 40), (70, 30), (24, 24)),
                                         sigmas=(16, 16, 16))
    else:
        frames, temps, _, pairs = _multi(90, B=4, M=320, N=200,
                                         sides=((24, 24), (40, 30), (64, 48), (33, 70), (90, 41)),
                                         sigmas=(16, 16, 16, 16, 16))
    print("case", case, flush=True)
    B, N, M = len(frames), frames[0].shape[0], frames[0].shape[1]
    k, radius = (64, 1) if case == "narrow" else (16, 2)   # k = 64: one item per merge load
    f = torch.from_numpy(np.stack(frames)).cuda()
    P = S.sncc_sat_pitch(M)
    s = torch.zeros((B, N + 1, P), dtype=torch.int32, device="cuda")
    s2 = torch.zeros_like(s)
    coarse = lib_templates(S, ctx, temps, [16] * len(temps))
    fine = lib_templates(S, ctx, temps, [4] * len(temps))
    topk = torch.zeros((len(pairs), k, 3), dtype=torch.int32, device="cuda")
    best = torch.zeros((len(pairs), 4), dtype=torch.int32, device="cuda")
    cnt = torch.zeros(len(pairs), dtype=torch.int32, device="cuda")
    batch = S.sncc_batch_create(ctx, coarse, s, s2, B, M, N, pairs, k, topk, fine=fine,
                                radius=radius, best_out=best, count_out=cnt, frames=f)
    tas_c = oracle_templates(temps, [16] * len(temps))
    tas_f = oracle_templates(temps, [4] * len(temps))
    tables = [O.sum_tables(fr) for fr in frames]
    results = []
    for rep in range(3):
        topk.zero_()
        best.zero_()
        S.sncc_batch_run(batch)
        S.sncc_sync(ctx)
        results.append((topk.clone(), best.clone()))
        _ = torch.randn(1000, device="cuda").sum().item()   # eager work between replays
    for a, b in results[1:]:
        assert torch.equal(a, results[0][0]) and torch.equal(b, results[0][1])
    st = batch.stats()
    assert st["coarse_evals"] > 0 and st["ms_total"] != 0
    assert st["n_launch_classes"] == 2
    got = S.decode_matches(results[0][0])
    gbest = S.decode_matches64(results[0][1])
    for p, (b, ti) in enumerate(pairs):
        cmap = O.rho_map(frames[b], tas_c[ti], tables=tables[b])
        errs = topk_ok(cmap, got[p], k, TOL32)
        assert not errs, (p, errs[:4])
        want = O.topk(cmap, k + 1)
        res = O.coarse_fine(*tables[b], tas_c[ti], tas_f[ti], M, N, k=k, radius=radius,
                            coarse_map=cmap)
        gu, gv, gr = int(gbest[p]["u"]), int(gbest[p]["v"]), float(gbest[p]["rho"])
        # the fine score the GPU reports is the oracle's fine score there
        assert abs(O.rho_at(*tables[b], tas_f[ti], gu, gv) - gr) <= TOL64
        if want[k - 1][2] - want[k][2] > 2e-5:   # coarse candidate sets are unique
            assert (gu, gv) == res["best"][:2], p
    batch.destroy()
    assert _u32(s)[0, 0, 0] == 0


@pytest.mark.parametrize("case", ["staged", "direct"])
def test_batch_every_tile_config(S, ctx, tmp_path, case):
    """Every tile configuration the tuner can choose gives the oracle's top-k.
    The first creation times them all and records the winner in the tuning
    cache under the batch's key; each configuration is then forced by
    rewriting that entry.  The shapes: 128x32, 128x16 (four or eight waves),
    64x64, 64x32 and 64x16 offsets per tile, the 128-wide ones with their
    last-column launch where they have a half-width twin (a 70 px template on
    260 px frames leaves a last column of 63 offsets).  In `direct` a 530 px
    wide template is too wide for one LDS row: the 16-row tiles stage it in
    two column bands (384 + 146 columns); for the 32- and 64-row tiles a
    chain of its 36 px tall segments needs more band rows than the LDS holds,
    so they score it in the direct form; next to a staged template."""
    import re
    import torch
    if case == "direct":
        frames, temps, _, pairs = _multi(93, B=2, M=700, N=160,
                                         sides=((530, 36), (30, 30)), sigmas=(16, 16))
    else:
        frames, temps, _, pairs = _multi(92, B=3, M=260, N=170,
                                         sides=((24, 24), (40, 30), (70, 41), (33, 60)),
                                         sigmas=(16, 16, 16, 16))
    B, N, M = len(frames), frames[0].shape[0], frames[0].shape[1]
    k = 8
    f = torch.from_numpy(np.stack(frames)).cuda()
    P = S.sncc_sat_pitch(M)
    s = torch.zeros((B, N + 1, P), dtype=torch.int32, device="cuda")
    s2 = torch.zeros_like(s)
    coarse = lib_templates(S, ctx, temps, [16] * len(temps))
    topk = torch.zeros((len(pairs), k, 3), dtype=torch.int32, device="cuda")
    cache = str(tmp_path / "tune.json")
    S.sncc_batch_create(ctx, coarse, s, s2, B, M, N, pairs, k, topk, frames=f, tune=1,
                        tune_cache=cache).destroy()
    key = re.search(r'"([^"]+)"\s*:', open(cache).read()).group(1)
    tas = oracle_templates(temps, [16] * len(temps))
    tables = [O.sum_tables(fr) for fr in frames]
    maps = [O.rho_map(frames[b], tas[ti], tables=tables[b]) for b, ti in pairs]
    shapes = set()
    for cfg in range(8):
        with open(cache, "w") as fh:
            fh.write('{\n  "%s": %d\n}\n' % (key, cfg))
        print("tile config", cfg, flush=True)
        batch = S.sncc_batch_create(ctx, coarse, s, s2, B, M, N, pairs, k, topk, frames=f,
                                    tune=1, tune_cache=cache)
        topk.zero_()
        S.sncc_batch_run(batch)
        S.sncc_sync(ctx)
        st = batch.stats()
        shapes.add((st["tile_u"], st["tile_v"], st["wg_threads"]))
        got = S.decode_matches(topk)
        for p in range(len(pairs)):
            errs = topk_ok(maps[p], got[p], k, TOL32)
            assert not errs, (cfg, p, errs[:4])
        batch.destroy()
    assert shapes == {(128, 32, 512), (128, 16, 256), (128, 16, 512), (64, 64, 512),
                      (64, 32, 512), (64, 16, 256)}


# ------------------------------------------------------------- edge cases
def test_errors(S, ctx):
    import torch
    f = synth.scene(3, 50, 40)
    _, s, s2 = build_sats(S, ctx, [f])
    rng = np.random.default_rng(0)
    t = rng.integers(0, 256, (10, 60)).astype(np.uint8)      # wider than the image
    tm = lib_templates(S, ctx, [t], [8])
    out = torch.zeros((1, 1, 3), dtype=torch.int32, device="cuda")
    with pytest.raises(S.SnccError) as e:
        S.sncc_topk(ctx, tm, s, s2, 1, 50, 40, [(0, 0)], 1, S.SNCC_FP32_KAHAN, out)
    assert e.value.code == S.SNCC_EINVAL
    with pytest.raises(ValueError):                            # frame index out of range
        S.sncc_topk(ctx, tm, s, s2, 1, 50, 40, [(1, 0)], 1, S.SNCC_FP32_KAHAN, out)
    p = np.array([[1, 0]], np.int32)                          # the C side checks it too
    assert S.lib.sncc_topk(ctx, tm, s.data_ptr(), s2.data_ptr(), 1, 50, 40, s.shape[-1], 1,
                           p.ctypes.data, 1, S.SNCC_FP32_KAHAN, out.data_ptr()) == S.SNCC_EINVAL
    halves = np.zeros(2, S.SEGMENT_DTYPE)                     # area above the exact bound
    halves[0] = (0, 0, 2048, 2049, 0, 2048 * 2049, 0)
    halves[1] = (2048, 0, 2048, 2049, 2048 * 2049 * 9, 2048 * 2049, 0)
    with pytest.raises(S.SnccError) as e:
        S.sncc_upload_templates(ctx, [halves], [4096], [2049])
    assert e.value.code == S.SNCC_ERANGE
    big = rng.integers(0, 256, (260, 260)).astype(np.uint8)
    segs, _, _ = S.sncc_segment_template(big, 40)
    bad = segs.copy()
    bad[0]["w"] += 1                                          # overlapping segments
    with pytest.raises(S.SnccError) as e:
        S.sncc_upload_templates(ctx, [bad[:5]], [260], [260])
    assert e.value.code in (S.SNCC_EINVAL, S.SNCC_ERANGE)
    small = rng.integers(0, 256, (12, 12)).astype(np.uint8)
    segs, _, _ = S.sncc_segment_template(small, 30)
    with pytest.raises(S.SnccError) as e:
        S.sncc_upload_templates(ctx, [segs[:-1]], [12], [12])  # hole
    assert e.value.code == S.SNCC_EINVAL
    flat = np.zeros(1, S.SEGMENT_DTYPE)
    flat[0] = (0, 0, 12, 12, 144 * 9, 144, 0)
    with pytest.raises(S.SnccError) as e:
        S.sncc_upload_templates(ctx, [flat], [12], [12])
    assert e.value.code == S.SNCC_EDEGENERATE
    with pytest.raises(S.SnccError):
        S.sncc_score(ctx, tm, 5, s, s2, 50, 40, S.SNCC_FP64,
                     torch.zeros((1, 1), dtype=torch.float64, device="cuda"))
