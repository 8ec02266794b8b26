"""The paper's two-threshold search (Section 5, steps 5 and 7a-j) on the HIP
path against the oracle's ``threshold_match`` (MI355X).

The fast test is taken on the FP32-compensated rho (error <= 1e-5) and the
slow rho in FP64 (<= 1e-9), so survivor and match sets are compared where the
decision is unambiguous: an offset whose oracle fast rho lies within 1e-5 of
the fast threshold, or whose slow rho lies within 1e-9 of the slow threshold,
may fall on either side.  Every reported value is checked against the oracle
at its offset, and every planted copy of a template must be reported.
"""

import numpy as np
import pytest

import oracle as O
from workloads import synth

from gpu_util import build_sats

pytestmark = pytest.mark.gpu

TOL32 = 1e-5
TOL64 = 1e-9
PRECISION = 0.9


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


def _prepare(S, ctx, templates):
    """Both approximations of every template through the library (host C++),
    with the paper's relative thresholds; returns the device sets and the
    per-template thresholds."""
    fast_l, slow_l, tf, ts, W, H = [], [], [], [], [], []
    for t in templates:
        sf, ss = O.paper_sigmas(t)
        a, _, rf = S.sncc_segment_template(t, sf)
        b, _, rs = S.sncc_segment_template(t, ss)
        fast_l.append(a)
        slow_l.append(b)
        tf.append(PRECISION * rf)
        ts.append(PRECISION * rs)
        H.append(t.shape[0])
        W.append(t.shape[1])
    return (S.sncc_upload_templates(ctx, fast_l, W, H), S.sncc_upload_templates(ctx, slow_l, W, H),
            np.array(tf), np.array(ts))


def _run(S, ctx, frames, templates, pairs, cand_cap=1 << 16, out_cap=1 << 16, thr=None):
    import torch
    f, s, s2 = build_sats(S, ctx, frames)
    B, N, M = f.shape
    fast, slow, tf, ts = _prepare(S, ctx, templates)
    if thr is not None:
        tf, ts = thr
    cand = torch.full((cand_cap, 6), -7, dtype=torch.int32, device="cuda")
    out = torch.full((out_cap, 6), -7, dtype=torch.int32, device="cuda")
    counts = torch.zeros(4, dtype=torch.int32, device="cuda")
    S.sncc_threshold_match(ctx, fast, slow, tf, ts, s, s2, B, M, N, pairs, cand, out, counts)
    S.sncc_sync(ctx)
    nc, nm = (int(x) for x in counts[:2].cpu())
    res = dict(cand=S.decode_hits(cand, nc), out=S.decode_hits(out, nm), n_cand=nc, n_out=nm,
               cand_raw=cand.cpu().numpy(), out_raw=out.cpu().numpy(), tf=tf, ts=ts)
    S.sncc_tmpl_destroy(fast)
    S.sncc_tmpl_destroy(slow)
    return res


def _oracle_pair(frame, t, tables=None):
    sf, ss = O.paper_sigmas(t)
    fa = O.precompute_template_approximation(t, sf)
    sl = O.precompute_template_approximation(t, ss)
    N, M = frame.shape
    s, s2 = tables if tables is not None else O.sum_tables(frame)
    fmap = O.rho_map(frame, fa, tables=(s, s2))
    res = O.threshold_match(s, s2, fa, sl, M, N, precision=PRECISION, fast_map=fmap)
    return res, fa, sl, fmap, (s, s2)


def _compare_pair(got_c, got_m, res, sl, fmap, tables):
    """GPU survivors/matches of one pair against the oracle's."""
    s, s2 = tables
    tf, ts = res["thr_fast"], res["thr_slow"]
    cu, cv = got_c["u"].astype(np.int64), got_c["v"].astype(np.int64)
    # every GPU survivor: its fast rho agrees, and it clears the threshold
    want = fmap[cv, cu]
    assert np.abs(got_c["rho"] - want).max(initial=0) <= TOL32
    assert (want >= tf - TOL32).all()
    gset = set(zip(cu.tolist(), cv.tolist()))
    assert len(gset) == len(got_c), "a survivor reported twice"
    # every clear oracle survivor is reported
    vv, uu = np.nonzero(fmap >= tf + TOL32)
    missing = [(u, v) for u, v in zip(uu.tolist(), vv.tolist()) if (u, v) not in gset]
    assert not missing, ("missing survivors", missing[:5], len(missing))
    # matches: slow rho in FP64 at the offset, threshold respected
    mu, mv = got_m["u"].astype(np.int64), got_m["v"].astype(np.int64)
    mset = set(zip(mu.tolist(), mv.tolist()))
    assert len(mset) == len(got_m), "a match reported twice"
    assert mset <= gset
    if len(got_m):
        want = O.rho_at(s, s2, sl, mu, mv)
        assert np.abs(got_m["rho"] - want).max() <= TOL64
        assert (want >= ts - TOL64).all()
    miss = [(u, v) for (u, v, r) in res["matches"]
            if fmap[v, u] >= tf + TOL32 and r >= ts + TOL64 and (u, v) not in mset]
    assert not miss, ("missing matches", miss[:5], len(miss))
    return len(gset), len(mset)


def _split(hits, n_pairs):
    return [hits[hits["pair"] == p] for p in range(n_pairs)]


def test_small_batch_against_oracle(S, ctx):
    rng = np.random.default_rng(77)
    frames = [synth.scene(7000 + i, 200, 150) for i in range(3)]
    templates, planted = [], []
    for j, (w, h) in enumerate([(24, 20), (37, 29), (16, 40)]):
        fi = j % 3
        t, x, y = synth.crop_template(rng, frames[fi], w, h, sigma_max=10)
        templates.append(t)
        # an exact copy of the template in another frame
        fo = (fi + 1) % 3
        px, py = int(rng.integers(0, 200 - w + 1)), int(rng.integers(0, 150 - h + 1))
        frames[fo][py:py + h, px:px + w] = t
        planted.append((fo, j, px, py))
    pairs = [(b, j) for b in range(3) for j in range(3)]
    print("3 frames 200x150 x 3 templates, relative thresholds", flush=True)
    got = _run(S, ctx, frames, templates, pairs)
    cands, outs = _split(got["cand"], len(pairs)), _split(got["out"], len(pairs))
    tables = {}
    tot_c = tot_m = 0
    for p, (b, j) in enumerate(pairs):
        if b not in tables:
            tables[b] = O.sum_tables(frames[b])
        res, fa, sl, fmap, tb = _oracle_pair(frames[b], templates[j], tables[b])
        assert got["tf"][j] == pytest.approx(res["thr_fast"], abs=1e-12)
        assert got["ts"][j] == pytest.approx(res["thr_slow"], abs=1e-12)
        nc, nm = _compare_pair(cands[p], outs[p], res, sl, fmap, tb)
        tot_c += nc
        tot_m += nm
    print(f"  {tot_c} survivors, {tot_m} matches", flush=True)
    assert got["n_cand"] == tot_c and got["n_out"] == tot_m
    for fo, j, px, py in planted:
        p = pairs.index((fo, j))
        assert any(int(h["u"]) == px and int(h["v"]) == py for h in outs[p]), (fo, j)


def test_staged_and_global_slow_forms_together(S, ctx):
    """A small template (its runs' regions fit LDS: staged slow pass) and a
    large one (110 x 100: scored from the global tables) in one call."""
    rng = np.random.default_rng(91)
    frames = [synth.scene(7600 + i, 320, 240) for i in range(2)]
    templates = []
    for j, (w, h) in enumerate([(24, 20), (110, 100)]):
        t, _, _ = synth.crop_template(rng, frames[j], w, h, sigma_max=10)
        templates.append(t)
        px, py = int(rng.integers(0, 320 - w + 1)), int(rng.integers(0, 240 - h + 1))
        frames[1 - j][py:py + h, px:px + w] = t
    pairs = [(b, j) for b in range(2) for j in range(2)]
    print("2 frames 320x240 x templates 24x20, 110x100", flush=True)
    got = _run(S, ctx, frames, templates, pairs, cand_cap=1 << 17, out_cap=1 << 17)
    cands, outs = _split(got["cand"], len(pairs)), _split(got["out"], len(pairs))
    tot_m = 0
    for p, (b, j) in enumerate(pairs):
        res, fa, sl, fmap, tb = _oracle_pair(frames[b], templates[j])
        _, nm = _compare_pair(cands[p], outs[p], res, sl, fmap, tb)
        tot_m += nm
    assert tot_m > 0 and got["n_out"] == tot_m


def test_wide_frames_row_relative_regions(S, ctx):
    """8300-wide frames: the 64-tall template's run regions are made
    row-relative before scoring (255 H P >= 2^27), the 20-tall template's are
    not; both against the oracle, with a planted copy of each."""
    rng = np.random.default_rng(93)
    M, N = 8300, 80
    frames = [synth.scene(7700 + i, M, N) for i in range(2)]
    templates = []
    for j, (w, h) in enumerate([(24, 64), (24, 20)]):
        t, _, _ = synth.crop_template(rng, frames[j], w, h, sigma_max=10)
        templates.append(t)
        px, py = int(rng.integers(0, M - w + 1)), int(rng.integers(0, N - h + 1))
        frames[1 - j][py:py + h, px:px + w] = t
    pairs = [(b, j) for b in range(2) for j in range(2)]
    print("2 frames 8300x80 x templates 24x64, 24x20", flush=True)
    got = _run(S, ctx, frames, templates, pairs, cand_cap=1 << 18, out_cap=1 << 18)
    cands, outs = _split(got["cand"], len(pairs)), _split(got["out"], len(pairs))
    tot_m = 0
    for p, (b, j) in enumerate(pairs):
        res, fa, sl, fmap, tb = _oracle_pair(frames[b], templates[j])
        _, nm = _compare_pair(cands[p], outs[p], res, sl, fmap, tb)
        tot_m += nm
    assert tot_m > 0 and got["n_out"] == tot_m


def test_capacity_overflow_counts_and_truncates(S, ctx):
    frames = [synth.scene(7100, 160, 120)]
    rng = np.random.default_rng(5)
    t, _, _ = synth.crop_template(rng, frames[0], 20, 18, sigma_max=10)
    full = _run(S, ctx, frames, [t], [(0, 0)], thr=(np.array([-2.0]), np.array([-2.0])))
    n = (160 - 20 + 1) * (120 - 18 + 1)
    assert full["n_cand"] == n and full["n_out"] == n     # every offset survives
    small = _run(S, ctx, frames, [t], [(0, 0)], cand_cap=5, out_cap=3,
                 thr=(np.array([-2.0]), np.array([-2.0])))
    assert small["n_cand"] == n                           # wanted, not written
    assert small["n_out"] == 5                            # the slow pass saw 5
    assert len(small["cand"]) == 5 and len(small["out"]) == 3
    assert (small["cand_raw"][5:] == -7).all() and (small["out_raw"][3:] == -7).all()


def test_no_survivors(S, ctx):
    frames = [synth.scene(7200, 128, 96)]
    rng = np.random.default_rng(6)
    t, _, _ = synth.crop_template(rng, frames[0], 17, 23, sigma_max=10)
    got = _run(S, ctx, frames, [t], [(0, 0)], thr=(np.array([1.5]), np.array([0.0])))
    assert got["n_cand"] == 0 and got["n_out"] == 0
    assert (got["cand_raw"] == -7).all() and (got["out_raw"] == -7).all()


def test_scene_1920x1080_paper_thresholds(S, ctx):
    """One 1920x1080 scene and its 64x64 template: the whole fast map from the
    oracle (the fast approximation has few segments), the slow rho at every
    survivor the oracle finds."""
    wl = synth.scene_1920x1080()
    f, t = wl.frames[0], wl.templates[0]
    _, x0, y0 = wl.origin[0]
    print("scene 1920x1080, 64x64 template, paper thresholds", flush=True)
    n_off = (f.shape[1] - t.shape[1] + 1) * (f.shape[0] - t.shape[0] + 1)
    got = _run(S, ctx, [f], [t], [(0, 0)], cand_cap=n_off, out_cap=n_off)
    res, fa, sl, fmap, tb = _oracle_pair(f, t)
    print(f"  K fast {fa.K}, K slow {sl.K}; GPU {got['n_cand']} survivors, {got['n_out']} "
          f"matches; oracle {len(res['cand_u'])} / {len(res['matches'])}", flush=True)
    _compare_pair(got["cand"], got["out"], res, sl, fmap, tb)
    # the crop origin is found when the noisy crop still clears both tests
    if fmap[y0, x0] >= res["thr_fast"] + TOL32:
        r = float(O.rho_at(*tb, sl, x0, y0))
        if r >= res["thr_slow"] + TOL64:
            assert any(int(h["u"]) == x0 and int(h["v"]) == y0 for h in got["out"])


def test_repeated_calls_match_fresh_contexts(S, ctx):
    """A context keeps the plan of its last threshold search and reuses it
    when the call repeats; a change of either threshold, of the pair list or
    of the tables must give what a fresh context gives."""
    import torch
    rng = np.random.default_rng(31)
    frames = [synth.scene(7400 + i, 180, 140) for i in range(2)]
    templates = [synth.crop_template(rng, frames[j], w, h, sigma_max=10)[0]
                 for j, (w, h) in enumerate([(21, 17), (30, 26)])]
    _, s, s2 = build_sats(S, ctx, frames)
    _, r, r2 = build_sats(S, ctx, [synth.scene(7500 + i, 180, 140) for i in range(2)])
    fast, slow, tf, ts = _prepare(S, ctx, templates)
    pairs = [(b, j) for b in range(2) for j in range(2)]
    cap = 2 * 180 * 140

    def run(c, tabs, pr, a, b):
        cand = torch.zeros((cap, 6), dtype=torch.int32, device="cuda")
        out = torch.zeros((cap, 6), dtype=torch.int32, device="cuda")
        counts = torch.zeros(4, dtype=torch.int32, device="cuda")
        S.sncc_threshold_match(c, fast, slow, a, b, tabs[0], tabs[1], 2, 180, 140, pr, cand, out,
                               counts)
        S.sncc_sync(c)
        nc, nm = (int(x) for x in counts[:2].cpu())
        key = lambda h: np.sort(h, order=["pair", "v", "u"])  # noqa: E731
        return nc, nm, key(S.decode_hits(cand, nc)), key(S.decode_hits(out, nm))

    lo = tf - 0.3
    calls = [((s, s2), pairs, tf, ts), ((s, s2), pairs, tf, ts), ((r, r2), pairs, tf, ts),
             ((r, r2), pairs, lo, ts), ((r, r2), pairs, lo, ts - 0.2),
             ((r, r2), pairs[::-1], lo, ts - 0.2), ((s, s2), pairs, tf, ts)]
    got = [run(ctx, *c) for c in calls]
    for i, (c, g) in enumerate(zip(calls, got)):
        fresh = S.sncc_ctx_create(0)
        try:
            want = run(fresh, *c)
        finally:
            S.sncc_ctx_destroy(fresh)
        assert g[:2] == want[:2], (i, g[:2], want[:2])
        for a, b in ((g[2], want[2]), (g[3], want[3])):
            for f in ("pair", "u", "v"):
                assert np.array_equal(a[f], b[f]), (i, f)
            # the slow pass may sum a survivor in either of its two orders
            assert np.abs(a["rho"] - b["rho"]).max(initial=0) <= 1e-12, i
    assert got[0][:2] == got[1][:2] == got[-1][:2]
    assert got[3][0] > got[2][0] and got[4][1] > got[3][1]
    S.sncc_tmpl_destroy(fast)
    S.sncc_tmpl_destroy(slow)


def test_errors(S, ctx):
    import torch
    frames = [synth.scene(7300, 64, 48)]
    _, s, s2 = build_sats(S, ctx, frames)
    rng = np.random.default_rng(8)
    t, _, _ = synth.crop_template(rng, frames[0], 12, 10, sigma_max=10)
    t2, _, _ = synth.crop_template(rng, frames[0], 11, 10, sigma_max=10)
    fast, slow, tf, ts = _prepare(S, ctx, [t])
    other, _, _, _ = _prepare(S, ctx, [t2])
    cand = torch.zeros((16, 6), dtype=torch.int32, device="cuda")
    out = torch.zeros((16, 6), dtype=torch.int32, device="cuda")
    counts = torch.zeros(4, dtype=torch.int32, device="cuda")
    with pytest.raises(S.SnccError):      # sizes differ between the sets
        S.sncc_threshold_match(ctx, fast, other, tf, ts, s, s2, 1, 64, 48, [(0, 0)], cand, out,
                               counts)
    with pytest.raises(S.SnccError):      # threshold not finite
        S.sncc_threshold_match(ctx, fast, slow, [np.nan], ts, s, s2, 1, 64, 48, [(0, 0)], cand,
                               out, counts)
    with pytest.raises(ValueError):       # pair out of range (binding)
        S.sncc_threshold_match(ctx, fast, slow, tf, ts, s, s2, 1, 64, 48, [(1, 0)], cand, out,
                               counts)
    p = np.array([[1, 0]], np.int32)      # and the C side
    tfa, tsa = np.asarray(tf, np.float64), np.asarray(ts, np.float64)
    assert S.lib.sncc_threshold_match(ctx, fast, slow, tfa.ctypes.data, tsa.ctypes.data,
                                      s.data_ptr(), s2.data_ptr(), 1, 64, 48, s.shape[-1], 1,
                                      p.ctypes.data, cand.data_ptr(), 16, out.data_ptr(), 16,
                                      counts.data_ptr()) == S.SNCC_EINVAL
    for h in (fast, slow, other):
        S.sncc_tmpl_destroy(h)


def test_stage_timing(S, ctx):
    import torch
    frames = [synth.scene(7400, 256, 192)]
    rng = np.random.default_rng(9)
    t, _, _ = synth.crop_template(rng, frames[0], 30, 26, sigma_max=10)
    _, s, s2 = build_sats(S, ctx, frames)
    fast, slow, tf, ts = _prepare(S, ctx, [t])
    cand = torch.zeros((1 << 15, 6), dtype=torch.int32, device="cuda")
    out = torch.zeros((1 << 15, 6), dtype=torch.int32, device="cuda")
    counts = torch.zeros(4, dtype=torch.int32, device="cuda")
    S.sncc_ctx_set_timing(ctx, True)
    try:
        S.sncc_threshold_match(ctx, fast, slow, tf, ts, s, s2, 1, 256, 192, [(0, 0)], cand, out,
                               counts)
        ms = S.sncc_ctx_stage_ms(ctx)
        assert len(ms) == 2 and all(m > 0 for m in ms)
    finally:
        S.sncc_ctx_set_timing(ctx, False)
    assert S.sncc_ctx_stage_ms(ctx) == []
    S.sncc_tmpl_destroy(fast)
    S.sncc_tmpl_destroy(slow)
