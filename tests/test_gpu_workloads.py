"""Parity at the workloads' full sizes, in the launch configurations the
benchmark uses (MI355X).

Every single-frame workload is compared element by element over its whole
rho map with an oracle map computed in row bands by a process pool
(tests/oracle_pool.py).  The batched workloads compare the GPU's top-k lists
with whole oracle maps on stratified samples of pairs (every template of the
coarse-fine batch, the costliest, widest and tallest templates of the 16 x 64
batch) and re-score every reported match at its position; the coarse-fine
batch's final argmax is checked on every sampled pair (where the candidate
set is not unique, against the oracle's fine step over the GPU's own
candidates).  Inputs come from workloads.synth; no oracle input comes from
the GPU.
"""

import numpy as np
import pytest

import oracle as O
from oracle import select as OSEL
from workloads import synth

from gpu_util import build_sats, lib_templates, oracle_templates, topk_ok
from oracle_pool import OraclePool

pytestmark = pytest.mark.gpu

TOL32 = 1e-5
TOL64 = 1e-9
SET_GAP = 2e-5        # a rank-k / rank-k+1 gap above twice the FP32 tolerance fixes the set
ARGMAX_MARGIN = 1e-4  # argmax parity where the oracle's top-2 margin exceeds this


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


@pytest.fixture(scope="module")
def pool():
    p = OraclePool()
    yield p
    p.close()


def _maps(S, ctx, f, t, sigma, k_max=5000):
    """GPU FP32 and FP64 maps of one frame and template, plus the batched
    top-1 (sncc_argmax, FP32) of the pair."""
    import torch
    N, M = f.shape
    H, W = t.shape
    _, s, s2 = build_sats(S, ctx, [f])
    tm = lib_templates(S, ctx, [t], [sigma], k_max)
    nu, nv = M - W + 1, N - H + 1
    r32 = torch.empty((nv, nu), dtype=torch.float32, device="cuda")
    r64 = torch.empty((nv, nu), dtype=torch.float64, device="cuda")
    top1 = torch.zeros((1, 1, 3), dtype=torch.int32, device="cuda")
    S.sncc_score(ctx, tm, 0, s, s2, M, N, S.SNCC_FP32_KAHAN, r32)
    S.sncc_score(ctx, tm, 0, s, s2, M, N, S.SNCC_FP64, r64)
    S.sncc_argmax(ctx, tm, s, s2, 1, M, N, [(0, 0)], S.SNCC_FP32_KAHAN, top1)
    S.sncc_sync(ctx)
    S.sncc_tmpl_destroy(tm)
    best = S.decode_matches(top1)[0, 0]
    return r32.cpu().numpy().astype(np.float64), r64.cpu().numpy(), best


def _check_single(S, ctx, pool, wl, sigma, k_max=5000):
    f, t = wl.frames[0], wl.templates[0]
    g32, g64, best = _maps(S, ctx, f, t, sigma, k_max)
    ta = O.precompute_template_approximation(t, sigma, k_max)
    want = pool.maps([(f, ta)])[0]
    e32, e64 = np.abs(g32 - want).max(), np.abs(g64 - want).max()
    margin = O.top2_margin(want)
    u, v, r = O.argmax(want)
    print(f"  K {ta.K} (sigma used {ta.sigma_used}), {want.size} offsets: max|drho| "
          f"fp32 {e32:.2e} fp64 {e64:.2e}; oracle argmax ({u},{v}) rho {r:.6f}, top-2 margin "
          f"{margin:.2e}; GPU top-1 ({int(best['u'])},{int(best['v'])})", flush=True)
    assert e64 <= TOL64 and e32 <= TOL32
    assert abs(float(best["rho"]) - want[int(best["v"]), int(best["u"])]) <= TOL32
    assert float(best["rho"]) >= r - TOL32
    if margin > ARGMAX_MARGIN:
        assert (int(best["u"]), int(best["v"])) == (u, v)
        assert np.unravel_index(np.argmax(g32), g32.shape) == (v, u)
        assert np.unravel_index(np.argmax(g64), g64.shape) == (v, u)
    else:
        # several offsets are within the tolerance of the best: the GPU's choice is one of them
        assert want[np.unravel_index(np.argmax(g64), g64.shape)] >= r - TOL64
    return ta


def test_scene_640x480_full_map(S, ctx, pool):
    wl = synth.scene_640x480()
    print("single scene 640x480, 32x32 template, sigma 8", flush=True)
    _check_single(S, ctx, pool, wl, 8)


@pytest.mark.parametrize("sigma", [16, 8, 4])
def test_scene_1920x1080_full_map(S, ctx, pool, sigma):
    wl = synth.scene_1920x1080(sigma)
    print(f"single scene 1920x1080, 64x64 template, sigma {sigma}", flush=True)
    _check_single(S, ctx, pool, wl, sigma)


@pytest.mark.parametrize("size,k_max", [(128, 5000), (256, 5000), (128, 10 ** 9)])
def test_texture_3840x2160_full_map(S, ctx, pool, size, k_max):
    """The whole 3840 x 2160 map against the oracle's, thousands of segments
    per template (K_max 5000, and uncapped: the FP32 error-growth stress)."""
    wl = synth.texture_3840x2160(size, k_max=k_max)
    print(f"texture 3840x2160, {size}x{size} template, sigma 4, K_max {k_max}", flush=True)
    _check_single(S, ctx, pool, wl, 4, k_max)


def _batch(S, ctx, wl, fine=False, k=None):
    import torch
    B, N, M = len(wl.frames), wl.N, wl.M
    k = k or wl.k
    f = torch.from_numpy(np.stack(wl.frames)).cuda()
    P = S.sncc_sat_pitch(M)
    s = torch.empty((B, N + 1, P), dtype=torch.int32, device="cuda")
    s2 = torch.empty_like(s)
    coarse = lib_templates(S, ctx, wl.templates, wl.sigmas, wl.k_max)
    fn = lib_templates(S, ctx, wl.templates, [wl.fine_sigma] * len(wl.templates)) if fine else None
    n = len(wl.pairs)
    topk = torch.zeros((n, k, 3), dtype=torch.int32, device="cuda")
    best = torch.zeros((n, 4), dtype=torch.int32, device="cuda") if fine else None
    cnt = torch.zeros(n, dtype=torch.int32, device="cuda") if fine else None
    batch = S.sncc_batch_create(ctx, coarse, s, s2, B, M, N, wl.pairs, k, topk, fine=fn,
                                radius=2, best_out=best, count_out=cnt, frames=f, tune=1)
    batch.run()
    S.sncc_sync(ctx)
    out = (S.decode_matches(topk), S.decode_matches64(best) if fine else None,
           cnt.cpu().numpy() if fine else None)
    batch.destroy()
    S.sncc_tmpl_destroy(coarse)
    if fn:
        S.sncc_tmpl_destroy(fn)
    return out


def _set_check(cmap, got, k):
    """Where the oracle's rank-k / rank-k+1 gap exceeds SET_GAP the k best
    offsets are fixed, and the GPU's list must hold exactly those."""
    ref = O.topk(cmap, k + 1)
    gap = ref[k - 1][2] - ref[k][2] if len(ref) > k else np.inf
    if gap > SET_GAP:
        want = {(u, v) for u, v, _ in ref[:k]}
        have = {(int(a), int(b)) for a, b in zip(got["u"], got["v"])}
        assert have == want
        return True
    return False


def test_batch_16x64_top5(S, ctx, pool):
    wl = synth.batch_16x64()
    print("16 frames 1920x1080 x 64 templates, top-5", flush=True)
    got, _, _ = _batch(S, ctx, wl)
    tas = oracle_templates(wl.templates, wl.sigmas)
    tables = {}
    rng = np.random.default_rng(33)
    # every reported match of 256 random pairs re-scored by the oracle at its position
    worst = 0.0
    for p in rng.permutation(len(wl.pairs))[:256]:
        b, ti = wl.pairs[p]
        if b not in tables:
            tables[b] = O.sum_tables(wl.frames[b])
        g = got[p]
        want = O.rho_at(*tables[b], tas[ti], g["u"].astype(np.int64), g["v"].astype(np.int64))
        worst = max(worst, float(np.abs(want - g["rho"]).max()))
        assert (np.diff(g["rho"]) <= 0).all()
    print(f"  256 pairs re-scored: max|drho| {worst:.2e}", flush=True)
    assert worst <= TOL32
    # whole oracle maps: the costliest, widest and tallest templates and random ones,
    # each against a random frame
    K = np.array([ta.K for ta in tas])
    Ws = np.array([ta.W for ta in tas])
    Hs = np.array([ta.H for ta in tas])
    pick = list(np.argsort(-K)[:6]) + list(np.argsort(-Ws)[:3]) + list(np.argsort(-Hs)[:3])
    pick += list(rng.permutation(len(tas))[:6])
    pick = list(dict.fromkeys(int(i) for i in pick))
    sample = []
    for ti in pick:
        b = int(rng.integers(0, len(wl.frames)))
        sample.append(wl.pairs.index((b, ti)))
    maps = pool.maps([(wl.frames[wl.pairs[p][0]], tas[wl.pairs[p][1]]) for p in sample])
    n_sets = 0
    for p, m in zip(sample, maps):
        b, ti = wl.pairs[p]
        errs = topk_ok(m, got[p], 5, TOL32)
        assert not errs, (p, errs[:3])
        n_sets += _set_check(m, got[p], 5)
    print(f"  {len(sample)} pairs with whole oracle maps (K up to {K[pick].max()}, sides up to "
          f"{Ws[pick].max()}x{Hs[pick].max()}): top-5 ranks match; {n_sets} with a fixed "
          f"top-5 set, identical", flush=True)
    assert len(sample) >= 12


def _fine_step(tables, ta_f, cands, nu, nv, radius=2):
    """The oracle's fine step (Section 5, steps 7f-i) over a given candidate
    list: FP64 rho with the fine approximation on the union of the
    candidates' neighbourhoods, best by (rho desc, v, u)."""
    cu, cv = OSEL.neighbourhood(cands, radius, nu, nv)
    fr = O.rho_at(*tables, ta_f, cu, cv)
    order = np.lexsort((cu, cv, -fr))
    return cu, cv, fr, order


def test_coarse_fine_256x32(S, ctx, pool):
    wl = synth.coarse_fine_256x32()
    print("256 frames 1280x720 x 32 templates, top-32 + FP64 refine", flush=True)
    got, best, counts = _batch(S, ctx, wl, fine=True)
    tas_c = oracle_templates(wl.templates, wl.sigmas)
    tas_f = oracle_templates(wl.templates, [wl.fine_sigma] * len(wl.templates))
    rng = np.random.default_rng(44)
    # stratified sample: every template against three random frames
    sample = []
    for ti in range(len(wl.templates)):
        for b in rng.choice(len(wl.frames), 3, replace=False):
            sample.append(wl.pairs.index((int(b), ti)))
    maps = pool.maps([(wl.frames[wl.pairs[p][0]], tas_c[wl.pairs[p][1]]) for p in sample])
    tables = {}
    worst_c = worst_f = 0.0
    n_sets = n_final = n_exact = 0
    for p, cmap in zip(sample, maps):
        b, ti = wl.pairs[p]
        if b not in tables:
            tables[b] = O.sum_tables(wl.frames[b])
        g = got[p]
        errs = topk_ok(cmap, g, 32, TOL32)
        assert not errs, (p, errs[:3])
        worst_c = max(worst_c, float(np.abs(cmap[g["v"], g["u"]] - g["rho"]).max()))
        fixed = _set_check(cmap, g, 32)
        n_sets += fixed
        # final argmax: the oracle's fine step over the GPU's own candidates (equal to the
        # oracle's whole coarse-fine result where the candidate set is fixed)
        nv, nu = cmap.shape
        cands = [(int(u), int(v), 0.0) for u, v in zip(g["u"], g["v"]) if u >= 0]
        cu, cv, fr, order = _fine_step(tables[b], tas_f[ti], cands, nu, nv)
        assert counts[p] == len(cu)
        bu, bv, br = int(best[p]["u"]), int(best[p]["v"]), float(best[p]["rho"])
        i0 = order[0]
        margin = fr[i0] - fr[order[1]] if len(order) > 1 else np.inf
        worst_f = max(worst_f, abs(br - float(O.rho_at(*tables[b], tas_f[ti], bu, bv))))
        if margin > TOL64:
            assert (bu, bv) == (int(cu[i0]), int(cv[i0])), (p, (bu, bv), (cu[i0], cv[i0]))
            n_exact += 1
        else:
            assert br >= fr[i0] - TOL64
        assert abs(br - fr[i0]) <= TOL64
        if fixed:
            res = O.coarse_fine(*tables[b], tas_c[ti], tas_f[ti], wl.M, wl.N, k=32, radius=2,
                                coarse_map=cmap)
            assert abs(br - res["best"][2]) <= TOL64
            if margin > TOL64:
                assert (bu, bv) == res["best"][:2]
        n_final += 1
    print(f"  {len(sample)} pairs with whole oracle coarse maps: coarse max|drho| {worst_c:.2e}, "
          f"fine max|drho| {worst_f:.2e}; {n_sets} with a fixed top-32 set (identical); final "
          f"argmax checked on {n_final} ({n_exact} with a fine margin above 1e-9, exact)",
          flush=True)
    assert n_final == len(sample) == 3 * len(wl.templates)
    assert worst_c <= TOL32 and worst_f <= TOL64
