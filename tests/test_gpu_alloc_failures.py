"""Device allocation failures are reported, not fatal.  With
SNCC_TEST_FAIL_ALLOC=1 in the environment every device allocation the
library makes is refused as if the device were out of memory (a test hook
read at each allocation; no kernel runs on memory that was not obtained):
each entry point that needs new device memory returns SNCC_ENOMEM with a
message, the ones that need none still work, and once the variable is
cleared the same context gives the oracle's results."""

import numpy as np
import pytest

import oracle as O
from workloads import synth

from gpu_util import topk_ok

pytestmark = pytest.mark.gpu


def test_allocation_failures(monkeypatch):
    import torch
    import paper_2502_01286_amd as S
    torch.cuda.init()
    M, N, W, H = 160, 120, 24, 20
    frames = [synth.scene(9900 + b, M, N) for b in range(2)]
    rng = np.random.default_rng(99)
    t, _, _ = synth.crop_template(rng, frames[1], W, H, sigma_max=8)
    segs, _, _ = S.sncc_segment_template(t, 8)          # host only
    segf, _, _ = S.sncc_segment_template(t, 2)
    f = torch.from_numpy(np.stack(frames)).cuda()
    P = S.sncc_sat_pitch(M)
    s = torch.zeros((2, N + 1, P), dtype=torch.int32, device="cuda")
    s2 = torch.zeros_like(s)
    nu, nv = M - W + 1, N - H + 1
    rho = torch.zeros((nv, nu), dtype=torch.float32, device="cuda")
    rho64 = torch.zeros((nv, nu), dtype=torch.float64, device="cuda")
    top = torch.zeros((2, 4, 3), dtype=torch.int32, device="cuda")
    pairs = [(0, 0), (1, 0)]
    ctx = S.sncc_ctx_create(0)              # fresh: none of its scratch is allocated yet
    try:
        def refused(fn, *a, **kw):
            with pytest.raises(S.SnccError) as e:
                fn(*a, **kw)
            assert e.value.code == S.SNCC_ENOMEM, e.value
            assert "SNCC_TEST_FAIL_ALLOC" in str(e.value)

        monkeypatch.setenv("SNCC_TEST_FAIL_ALLOC", "1")
        refused(S.sncc_upload_templates, ctx, [segs], [W], [H])
        monkeypatch.delenv("SNCC_TEST_FAIL_ALLOC")
        tm = S.sncc_upload_templates(ctx, [segs], [W], [H])
        fine = S.sncc_upload_templates(ctx, [segf], [W], [H])

        monkeypatch.setenv("SNCC_TEST_FAIL_ALLOC", "1")
        refused(S.sncc_build_sats, ctx, f, s, s2)
        monkeypatch.delenv("SNCC_TEST_FAIL_ALLOC")
        S.sncc_build_sats(ctx, f, s, s2)

        monkeypatch.setenv("SNCC_TEST_FAIL_ALLOC", "1")
        refused(S.sncc_topk, ctx, tm, s, s2, 2, M, N, pairs, 4, S.SNCC_FP32_KAHAN, top)
        refused(S.sncc_topk, ctx, tm, s, s2, 2, M, N, pairs, 4, S.SNCC_FP64, top)
        refused(S.sncc_score, ctx, tm, 0, s[1], s2[1], M, N, S.SNCC_FP32_KAHAN, rho)
        refused(S.sncc_score_frame, ctx, tm, 0, f[1], rho, form=S.SNCC_FORM_GLOBAL)
        refused(S.sncc_batch_create, ctx, tm, s, s2, 2, M, N, pairs, 4, top, frames=f)
        cand = torch.zeros((1024, 6), dtype=torch.int32, device="cuda")
        out = torch.zeros((1024, 6), dtype=torch.int32, device="cuda")
        counts = torch.zeros(2, dtype=torch.int32, device="cuda")
        refused(S.sncc_threshold_match, ctx, tm, fine, [0.5], [0.5], s, s2, 2, M, N, pairs,
                cand, out, counts)
        # calls that need no new device memory still run
        S.sncc_score(ctx, tm, 0, s[1], s2[1], M, N, S.SNCC_FP64, rho64)
        assert S.sncc_score_frame(ctx, tm, 0, f[1], rho,
                                  form=S.SNCC_FORM_TILE_LOCAL) == S.SNCC_FORM_TILE_LOCAL
        S.sncc_sync(ctx)
        monkeypatch.delenv("SNCC_TEST_FAIL_ALLOC")

        ta = O.precompute_template_approximation(t, 8)
        want = O.rho_map(frames[1], ta)
        assert np.abs(rho64.cpu().numpy() - want).max() <= 1e-9
        assert np.abs(rho.cpu().numpy() - want).max() <= 1e-5
        # the same context, allocations allowed again
        S.sncc_topk(ctx, tm, s, s2, 2, M, N, pairs, 4, S.SNCC_FP32_KAHAN, top)
        S.sncc_score(ctx, tm, 0, s[1], s2[1], M, N, S.SNCC_FP32_KAHAN, rho)
        S.sncc_sync(ctx)
        got = S.decode_matches(top)
        for p, (b, _) in enumerate(pairs):
            assert not topk_ok(O.rho_map(frames[b], ta), got[p], 4, 1e-5)
        assert np.abs(rho.cpu().numpy() - want).max() <= 1e-5
        S.sncc_tmpl_destroy(tm)
        S.sncc_tmpl_destroy(fine)
    finally:
        S.sncc_ctx_destroy(ctx)
