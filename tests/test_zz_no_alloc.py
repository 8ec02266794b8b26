"""The allocation-free sum-table entry point (static carry scratch) against
sncc_build_sats, bit for bit, called through the raw C-ABI: two calls in a
row, the second with fewer and smaller frames than the first (the static
array keeps the first call's carries), then a call that needs more carry
space than the array holds, which is refused before anything is launched."""

import ctypes as C

import numpy as np
import pytest

import oracle as O
from workloads import synth

pytestmark = pytest.mark.gpu


def _tables(torch, B, M, N, P, fill):
    return (torch.full((B, N + 1, P), fill, dtype=torch.int32, device="cuda"),
            torch.full((B, N + 1, P), fill, dtype=torch.int32, device="cuda"))


def test_noalloc_sum_tables_match_build_sats():
    import torch
    import paper_2502_01286_amd as S
    torch.cuda.init()
    ctx = S.sncc_ctx_create(0)
    try:
        for case, (B, M, N) in enumerate([(3, 700, 500), (1, 300, 200)]):
            print(f"noalloc case {case}: {B} frames {M}x{N}", flush=True)
            frames = [synth.scene(7700 + 10 * case + b, M, N) for b in range(B)]
            f = torch.from_numpy(np.stack(frames)).cuda()
            P = S.sncc_sat_pitch(M)
            words = 2 * B * (-(-N // 64) * M + N * -(-M // 256) + -(-N // 64) * -(-M // 256))
            assert 4 * words <= S.SNCC_NOALLOC_SCRATCH_BYTES
            s_ref, s2_ref = _tables(torch, B, M, N, P, 0)
            S.sncc_build_sats(ctx, f, s_ref, s2_ref)
            s_na, s2_na = _tables(torch, B, M, N, P, -1)     # garbage where nothing is written
            rc = S.lib.sncc_build_sats_noalloc(ctx, f.data_ptr(), B, M, N, M, s_na.data_ptr(),
                                               s2_na.data_ptr(), P)
            assert rc == S.SNCC_OK, S.sncc_last_error()
            S.sncc_sync(ctx)
            assert torch.equal(s_na, s_ref) and torch.equal(s2_na, s2_ref)
            # and the tables are Eqs. (10), (14) modulo 2^32
            so, s2o = O.sum_tables(frames[-1])
            got = s_na[-1].cpu().numpy().view(np.uint32)[:, :M + 1].astype(np.int64)
            got2 = s2_na[-1].cpu().numpy().view(np.uint32)[:, :M + 1].astype(np.int64)
            assert (got == so % 2 ** 32).all() and (got2 == s2o % 2 ** 32).all()
        # too many frames for the static array: refused, nothing written
        B, M, N = 7, 3840, 2160
        P = S.sncc_sat_pitch(M)
        f = torch.zeros((B, N, M), dtype=torch.uint8, device="cuda")
        s_big, s2_big = _tables(torch, B, M, N, P, 5)
        rc = S.lib.sncc_build_sats_noalloc(ctx, f.data_ptr(), B, M, N, M, s_big.data_ptr(),
                                           s2_big.data_ptr(), P)
        assert rc == S.SNCC_ENOSPC
        assert "static scratch" in S.sncc_last_error()
        S.sncc_sync(ctx)
        assert int(s_big[0, 1, 1]) == 5
        with pytest.raises(S.SnccError):
            S.sncc_build_sats_noalloc(ctx, f, s_big, s2_big)
    finally:
        S.sncc_ctx_destroy(ctx)
