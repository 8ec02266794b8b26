"""The binding rejects tensors of the wrong shape, size, dtype or layout
before anything reaches the C-ABI (which sees raw pointers only), so a caller's
slip raises in Python instead of writing out of bounds on the device.  The
size checks run before the device check, so they are exercised here on CPU
tensors; no GPU call is made."""

import pytest
import torch

import paper_2502_01286_amd as S


def _i32(*shape):
    return torch.zeros(shape, dtype=torch.int32)


def test_tables_must_match_each_other_and_the_frames():
    f = torch.zeros((2, 10, 20), dtype=torch.uint8)
    with pytest.raises(ValueError, match="differ in shape"):
        S.sncc_build_sats(None, f, _i32(2, 11, 64), _i32(2, 11, 128))
    with pytest.raises(ValueError, match="frames"):
        S.sncc_build_sats(None, f, _i32(3, 11, 64), _i32(3, 11, 64))
    with pytest.raises(ValueError, match="N \\+ 1"):
        S.sncc_build_sats(None, f, _i32(2, 10, 64), _i32(2, 10, 64))
    with pytest.raises(TypeError, match="int32"):
        S.sncc_build_sats(None, f, torch.zeros((2, 11, 64)), torch.zeros((2, 11, 64)))
    with pytest.raises(ValueError, match="contiguous"):
        S.sncc_build_sats(None, f, _i32(2, 64, 11).transpose(1, 2), _i32(2, 64, 11).transpose(1, 2))
    # right sizes, host memory: only then is the device checked
    with pytest.raises(ValueError, match="device tensor"):
        S.sncc_build_sats(None, f, _i32(2, 11, 64), _i32(2, 11, 64))


def test_tables_hold_every_frame():
    # one 2-D table passed for a batch of three frames
    with pytest.raises(ValueError, match="elements"):
        S.sncc_topk(None, None, _i32(11, 64), _i32(11, 64), 3, 20, 10, [(0, 0)], 5, 0,
                    _i32(1, 5, 3))


def test_topk_output_shape():
    s = _i32(2, 11, 64)
    with pytest.raises(ValueError, match="shape \\(2, 5, 3\\)"):
        S.sncc_topk(None, None, s, s, 2, 20, 10, [(0, 0), (1, 0)], 5, 0, _i32(2, 4, 3))
    with pytest.raises(ValueError, match="shape"):
        S.sncc_topk(None, None, s, s, 2, 20, 10, [(0, 0), (1, 0)], 5, 0, _i32(1, 5, 3))
    with pytest.raises(ValueError, match="shape"):
        S.sncc_argmax(None, None, s, s, 2, 20, 10, [(0, 0)], 0, _i32(2, 3))


def test_refine_buffer_shapes():
    s = _i32(2, 11, 64)
    pairs = [(0, 0), (1, 0)]
    with pytest.raises(ValueError, match="cand"):
        S.sncc_refine(None, None, s, s, 2, 20, 10, pairs, _i32(2, 4), 2, _i32(2, 4))
    with pytest.raises(ValueError, match="cand must have shape"):
        S.sncc_refine(None, None, s, s, 2, 20, 10, pairs, _i32(3, 4, 3), 2, _i32(2, 4))
    with pytest.raises(ValueError, match="out must have shape"):
        S.sncc_refine(None, None, s, s, 2, 20, 10, pairs, _i32(2, 4, 3), 2, _i32(2, 3))
    with pytest.raises(ValueError, match="count must have shape"):
        S.sncc_refine(None, None, s, s, 2, 20, 10, pairs, _i32(2, 4, 3), 2, _i32(2, 4),
                      count=_i32(1))


def test_threshold_buffers():
    s = _i32(1, 11, 64)
    with pytest.raises(ValueError, match="cand must be"):
        S.sncc_threshold_match(None, None, None, [0.5], [0.5], s, s, 1, 20, 10, [(0, 0)],
                               _i32(8, 5), _i32(8, 6), _i32(2))
    with pytest.raises(ValueError, match="counts holds 1"):
        S.sncc_threshold_match(None, None, None, [0.5], [0.5], s, s, 1, 20, 10, [(0, 0)],
                               _i32(8, 6), _i32(8, 6), _i32(1))


def test_batch_buffers():
    s = _i32(2, 11, 64)
    pairs = [(0, 0), (1, 0)]
    with pytest.raises(ValueError, match="topk_out must have shape"):
        S.sncc_batch_create(None, None, s, s, 2, 20, 10, pairs, 4, _i32(2, 5, 3))
    with pytest.raises(ValueError, match="best_out"):
        S.sncc_batch_create(None, None, s, s, 2, 20, 10, pairs, 4, _i32(2, 4, 3),
                            fine=object())
    with pytest.raises(ValueError, match="frames must have shape"):
        S.sncc_batch_create(None, None, s, s, 2, 20, 10, pairs, 4, _i32(2, 4, 3),
                            frames=torch.zeros((2, 10, 21), dtype=torch.uint8))


def test_pair_indices_checked_against_frames():
    import numpy as np
    from paper_2502_01286_amd._native import _check_pairs
    with pytest.raises(ValueError, match="frame index"):
        _check_pairs(np.array([[2, 0]], np.int32), 2)
    with pytest.raises(ValueError, match="template index"):
        _check_pairs(np.array([[0, 3]], np.int32), 2, 3)
    _check_pairs(np.array([[1, 2]], np.int32), 2, 3)
    # a few pairs and many pairs take different code paths; a bad index in
    # the last row, negative or past the end, is found by both
    for n in (3, 8, 9, 100):
        ok = np.zeros((n, 2), np.int32)
        _check_pairs(ok, 1, 1)
        for col, bad, what in ((0, -1, "frame"), (0, 1, "frame"), (1, -1, "template"),
                               (1, 1, "template")):
            p = ok.copy()
            p[-1, col] = bad
            with pytest.raises(ValueError, match=f"{what} index"):
                _check_pairs(p, 1, 1)
    _check_pairs(np.zeros((0, 2), np.int32), 1, 1)


def test_tmpl_count_rejects_null():
    with pytest.raises(S.SnccError):
        S.sncc_tmpl_count(None)
