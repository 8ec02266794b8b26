"""Host split-and-merge of libsncc (C++) against the oracle, and the C-ABI's
argument checks that need no GPU.

The C++ segmentation must give the same rectangle lists, in the same order,
as the oracle's precompute_template_approximation (Section 5) on many seeded
templates; the deviation test of Eq. (2) must decide ties the same way.
"""

import ctypes as C
import os

import numpy as np
import pytest

import oracle as O
import paper_2502_01286_amd as S


def _oracle_list(t, sigma, k_max):
    ta = O.precompute_template_approximation(t, sigma, k_max)
    return [s.as_tuple() for s in ta.segments], ta.sigma_used, ta.rho_max


def _lib_list(t, sigma, k_max):
    segs, su, rm = S.sncc_segment_template(t, sigma, k_max)
    return [(int(s["x"]), int(s["y"]), int(s["w"]), int(s["h"]), int(s["sum"]), int(s["area"]))
            for s in segs], su, rm


def _random_template(rng):
    H, W = int(rng.integers(1, 17)), int(rng.integers(1, 17))
    kind = int(rng.integers(0, 4))
    if kind == 0:
        t = rng.integers(0, 256, (H, W))
    elif kind == 1:   # few levels: many exact-mean merges
        t = rng.integers(0, 3, (H, W)) * 100
    elif kind == 2:   # smooth ramp plus noise
        yy, xx = np.mgrid[0:H, 0:W]
        t = 8 * xx + 5 * yy + rng.integers(0, 4, (H, W))
    else:             # blocks
        t = np.kron(rng.integers(0, 256, (H // 2 + 1, W // 2 + 1)), np.ones((2, 2)))[:H, :W]
    return np.clip(t, 0, 255).astype(np.uint8)


N_TEMPLATES = int(os.environ.get("SNCC_P11_COUNT", "10000"))


def _oracle_case(args):
    t, sigma, k_max = args
    try:
        return _oracle_list(t, sigma, k_max)
    except ValueError:
        return None


def test_p11_host_segmentation_equals_oracle():
    from concurrent.futures import ProcessPoolExecutor
    rng = np.random.default_rng(11)
    cases = []
    for _ in range(N_TEMPLATES):
        t = _random_template(rng)
        sigma = float(rng.choice([0.5, 1, 2, 3, 4, 8, 12, 16, 2.75, 7.3]))
        k_max = int(rng.choice([5000, 5000, 20, 6]))
        cases.append((t, sigma, k_max))
    workers = max(1, min(8, len(os.sched_getaffinity(0))))
    with ProcessPoolExecutor(max_workers=workers) as ex:
        wants = list(ex.map(_oracle_case, cases, chunksize=64))
    compared = 0
    for i, ((t, sigma, k_max), want) in enumerate(zip(cases, wants)):
        if want is None:
            with pytest.raises(S.SnccError) as ei:
                S.sncc_segment_template(t, sigma, k_max)
            assert ei.value.code == S.SNCC_EDEGENERATE
            continue
        got = _lib_list(t, sigma, k_max)
        assert got[0] == want[0], (i, t.shape, sigma, k_max)
        assert got[1] == want[1]
        assert got[2] == pytest.approx(want[2], abs=1e-12)
        compared += 1
    assert compared > N_TEMPLATES // 2


@pytest.mark.parametrize("size,sigma", [((64, 64), 4), ((64, 64), 16), ((32, 48), 8),
                                        ((96, 40), 4)])
def test_host_segmentation_equals_oracle_on_workload_crops(size, sigma):
    from workloads import synth
    f = synth.scene(77, 400, 300)
    rng = np.random.default_rng(5)
    t, _, _ = synth.crop_template(rng, f, size[0], size[1], sigma_max=sigma)
    assert _lib_list(t, sigma, 5000)[0] == _oracle_list(t, sigma, 5000)[0]


def test_deviation_ties_decided_exactly():
    # left half 0/16 (population std exactly 8), right half flat 200
    t = np.array([[0, 16, 200, 200]], np.uint8)
    assert len(_lib_list(t, 8, 5000)[0]) == 3            # 8 is not below 8: split
    assert len(_lib_list(t, np.nextafter(8, 9), 5000)[0]) == 2
    # top block rows [0 2 4] (variance 8/3), bottom block flat: thresholds
    # around sqrt(8/3), including non-integers one ulp either side
    t = np.array([[0, 2, 4], [0, 2, 4], [100, 100, 100], [100, 100, 100]], np.uint8)
    std = float(np.sqrt(8 / 3))
    for sig in [std, np.nextafter(std, 0), np.nextafter(std, 10), 1.6329, 1.633]:
        assert _lib_list(t, sig, 5000)[0] == _oracle_list(t, sig, 5000)[0]
    assert len(_lib_list(t, 1.633, 5000)[0]) == 2
    assert len(_lib_list(t, 1.6329, 5000)[0]) == 3


def test_segment_errors():
    t = np.zeros((4, 4), np.uint8)
    with pytest.raises(S.SnccError) as e:
        S.sncc_segment_template(t, 4)
    assert e.value.code == S.SNCC_EDEGENERATE
    t = np.arange(16, dtype=np.uint8).reshape(4, 4) * 10
    with pytest.raises(S.SnccError) as e:
        S.sncc_segment_template(t, 4, K_max=0)
    assert e.value.code == S.SNCC_EINVAL
    # capacity too small reports the needed count
    segs = np.zeros(1, dtype=S.SEGMENT_DTYPE)
    K = C.c_int(0)
    rc = S.lib.sncc_segment_template(np.ascontiguousarray(t).ctypes.data, 4, 4, 4, 1.0, 5000,
                                     segs.ctypes.data, 1, C.byref(K), None, None)
    assert rc == S.SNCC_ENOSPC and K.value > 1
    rc = S.lib.sncc_segment_template(None, 4, 4, 4, 1.0, 5000, segs.ctypes.data, 1,
                                     C.byref(K), None, None)
    assert rc == S.SNCC_EINVAL
    rc = S.lib.sncc_segment_template(np.ascontiguousarray(t).ctypes.data, 4, 4, 3, 1.0, 5000,
                                     segs.ctypes.data, 1, C.byref(K), None, None)
    assert rc == S.SNCC_EINVAL


def test_kmax_loop_matches_oracle_sigma_used():
    rng = np.random.default_rng(3)
    yy, xx = np.mgrid[0:24, 0:24]
    t = np.clip(9 * xx + rng.integers(0, 40, (24, 24)), 0, 255).astype(np.uint8)
    for k_max in [4, 50, 200, 576]:
        got = _lib_list(t, 4, k_max)
        want = _oracle_list(t, 4, k_max)
        assert got[0] == want[0] and got[1] == want[1]


# ------------------------------------------------ batched preparation (host)
def _batch_cases(seed, n):
    rng = np.random.default_rng(seed)
    ts, sg = [], []
    for i in range(n):
        t = _random_template(rng) if i % 3 else \
            rng.integers(0, 256, (int(rng.integers(8, 65)), int(rng.integers(8, 65)))).astype(np.uint8)
        ts.append(t)
        sd = float(t.astype(np.float64).std())
        sg.append([0.99 * sd, 0.1 * sd, float(rng.choice([0, 4, 16, 60]))][i % 3])
    return ts, sg


@pytest.mark.parametrize("n_threads", [1, 4, 0])
def test_batched_preparation_equals_single_calls(n_threads):
    ts, sg = _batch_cases(21, 300)
    lists, su, rm, st = S.sncc_segment_templates(ts, sg, 5000, n_threads, check=False)
    for i, (t, s) in enumerate(zip(ts, sg)):
        try:
            one, su1, rm1 = S.sncc_segment_template(t, s, 5000)
        except S.SnccError as e:
            assert e.code == S.SNCC_EDEGENERATE and st[i] == S.SNCC_EDEGENERATE
            continue
        assert st[i] == S.SNCC_OK
        assert (lists[i] == one).all() and len(lists[i]) == len(one)
        assert su[i] == su1 and rm[i] == rm1


def test_batched_preparation_equals_oracle():
    ts, sg = _batch_cases(22, 120)
    lists, su, rm, st = S.sncc_segment_templates(ts, sg, 200, 0, check=False)
    for i, (t, s) in enumerate(zip(ts, sg)):
        try:
            want, wsu, wrm = _oracle_list(t, s, 200)
        except ValueError:
            assert st[i] == S.SNCC_EDEGENERATE
            continue
        got = [(int(g["x"]), int(g["y"]), int(g["w"]), int(g["h"]), int(g["sum"]),
                int(g["area"])) for g in lists[i]]
        assert got == want and su[i] == wsu
        assert rm[i] == pytest.approx(wrm, abs=1e-12)


def test_batched_preparation_degenerate_and_capacity():
    rng = np.random.default_rng(23)
    ts = [rng.integers(0, 256, (9, 7)).astype(np.uint8), np.full((5, 6), 17, np.uint8),
          rng.integers(0, 256, (4, 12)).astype(np.uint8)]
    sg = [10.0, 3.0, 10.0]
    with pytest.raises(S.SnccError) as e:
        S.sncc_segment_templates(ts, sg)
    assert e.value.code == S.SNCC_EDEGENERATE and "template 1" in str(e.value)
    lists, su, rm, st = S.sncc_segment_templates(ts, sg, check=False)
    assert list(st) == [S.SNCC_OK, S.SNCC_EDEGENERATE, S.SNCC_OK]
    assert np.isnan(rm[1]) and len(lists[1]) == 1
    for i in (0, 2):
        one, _, _ = S.sncc_segment_template(ts[i], sg[i])
        assert (lists[i] == one).all()
    # capacity: offsets are filled, nothing is written
    W = np.array([t.shape[1] for t in ts], np.int32)
    H = np.array([t.shape[0] for t in ts], np.int32)
    ptrs = (C.c_void_p * 3)(*[t.ctypes.data for t in ts])
    sgs = np.array(sg)
    out = np.zeros(2, dtype=S.SEGMENT_DTYPE)
    off = np.zeros(4, np.int64)
    rc = S.lib.sncc_segment_templates(3, ptrs, W.ctypes.data, H.ctypes.data, W.ctypes.data,
                                      sgs.ctypes.data, 5000, 2, out.ctypes.data, 2,
                                      off.ctypes.data, None, None, None)
    assert rc == S.SNCC_ENOSPC and off[3] > 2 and (out["area"] == 0).all()
