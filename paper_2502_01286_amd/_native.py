"""ctypes binding of libsncc.so (include/sncc.h).

Argument marshalling only: every function keeps the C name, checks that
tensors are on the right device with the right dtype and layout, passes raw
pointers and sizes, and raises ``SnccError`` on a negative status.  All device
work happens in the library's HIP kernels.  Importing this module fails loudly
when the library has not been built.
"""

from __future__ import annotations

import ctypes as C
import os
import re

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsncc.so")
HEADER_PATH = os.path.join(os.path.dirname(_HERE), "include", "sncc.h")

if not os.path.exists(LIB_PATH):
    raise ImportError(
        f"{LIB_PATH} is missing: build it with `python paper_2502_01286_amd/build.py` "
        "(the HIP library is required; there is no fallback)")

# PyTorch bundles its own HIP runtime (same soname as ROCm's).  Loading torch
# first makes this library bind to that already-loaded runtime, so the process
# holds a single HIP runtime whichever module the caller imports first.
try:
    import torch  # noqa: F401
except ImportError:  # the C-ABI itself does not need torch
    pass

lib = C.CDLL(LIB_PATH)

SNCC_OK = 0
SNCC_EINVAL = -1
SNCC_ENOMEM = -2
SNCC_ENOSPC = -3
SNCC_ERANGE = -4
SNCC_EDEGENERATE = -5
SNCC_EDEVICE = -6
SNCC_FP32_KAHAN = 0
SNCC_FP64 = 1
SNCC_FORM_AUTO = 0
SNCC_FORM_TILE_LOCAL = 1
SNCC_FORM_GLOBAL = 2
SNCC_MAX_TEMPLATE_AREA = 8388607
SNCC_MAX_SQ_BOX_AREA = 66051
SNCC_MAX_TABLE_BYTES = 2147483647
SNCC_NOALLOC_SCRATCH_BYTES = 8388608


class sncc_segment(C.Structure):
    _fields_ = [("x", C.c_int32), ("y", C.c_int32), ("w", C.c_int32), ("h", C.c_int32),
                ("sum", C.c_int64), ("area", C.c_int32), ("reserved", C.c_int32)]


SEGMENT_DTYPE = np.dtype([("x", "<i4"), ("y", "<i4"), ("w", "<i4"), ("h", "<i4"),
                          ("sum", "<i8"), ("area", "<i4"), ("reserved", "<i4")])
assert SEGMENT_DTYPE.itemsize == C.sizeof(sncc_segment) == 32


class sncc_batch_desc(C.Structure):
    _fields_ = [("coarse", C.c_void_p), ("fine", C.c_void_p),
                ("d_f", C.c_void_p), ("f_pitch", C.c_int),
                ("d_s", C.c_void_p), ("d_s2", C.c_void_p), ("sat_pitch", C.c_int),
                ("B", C.c_int), ("M", C.c_int), ("N", C.c_int),
                ("n_pairs", C.c_int), ("pairs", C.c_void_p),
                ("k", C.c_int), ("radius", C.c_int),
                ("d_topk", C.c_void_p), ("d_best", C.c_void_p), ("d_count", C.c_void_p),
                ("tune", C.c_int), ("tune_cache", C.c_char_p)]


class sncc_batch_stats(C.Structure):
    _fields_ = [("coarse_evals", C.c_int64), ("n_offsets", C.c_int64),
                ("work_items", C.c_int64), ("computed_evals", C.c_int64),
                ("n_passes", C.c_int64), ("n_launch_classes", C.c_int),
                ("tile_u", C.c_int), ("tile_v", C.c_int), ("wg_threads", C.c_int),
                ("lds_bytes", C.c_int), ("timed", C.c_int),
                ("ms_sat", C.c_float), ("ms_score", C.c_float), ("ms_select", C.c_float),
                ("ms_refine", C.c_float), ("ms_total", C.c_float)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


_vp, _i, _d, _u = C.c_void_p, C.c_int, C.c_double, C.c_size_t
_SIGS = {
    "sncc_status_string": (C.c_char_p, [_i]),
    "sncc_last_error": (C.c_char_p, []),
    "sncc_version": (_i, []),
    "sncc_segment_template": (_i, [_vp, _i, _i, _i, _d, _i, _vp, _i, _vp, _vp, _vp]),
    "sncc_segment_templates": (_i, [_i, _vp, _vp, _vp, _vp, _vp, _i, _i, _vp, C.c_int64, _vp,
                                    _vp, _vp, _vp]),
    "sncc_ctx_create": (_i, [_i, C.c_size_t, _vp]),
    "sncc_ctx_destroy": (_i, [_vp]),
    "sncc_sync": (_i, [_vp]),
    "sncc_ctx_set_timing": (_i, [_vp, _i]),
    "sncc_ctx_stage_ms": (_i, [_vp, _vp, _i, _vp]),
    "sncc_sat_pitch": (_i, [_i, _vp]),
    "sncc_build_sats": (_i, [_vp, _vp, _i, _i, _i, _i, _vp, _vp, _i]),
    "sncc_build_sats_noalloc": (_i, [_vp, _vp, _i, _i, _i, _i, _vp, _vp, _i]),
    "sncc_upload_templates": (_i, [_vp, _i, _vp, _vp, _vp, _vp, _vp]),
    "sncc_tmpl_destroy": (_i, [_vp]),
    "sncc_tmpl_info": (_i, [_vp, _i, _vp, _vp, _vp, _vp]),
    "sncc_tmpl_count": (_i, [_vp, _vp]),
    "sncc_score": (_i, [_vp, _vp, _i, _vp, _vp, _i, _i, _i, _i, _vp, _i, _vp]),
    "sncc_score_frame": (_i, [_vp, _vp, _i, _vp, _i, _i, _i, _i, _vp, _i, _vp, _vp, _vp]),
    "sncc_topk": (_i, [_vp, _vp, _vp, _vp, _i, _i, _i, _i, _i, _vp, _i, _i, _vp]),
    "sncc_argmax": (_i, [_vp, _vp, _vp, _vp, _i, _i, _i, _i, _i, _vp, _i, _vp]),
    "sncc_refine": (_i, [_vp, _vp, _vp, _vp, _i, _i, _i, _i, _i, _vp, _vp, _i, _i, _vp, _vp]),
    "sncc_threshold_match": (_i, [_vp, _vp, _vp, _vp, _vp, _vp, _vp, _i, _i, _i, _i, _i, _vp,
                                  _vp, _i, _vp, _i, _vp]),
    "sncc_batch_create": (_i, [_vp, _vp, _vp]),
    "sncc_batch_run": (_i, [_vp]),
    "sncc_batch_stats_get": (_i, [_vp, _vp]),
    "sncc_batch_destroy": (_i, [_vp]),
}
for _name, (_res, _args) in _SIGS.items():
    try:
        _f = getattr(lib, _name)
    except AttributeError as _e:
        raise ImportError(f"{LIB_PATH} does not export {_name}: it is older than the sources; "
                          "rebuild it with `python paper_2502_01286_amd/build.py`") from _e
    _f.restype = _res
    _f.argtypes = _args


def header_functions():
    """Names of the functions declared in include/sncc.h."""
    with open(HEADER_PATH) as fh:
        text = fh.read()
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(sncc_\w+)\s*\(", text, re.M)))


class SnccError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{lib.sncc_status_string(code).decode()} ({code}): {msg}")
        self.code = code


def _check(rc):
    if rc != SNCC_OK:
        raise SnccError(rc, lib.sncc_last_error().decode())


def sncc_status_string(code: int) -> str:
    return lib.sncc_status_string(code).decode()


def sncc_last_error() -> str:
    return lib.sncc_last_error().decode()


def sncc_version() -> int:
    return lib.sncc_version()


# ----------------------------------------------------------- host (no device)
def sncc_segment_template(t, sigma_max: float, K_max: int = 5000):
    """Returns (segments as a SEGMENT_DTYPE array, sigma_used, rho_max)."""
    t = np.ascontiguousarray(t, dtype=np.uint8)
    if t.ndim != 2:
        raise ValueError("template must be 2-D")
    H, W = t.shape
    cap = W * H
    out = np.zeros(cap, dtype=SEGMENT_DTYPE)
    K = C.c_int(0)
    su = C.c_double(0)
    rm = C.c_double(0)
    _check(lib.sncc_segment_template(t.ctypes.data, W, H, W, float(sigma_max), int(K_max),
                                     out.ctypes.data, cap, C.byref(K), C.byref(su), C.byref(rm)))
    return out[:K.value].copy(), su.value, rm.value


def sncc_segment_templates(templates, sigmas, K_max: int = 5000, n_threads: int = 0,
                           check: bool = True):
    """Batched sncc_segment_template on host threads.  Returns (list of
    segment arrays, sigma_used array, rho_max array, status array); with
    check, a non-OK status raises SnccError."""
    ts = [np.ascontiguousarray(t, dtype=np.uint8) for t in templates]
    T = len(ts)
    if T < 1 or len(sigmas) != T:
        raise ValueError("need one sigma per template and at least one template")
    ptrs = (C.c_void_p * T)(*[t.ctypes.data for t in ts])
    W = np.array([t.shape[1] for t in ts], dtype=np.int32)
    H = np.array([t.shape[0] for t in ts], dtype=np.int32)
    sg = np.ascontiguousarray(sigmas, dtype=np.float64)
    cap = int((W.astype(np.int64) * H).sum())
    out = np.zeros(cap, dtype=SEGMENT_DTYPE)
    off = np.zeros(T + 1, dtype=np.int64)
    su = np.zeros(T)
    rm = np.zeros(T)
    st = np.zeros(T, dtype=np.int32)
    rc = lib.sncc_segment_templates(T, ptrs, W.ctypes.data, H.ctypes.data, W.ctypes.data,
                                    sg.ctypes.data, int(K_max), int(n_threads), out.ctypes.data,
                                    cap, off.ctypes.data, su.ctypes.data, rm.ctypes.data,
                                    st.ctypes.data)
    if check:
        _check(rc)
    lists = [out[off[i]:off[i + 1]].copy() for i in range(T)]
    return lists, su, rm, st


def sncc_sat_pitch(M: int) -> int:
    p = C.c_int(0)
    _check(lib.sncc_sat_pitch(int(M), C.byref(p)))
    return p.value


# ------------------------------------------------------------------ device
def _chk(t, dtype, name, shape=None, min_numel=None):
    """Checks a tensor argument's type, dtype, layout and size (the C side
    sees raw pointers only, so these checks are what keeps a caller's slip from
    becoming an out-of-bounds device access).  ``shape``: exact shape, None
    entries matching any size; ``min_numel``: least number of elements.
    None passes (nullable arguments)."""
    import torch
    if t is None:
        return
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None:
        got = tuple(t.shape)
        if got != shape and (len(got) != len(shape) or any(
                w is not None and int(g) != int(w) for g, w in zip(got, shape))):
            want = "(" + ", ".join("*" if w is None else str(int(w)) for w in shape) + ")"
            raise ValueError(f"{name} must have shape {want}, got {tuple(t.shape)}")
    if min_numel is not None and t.numel() < int(min_numel):
        raise ValueError(f"{name} holds {t.numel()} elements, needs at least {int(min_numel)}")


def _dev(**tensors):
    """Every given tensor (None skipped) is a device tensor, all on one device."""
    first = None
    for name, t in tensors.items():
        if t is None:
            continue
        if not t.is_cuda:
            raise ValueError(f"{name} must be a device tensor")
        if first is None:
            first = (name, t.device)
        elif t.device != first[1]:
            raise ValueError(f"{name} is on {t.device}, {first[0]} on {first[1]}")


def _p(t):
    return None if t is None else t.data_ptr()


def _tables(s, s2, B, N):
    """Checks a pair of sum-table tensors for B frames of N rows (layout of
    sncc_build_sats: B x (N + 1) x pitch int32, or (N + 1) x pitch for one
    frame) and returns their pitch."""
    import torch
    for t, nm in ((s, "s"), (s2, "s2")):
        if not isinstance(t, torch.Tensor) or t.dim() not in (2, 3):
            raise ValueError(f"{nm} must be a 2-D or 3-D int32 tensor")
    if tuple(s.shape) != tuple(s2.shape):
        raise ValueError(f"s and s2 differ in shape: {tuple(s.shape)} vs {tuple(s2.shape)}")
    P = int(s.shape[-1])
    if int(s.shape[-2]) != int(N) + 1:
        raise ValueError(f"s must have N + 1 = {int(N) + 1} rows per frame, got {int(s.shape[-2])}")
    _chk(s, torch.int32, "s", min_numel=int(B) * (int(N) + 1) * P)
    _chk(s2, torch.int32, "s2", min_numel=int(B) * (int(N) + 1) * P)
    return P


def _check_pairs(p, B, n_templates=None):
    if not p.size:
        return
    if len(p) <= 8:  # a few pairs: Python's min/max cost less than NumPy's reductions
        rows = p.tolist()
        f_lo, f_hi = min(r[0] for r in rows), max(r[0] for r in rows)
        t_lo, t_hi = min(r[1] for r in rows), max(r[1] for r in rows)
    else:
        f_lo, f_hi, t_lo, t_hi = p[:, 0].min(), p[:, 0].max(), p[:, 1].min(), p[:, 1].max()
    if f_lo < 0 or f_hi >= int(B):
        raise ValueError(f"pair frame index outside [0, {int(B)})")
    if n_templates is not None and (t_lo < 0 or t_hi >= n_templates):
        raise ValueError(f"pair template index outside [0, {n_templates})")


def sncc_ctx_create(device: int = 0, stream=None):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream(device).cuda_stream
    h = C.c_void_p()
    _check(lib.sncc_ctx_create(int(device), int(stream), C.byref(h)))
    return h


def sncc_ctx_destroy(ctx):
    _check(lib.sncc_ctx_destroy(ctx))


def sncc_sync(ctx):
    _check(lib.sncc_sync(ctx))


def sncc_build_sats(ctx, f, s, s2):
    """f: uint8 (B, N, M) or (N, M); s, s2: int32 (B, N+1, pitch) or (N+1, pitch)
    device tensors holding the uint32 tables."""
    import torch
    if not isinstance(f, torch.Tensor) or f.dim() not in (2, 3):
        raise ValueError("f must be a 2-D or 3-D uint8 tensor")
    if f.dim() == 2:
        f = f.unsqueeze(0)
    B, N, M = f.shape
    if s.dim() == 3 and int(s.shape[0]) != B:
        raise ValueError(f"s holds {int(s.shape[0])} frames, f holds {B}")
    P = _tables(s, s2, B, N)
    _chk(f, torch.uint8, "f")
    _dev(s=s, s2=s2, f=f)
    _check(lib.sncc_build_sats(ctx, f.data_ptr(), B, M, N, M, s.data_ptr(), s2.data_ptr(), P))


def sncc_build_sats_noalloc(ctx, f, s, s2):
    """sncc_build_sats through the allocation-free entry point (static
    carry scratch; SnccError SNCC_ENOSPC when the frames need more)."""
    import torch
    if not isinstance(f, torch.Tensor) or f.dim() not in (2, 3):
        raise ValueError("f must be a 2-D or 3-D uint8 tensor")
    if f.dim() == 2:
        f = f.unsqueeze(0)
    B, N, M = f.shape
    if s.dim() == 3 and int(s.shape[0]) != B:
        raise ValueError(f"s holds {int(s.shape[0])} frames, f holds {B}")
    P = _tables(s, s2, B, N)
    _chk(f, torch.uint8, "f")
    _dev(s=s, s2=s2, f=f)
    _check(lib.sncc_build_sats_noalloc(ctx, f.data_ptr(), B, M, N, M, s.data_ptr(),
                                       s2.data_ptr(), P))


def sncc_upload_templates(ctx, seg_lists, W, H):
    """seg_lists: list of SEGMENT_DTYPE arrays; W, H: sizes per template."""
    T = len(seg_lists)
    arrs = [np.ascontiguousarray(a, dtype=SEGMENT_DTYPE) for a in seg_lists]
    ptrs = (C.c_void_p * T)(*[a.ctypes.data for a in arrs])
    K = (C.c_int * T)(*[len(a) for a in arrs])
    Wa = (C.c_int * T)(*[int(w) for w in W])
    Ha = (C.c_int * T)(*[int(h) for h in H])
    h = C.c_void_p()
    _check(lib.sncc_upload_templates(ctx, T, ptrs, K, Wa, Ha, C.byref(h)))
    return h


def sncc_tmpl_destroy(tm):
    _check(lib.sncc_tmpl_destroy(tm))


def sncc_tmpl_info(tm, index):
    W, H, K, q = C.c_int(), C.c_int(), C.c_int(), C.c_double()
    _check(lib.sncc_tmpl_info(tm, int(index), C.byref(W), C.byref(H), C.byref(K), C.byref(q)))
    return W.value, H.value, K.value, q.value


def sncc_tmpl_count(tm):
    """Number of templates in a set."""
    n = C.c_int(0)
    _check(lib.sncc_tmpl_count(tm, C.byref(n)))
    return n.value


def sncc_score(ctx, tm, index, s, s2, M, N, precision, rho, degen=None):
    """rho: (N-H+1, pitch >= M-W+1) float32 (SNCC_FP32_KAHAN) or float64
    (SNCC_FP64); degen: nullable uint8 tensor of rho's shape."""
    import torch
    want = torch.float32 if precision == SNCC_FP32_KAHAN else torch.float64
    P = _tables(s, s2, 1, N)
    if not isinstance(rho, torch.Tensor) or rho.dim() != 2:
        raise ValueError("rho must be a 2-D tensor")
    _chk(rho, want, "rho")
    _chk(degen, torch.uint8, "degen", shape=tuple(rho.shape))
    W, H, _, _ = sncc_tmpl_info(tm, index)
    nu, nv = int(M) - W + 1, int(N) - H + 1
    if nu < 1 or nv < 1:
        raise ValueError(f"template {W}x{H} larger than the image {int(M)}x{int(N)}")
    pitch = int(rho.shape[-1])
    if int(rho.shape[0]) != nv or pitch < nu:
        raise ValueError(f"rho must have shape ({nv}, >= {nu}), got {tuple(rho.shape)}")
    _dev(s=s, s2=s2, rho=rho, degen=degen)
    _check(lib.sncc_score(ctx, tm, int(index), s.data_ptr(), s2.data_ptr(), int(M), int(N), P,
                          int(precision), rho.data_ptr(), pitch, _p(degen)))


def sncc_score_frame(ctx, tm, index, f, rho, form=SNCC_FORM_AUTO, degen=None, energy=None):
    """FP32-compensated rho map of one frame (uint8 (N, M) device tensor)
    for template `index`, without sum tables passed in; rho: float32
    (N-H+1, pitch >= M-W+1); degen: nullable uint8 and energy: nullable int64
    tensors of rho's shape.  Returns the form that ran."""
    import torch
    if not isinstance(f, torch.Tensor) or f.dim() != 2:
        raise ValueError("f must be a 2-D uint8 tensor")
    N, M = int(f.shape[0]), int(f.shape[1])
    _chk(f, torch.uint8, "f")
    if not isinstance(rho, torch.Tensor) or rho.dim() != 2:
        raise ValueError("rho must be a 2-D float32 tensor")
    _chk(rho, torch.float32, "rho")
    _chk(degen, torch.uint8, "degen", shape=tuple(rho.shape))
    _chk(energy, torch.int64, "energy", shape=tuple(rho.shape))
    W, H, _, _ = sncc_tmpl_info(tm, index)
    nu, nv = M - W + 1, N - H + 1
    if nu < 1 or nv < 1:
        raise ValueError(f"template {W}x{H} larger than the image {M}x{N}")
    if int(rho.shape[0]) != nv or int(rho.shape[1]) < nu:
        raise ValueError(f"rho must have shape ({nv}, >= {nu}), got {tuple(rho.shape)}")
    _dev(f=f, rho=rho, degen=degen, energy=energy)
    used = C.c_int(-1)
    _check(lib.sncc_score_frame(ctx, tm, int(index), f.data_ptr(), M, N, M, int(form),
                                rho.data_ptr(), int(rho.shape[1]), _p(degen), _p(energy),
                                C.byref(used)))
    return used.value


def _pairs_array(pairs):
    p = np.ascontiguousarray(np.asarray(pairs, dtype=np.int32).reshape(-1, 2))
    return p


def sncc_topk(ctx, tm, s, s2, B, M, N, pairs, k, precision, out):
    """out: int32 device tensor (n_pairs, k, 3) = {u, v, rho bits}."""
    import torch
    p = _pairs_array(pairs)
    P = _tables(s, s2, B, N)
    _chk(out, torch.int32, "out", shape=(len(p), int(k), 3))
    _dev(s=s, s2=s2, out=out)
    _check_pairs(p, B, sncc_tmpl_count(tm))
    _check(lib.sncc_topk(ctx, tm, s.data_ptr(), s2.data_ptr(), int(B), int(M), int(N), P,
                         len(p), p.ctypes.data, int(k), int(precision), out.data_ptr()))


def sncc_argmax(ctx, tm, s, s2, B, M, N, pairs, precision, out):
    """out: int32 device tensor (n_pairs, 1, 3) or (n_pairs, 3)."""
    import torch
    p = _pairs_array(pairs)
    P = _tables(s, s2, B, N)
    shape = (len(p), 1, 3) if isinstance(out, torch.Tensor) and out.dim() == 3 else (len(p), 3)
    _chk(out, torch.int32, "out", shape=shape)
    _dev(s=s, s2=s2, out=out)
    _check_pairs(p, B, sncc_tmpl_count(tm))
    _check(lib.sncc_argmax(ctx, tm, s.data_ptr(), s2.data_ptr(), int(B), int(M), int(N), P,
                           len(p), p.ctypes.data, int(precision), out.data_ptr()))


def sncc_refine(ctx, fine, s, s2, B, M, N, pairs, cand, radius, out, count=None):
    """cand: int32 (n_pairs, n_cand, 3); out: int32 (n_pairs, 4) = {u, v, rho f64};
    count: nullable int32 (n_pairs,)."""
    import torch
    p = _pairs_array(pairs)
    P = _tables(s, s2, B, N)
    if not isinstance(cand, torch.Tensor) or cand.dim() != 3:
        raise ValueError("cand must be an int32 (n_pairs, n_cand, 3) tensor")
    _chk(cand, torch.int32, "cand", shape=(len(p), None, 3))
    _chk(out, torch.int32, "out", shape=(len(p), 4))
    _chk(count, torch.int32, "count", shape=(len(p),))
    _dev(s=s, s2=s2, cand=cand, out=out, count=count)
    _check_pairs(p, B, sncc_tmpl_count(fine))
    _check(lib.sncc_refine(ctx, fine, s.data_ptr(), s2.data_ptr(), int(B), int(M), int(N), P,
                           len(p), p.ctypes.data, cand.data_ptr(), int(cand.shape[1]),
                           int(radius), out.data_ptr(), _p(count)))


def sncc_ctx_set_timing(ctx, enable: bool):
    _check(lib.sncc_ctx_set_timing(ctx, 1 if enable else 0))


def sncc_ctx_stage_ms(ctx):
    """Device times (ms) of the stages of the last timed call."""
    ms = (C.c_float * 4)()
    n = C.c_int(0)
    _check(lib.sncc_ctx_stage_ms(ctx, ms, 4, C.byref(n)))
    return [float(ms[i]) for i in range(n.value)]


def sncc_threshold_match(ctx, fast, slow, thr_fast, thr_slow, s, s2, B, M, N, pairs, cand,
                         out, counts):
    """Section 5's two-threshold search.  thr_fast, thr_slow: one float per
    template (host); cand, out: int32 (cap, 6) hit buffers (pair, u, v, 0,
    rho f64); counts: int32 (2,) device."""
    import torch
    p = _pairs_array(pairs)
    P = _tables(s, s2, B, N)
    for t, nm in ((cand, "cand"), (out, "out")):
        if not isinstance(t, torch.Tensor) or t.dim() != 2 or t.shape[1] != 6:
            raise ValueError(f"{nm} must be an int32 (cap, 6) tensor")
        _chk(t, torch.int32, nm)
    _chk(counts, torch.int32, "counts", min_numel=2)
    _dev(s=s, s2=s2, cand=cand, out=out, counts=counts)
    T = sncc_tmpl_count(fast)
    _check_pairs(p, B, T)
    tf = np.ascontiguousarray(thr_fast, dtype=np.float64)
    ts = np.ascontiguousarray(thr_slow, dtype=np.float64)
    if tf.shape != (T,) or ts.shape != (T,):
        raise ValueError(f"need one fast and one slow threshold per template ({T})")
    _check(lib.sncc_threshold_match(ctx, fast, slow, tf.ctypes.data, ts.ctypes.data,
                                    s.data_ptr(), s2.data_ptr(), int(B), int(M), int(N), P,
                                    len(p), p.ctypes.data, cand.data_ptr(), int(cand.shape[0]),
                                    out.data_ptr(), int(out.shape[0]), counts.data_ptr()))


class Batch:
    """Owns a sncc_batch handle.  The captured graph holds raw pointers to the
    buffers and template sets it was created with, so ``_keep`` holds
    references to all of them (and to the host copies the descriptor points
    to) for the life of the batch."""

    def __init__(self, handle, keep):
        self.handle = handle
        self._keep = keep

    def run(self):
        _check(lib.sncc_batch_run(self.handle))

    def stats(self):
        st = sncc_batch_stats()
        _check(lib.sncc_batch_stats_get(self.handle, C.byref(st)))
        return st.as_dict()

    def destroy(self):
        if self.handle:
            _check(lib.sncc_batch_destroy(self.handle))
            self.handle = None
            self._keep = None


def sncc_batch_create(ctx, coarse, s, s2, B, M, N, pairs, k, topk_out, fine=None,
                      radius=2, best_out=None, count_out=None, frames=None, tune=0,
                      tune_cache=None):
    import torch
    p = _pairs_array(pairs)
    P = _tables(s, s2, B, N)
    _chk(frames, torch.uint8, "frames", shape=(int(B), int(N), int(M)))
    _chk(topk_out, torch.int32, "topk_out", shape=(len(p), int(k), 3))
    if fine is not None and best_out is None:
        raise ValueError("a batch with a fine template set needs best_out")
    _chk(best_out, torch.int32, "best_out", shape=(len(p), 4))
    _chk(count_out, torch.int32, "count_out", shape=(len(p),))
    _dev(s=s, s2=s2, frames=frames, topk_out=topk_out, best_out=best_out, count_out=count_out)
    _check_pairs(p, B, sncc_tmpl_count(coarse))
    if fine is not None and sncc_tmpl_count(fine) != sncc_tmpl_count(coarse):
        raise ValueError("coarse and fine template sets differ in size")
    d = sncc_batch_desc()
    d.coarse = coarse
    d.fine = fine
    d.d_f = _p(frames)
    d.f_pitch = int(M)
    d.d_s = s.data_ptr()
    d.d_s2 = s2.data_ptr()
    d.sat_pitch = P
    d.B, d.M, d.N = int(B), int(M), int(N)
    d.n_pairs = len(p)
    d.pairs = p.ctypes.data
    d.k = int(k)
    d.radius = int(radius)
    d.d_topk = topk_out.data_ptr()
    d.d_best = _p(best_out)
    d.d_count = _p(count_out)
    d.tune = int(tune)
    cache = tune_cache.encode() if tune_cache else None
    d.tune_cache = cache
    h = C.c_void_p()
    _check(lib.sncc_batch_create(ctx, C.byref(d), C.byref(h)))
    return Batch(h, (p, cache, coarse, fine, s, s2, frames, topk_out, best_out, count_out))


def sncc_batch_run(batch: Batch):
    batch.run()


def sncc_batch_stats_get(batch: Batch):
    return batch.stats()


def sncc_batch_destroy(batch: Batch):
    batch.destroy()


# ------------------------------------------------------------ decoding helpers
def decode_matches(out) -> np.ndarray:
    """(n_pairs, k, 3) int32 match buffer -> structured numpy (u, v, rho)."""
    a = out.detach().cpu().numpy().astype(np.int32, copy=False)
    res = np.zeros(a.shape[:-1], dtype=[("u", "<i4"), ("v", "<i4"), ("rho", "<f4")])
    res["u"] = a[..., 0]
    res["v"] = a[..., 1]
    res["rho"] = a[..., 2].view(np.float32)
    return res


def decode_matches64(out) -> np.ndarray:
    """(n_pairs, 4) int32 buffer -> structured numpy (u, v, rho float64)."""
    a = np.ascontiguousarray(out.detach().cpu().numpy().astype(np.int32, copy=False))
    res = np.zeros(a.shape[0], dtype=[("u", "<i4"), ("v", "<i4"), ("rho", "<f8")])
    res["u"] = a[:, 0]
    res["v"] = a[:, 1]
    res["rho"] = a[:, 2:4].copy().view(np.float64)[:, 0]
    return res


def decode_hits(buf, count=None) -> np.ndarray:
    """(cap, 6) int32 hit buffer -> structured numpy (pair, u, v, rho float64),
    the first min(count, cap) entries (all when count is None)."""
    a = np.ascontiguousarray(buf.detach().cpu().numpy().astype(np.int32, copy=False))
    n = a.shape[0] if count is None else min(int(count), a.shape[0])
    a = a[:n]
    res = np.zeros(n, dtype=[("pair", "<i4"), ("u", "<i4"), ("v", "<i4"), ("rho", "<f8")])
    res["pair"] = a[:, 0]
    res["u"] = a[:, 1]
    res["v"] = a[:, 2]
    res["rho"] = a[:, 4:6].copy().view(np.float64)[:, 0]
    return res
