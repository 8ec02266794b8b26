"""Helpers for the GPU parity tests: device inputs through the HIP library,
expected values through the oracle.  Inputs come from workloads.synth or
seeded NumPy draws; nothing the GPU computes is fed to the oracle."""

from __future__ import annotations

import numpy as np

import oracle as O


def torch_mod():
    import torch
    return torch


def device_frames(frames):
    torch = torch_mod()
    a = np.stack([np.ascontiguousarray(f, dtype=np.uint8) for f in frames])
    return torch.from_numpy(a).cuda()


def build_sats(S, ctx, frames):
    torch = torch_mod()
    f = device_frames(frames)
    B, N, M = f.shape
    P = S.sncc_sat_pitch(M)
    s = torch.empty((B, N + 1, P), dtype=torch.int32, device="cuda")
    s2 = torch.empty_like(s)
    S.sncc_build_sats(ctx, f, s, s2)
    return f, s, s2


def lib_templates(S, ctx, templates, sigmas, k_max=5000):
    segs, W, H = [], [], []
    for t, sg in zip(templates, sigmas):
        a, _, _ = S.sncc_segment_template(t, sg, k_max)
        segs.append(a)
        H.append(t.shape[0])
        W.append(t.shape[1])
    return S.sncc_upload_templates(ctx, segs, W, H)


def oracle_templates(templates, sigmas, k_max=5000):
    return [O.precompute_template_approximation(t, s, k_max) for t, s in zip(templates, sigmas)]


def topk_ok(rho_map, got, k, tol):
    """Checks a GPU top-k list against an oracle map.

    Every reported rho must equal the oracle at the reported offset within
    `tol`; rank r must hold the oracle's rank-r offset wherever the oracle's
    gap around that rank exceeds 10*tol (elsewhere several orders are
    correct); the reported values must be non-increasing.
    """
    want = O.topk(rho_map, k + 1)
    errs = []
    for r in range(min(k, len(want))):
        u, v, rho = int(got[r]["u"]), int(got[r]["v"]), float(got[r]["rho"])
        if abs(rho_map[v, u] - rho) > tol:
            errs.append(f"rank {r}: rho {rho} vs oracle {rho_map[v, u]} at ({u},{v})")
        lo = want[r - 1][2] - want[r][2] if r > 0 else np.inf
        hi = want[r][2] - want[r + 1][2] if r + 1 < len(want) else np.inf
        if min(lo, hi) > 10 * tol and (u, v) != (want[r][0], want[r][1]):
            errs.append(f"rank {r}: ({u},{v}) vs oracle ({want[r][0]},{want[r][1]})")
        if r > 0 and float(got[r]["rho"]) > float(got[r - 1]["rho"]):
            errs.append(f"rank {r}: not sorted")
    return errs
