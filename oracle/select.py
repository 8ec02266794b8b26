"""Selection of matches: top-K, argmax, the coarse-to-fine refinement and the
paper's own two-threshold search.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Section 2 locates the template at the offset with the highest rho; the matching
algorithm of Section 5 outputs (u, v, rho) triplets.  Ordering key used
throughout: higher rho first, ties broken by the smaller row-major offset
index, i.e. by smaller v, then smaller u.  No non-maximum suppression.
"""

from __future__ import annotations

import numpy as np

from .ncc import rho_at
from .segmentation import TemplateApprox


def topk(rho: np.ndarray, k: int):
    """The k best offsets of a rho map (rows over v, columns over u).

    Returns a list of (u, v, rho) triplets in key order.  NaN entries are
    never selected.
    """
    rho = np.asarray(rho, dtype=np.float64)
    nv, nu = rho.shape
    vv, uu = np.meshgrid(np.arange(nv), np.arange(nu), indexing="ij")
    r = rho.ravel()
    ok = ~np.isnan(r)
    order = np.lexsort((uu.ravel()[ok], vv.ravel()[ok], -r[ok]))[:k]
    us, vs, rs = uu.ravel()[ok][order], vv.ravel()[ok][order], r[ok][order]
    return [(int(a), int(b), float(c)) for a, b, c in zip(us, vs, rs)]


def argmax(rho: np.ndarray):
    """(u, v, rho) of the best offset (Section 2, highest rho)."""
    return topk(rho, 1)[0]


def top2_margin(rho: np.ndarray) -> float:
    """rho of the best offset minus rho of the second best."""
    best = topk(rho, 2)
    return best[0][2] - best[1][2] if len(best) > 1 else float("inf")


def neighbourhood(cands, radius: int, nu: int, nv: int):
    """Union of the (2 radius + 1)^2 square neighbourhoods (Chebyshev
    distance <= radius) of the candidate offsets, clipped to valid offsets,
    as sorted arrays (u, v) without duplicates."""
    pts = set()
    for (u, v, _r) in cands:
        for dv in range(-radius, radius + 1):
            for du in range(-radius, radius + 1):
                uu, vv = u + du, v + dv
                if 0 <= uu < nu and 0 <= vv < nv:
                    pts.add((vv, uu))
    pts = sorted(pts)
    return (np.array([p[1] for p in pts], dtype=np.int64),
            np.array([p[0] for p in pts], dtype=np.int64))


def coarse_fine(s, s2, coarse: TemplateApprox, fine: TemplateApprox,
                M: int, N: int, k: int = 32, radius: int = 2,
                coarse_map=None):
    """Two-stage coarse-to-fine search (Section 5, steps 7a-j, with the
    threshold test replaced by a top-k candidate set).

    Coarse: rho with the coarse approximation at every offset, keep the k best.
    Fine:   rho with the fine approximation on the union of the candidates'
            square neighbourhoods; the result is the best of those.
    Returns a dict with the coarse candidates, the fine candidate set and the
    final (u, v, rho).
    """
    nu, nv = M - coarse.W + 1, N - coarse.H + 1
    if coarse_map is None:
        vv, uu = np.meshgrid(np.arange(nv), np.arange(nu), indexing="ij")
        coarse_map = rho_at(s, s2, coarse, uu, vv)
    cands = topk(coarse_map, k)
    cu, cv = neighbourhood(cands, radius, nu, nv)
    fr = rho_at(s, s2, fine, cu, cv)
    best = min(range(len(fr)), key=lambda i: (-fr[i], cv[i], cu[i]))
    return {
        "coarse": cands,
        "fine_u": cu,
        "fine_v": cv,
        "fine_rho": fr,
        "best": (int(cu[best]), int(cv[best]), float(fr[best])),
    }


def paper_sigmas(t: np.ndarray, fast: float = 0.99, slow: float = 0.1):
    """Section 5's experimental thresholds relative to the template:
    sigma_max,fast = 0.99 sigma_t and sigma_max,slow = 0.1 sigma_t, with
    sigma_t the population standard deviation of t (as in Eq. (2))."""
    tf = np.asarray(t, dtype=np.float64)
    sigma_t = float(np.sqrt(((tf - tf.mean()) ** 2).mean()))
    return fast * sigma_t, slow * sigma_t


def threshold_match(s, s2, fast: TemplateApprox, slow: TemplateApprox, M: int, N: int,
                    precision: float = 0.9, thr_fast=None, thr_slow=None, fast_map=None):
    """The matching algorithm of Section 5, steps 5 and 7a-j.

    threshold_fast = precision * rho_fast and threshold_slow = precision *
    rho_slow, where rho_fast and rho_slow are the NCCs of the two
    approximations with the template (the second output of
    precompute_template_approximation), unless given explicitly.  At every
    offset rho is computed with the fast approximation; offsets with
    rho < threshold_fast are skipped; the others are scored again with the
    slow approximation and appended to the matches when that rho is at least
    threshold_slow.

    Returns a dict: thresholds, the fast survivors (arrays u, v, rho_fast) and
    the matches as (u, v, rho_slow) triplets in row-major offset order.
    """
    if (fast.W, fast.H) != (slow.W, slow.H):
        raise ValueError("fast and slow approximations differ in size")
    tf = precision * fast.rho_max if thr_fast is None else float(thr_fast)
    ts = precision * slow.rho_max if thr_slow is None else float(thr_slow)
    nu, nv = M - fast.W + 1, N - fast.H + 1
    if fast_map is None:
        vv, uu = np.meshgrid(np.arange(nv), np.arange(nu), indexing="ij")
        fast_map = rho_at(s, s2, fast, uu, vv)
    keep = np.asarray(fast_map) >= tf          # step 7f: skip rho < threshold_fast
    cv, cu = np.nonzero(keep)                  # row-major order
    rf = np.asarray(fast_map)[cv, cu]
    rs = rho_at(s, s2, slow, cu, cv) if len(cu) else np.zeros(0)
    hit = rs >= ts                             # step 7j
    matches = [(int(u), int(v), float(r)) for u, v, r in zip(cu[hit], cv[hit], rs[hit])]
    return {"thr_fast": tf, "thr_slow": ts, "cand_u": cu.astype(np.int64),
            "cand_v": cv.astype(np.int64), "cand_rho": rf, "cand_rho_slow": rs,
            "matches": matches}
