"""Approximate NCC through sum tables, and brute-force exact NCC (oracle side).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Image f has M columns (x) and N rows (y) and is stored as an N x M array
(Section 2).  Offsets are u in [0, M-W], v in [0, N-H] (algorithm step 7 of
Section 5).  Maps over offsets are (N-H+1) x (M-W+1) arrays, rows over v.
"""

from __future__ import annotations

import numpy as np

from .segmentation import TemplateApprox


def sum_tables(f: np.ndarray):
    """Sum tables s and s^2 of Eqs. (10) and (14), int64, zero-padded.

    ``s[y + 1, x + 1]`` is the sum of f over columns 0..x and rows 0..y, which
    is s(x, y) of Eq. (10); row 0 and column 0 hold zeros, the values of
    s(-1, .) and s(., -1) needed by Eqs. (11), (13) and (15).
    """
    f64 = np.asarray(f).astype(np.int64)
    N, M = f64.shape
    s = np.zeros((N + 1, M + 1), dtype=np.int64)
    s2 = np.zeros((N + 1, M + 1), dtype=np.int64)
    s[1:, 1:] = f64.cumsum(axis=0).cumsum(axis=1)
    s2[1:, 1:] = (f64 * f64).cumsum(axis=0).cumsum(axis=1)
    return s, s2


def _box(s: np.ndarray, u, v, x: int, y: int, w: int, h: int):
    """Four-corner rectangle sum of Eq. (11) on a zero-padded table: the sum
    over pixels (u+x .. u+x+w-1, v+y .. v+y+h-1)."""
    return (s[v + y + h, u + x + w] - s[v + y + h, u + x]
            - s[v + y, u + x + w] + s[v + y, u + x])


def window_sums(s: np.ndarray, s2: np.ndarray, W: int, H: int, u, v):
    """Eqs. (13) and (15) plus the exact window energy.

    Returns (Sf, Sf2, V) as int64 arrays where V = n*Sf2 - Sf^2 = n times
    Eq. (16)'s sum (f - fbar)^2, n = W H.
    """
    u = np.asarray(u, dtype=np.int64)
    v = np.asarray(v, dtype=np.int64)
    sf = _box(s, u, v, 0, 0, W, H)
    sf2 = _box(s2, u, v, 0, 0, W, H)
    n = W * H
    V = n * sf2 - sf * sf
    return sf, sf2, V


def _rho(box, tmpl: TemplateApprox, shape, return_flag: bool):
    """Eqs. (12)-(18) given ``box(s_table, x, y, w, h)``, which returns the
    Eq. (11) rectangle sums of a table for every offset of interest."""
    W, H = tmpl.W, tmpl.H
    n = W * H
    sf = box(0, 0, 0, W, H)                          # Eq. (13)
    sf2 = box(1, 0, 0, W, H)                         # Eq. (15)
    V = n * sf2 - sf * sf                            # n * Eq. (16), exact
    fbar = sf.astype(np.float64) / n
    num = np.zeros(shape, dtype=np.float64)
    for seg, c_i in zip(tmpl.segments, tmpl.c):     # Eq. (12)
        b = box(0, seg.x, seg.y, seg.w, seg.h).astype(np.float64)
        b -= fbar * seg.area
        b *= c_i
        num += b
    energy = V.astype(np.float64) / n
    denom = np.sqrt(energy * tmpl.q_k)               # Eq. (17), area-weighted
    flat = V == 0
    with np.errstate(divide="ignore", invalid="ignore"):
        rho = np.where(flat, 0.0, num / np.where(flat, 1.0, denom))   # Eq. (18)
    if return_flag:
        return rho, flat
    return rho


def rho_at(s: np.ndarray, s2: np.ndarray, tmpl: TemplateApprox, u, v,
           return_flag: bool = False):
    """rho(u, v; f, k) of Eq. (18) at the given offsets (arrays of any shape).

    num   Eq. (12): sum_i (box_i - fbar * W_i H_i) (k_i - kbar), float64
    denom Eq. (17) (area-weighted reading): sqrt(energy * q_k) with
          energy = sum f^2 - fbar sum f (Eq. (16)) = V / n
    A window of equal pixels (V == 0) gets rho = 0 and is flagged.
    """
    u, v = np.broadcast_arrays(np.asarray(u, dtype=np.int64),
                               np.asarray(v, dtype=np.int64))
    tabs = (s, s2)

    def box(which, x, y, w, h):
        return _box(tabs[which], u, v, x, y, w, h)

    return _rho(box, tmpl, u.shape, return_flag)


def rho_map(f: np.ndarray, tmpl: TemplateApprox, return_flag: bool = False,
            tables=None):
    """rho over every offset (algorithm step 7 of Section 5), as an
    (N-H+1) x (M-W+1) float64 array.  Same arithmetic as ``rho_at``; the
    rectangle sums of all offsets are taken as shifted slices of the tables."""
    N, M = np.asarray(f).shape
    if tmpl.W > M or tmpl.H > N:
        raise ValueError("template larger than image")
    s, s2 = tables if tables is not None else sum_tables(f)
    nu, nv = M - tmpl.W + 1, N - tmpl.H + 1
    tabs = (s, s2)

    def box(which, x, y, w, h):
        t = tabs[which]
        return (t[y + h:y + h + nv, x + w:x + w + nu] - t[y + h:y + h + nv, x:x + nu]
                - t[y:y + nv, x + w:x + w + nu] + t[y:y + nv, x:x + nu])

    return _rho(box, tmpl, (nv, nu), return_flag)


def brute_ncc_map(f: np.ndarray, t: np.ndarray) -> np.ndarray:
    """Eq. (1) evaluated pixel by pixel (Section 2), float64, two-pass means.

    ``t`` may be any real H x W array (the template itself, or the float
    approximation image k).  Windows with zero variance get NaN.  Cost is
    W H (M-W+1)(N-H+1): tiny inputs only.
    """
    f = np.asarray(f, dtype=np.float64)
    t = np.asarray(t, dtype=np.float64)
    N, M = f.shape
    H, W = t.shape
    tz = t - t.mean()
    tq = float((tz * tz).sum())
    out = np.empty((N - H + 1, M - W + 1))
    for v in range(N - H + 1):
        for u in range(M - W + 1):
            win = f[v:v + H, u:u + W]
            wz = win - win.mean()
            den = np.sqrt(float((wz * wz).sum()) * tq)
            out[v, u] = float((wz * tz).sum()) / den if den > 0 else np.nan
    return out
