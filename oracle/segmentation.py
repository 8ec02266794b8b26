"""Split-and-merge segmented template approximation (oracle side).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Follows Section 3 (Eqs. (2)-(7)) and the three functions printed in Section 5:
``precompute_template_approximation``, ``split_segment`` and
``merge_redundant_segments``.  A segment is kept as its rectangle plus the exact
integer sum T_i of the template pixels it covers and its area A_i = W_i H_i, so
that its mean k_i = T_i / A_i (Eq. (4)) is an exact rational; floating point
appears only in the template constants.
"""

from __future__ import annotations

from dataclasses import dataclass, field
from fractions import Fraction
from typing import List

import numpy as np


@dataclass
class Segment:
    """One rectangle S_i of the approximation (the 5-tuple of Eq. (6)).

    ``x, y`` is the top-left template pixel, ``w, h`` the size W_i x H_i,
    ``total`` the integer sum of t over the rectangle and ``area`` = w * h
    (kept separately because merging adds areas).  k_i = total / area.
    """

    x: int
    y: int
    w: int
    h: int
    total: int
    area: int

    @property
    def mean(self) -> Fraction:
        """k_i of Eq. (4), exactly."""
        return Fraction(self.total, self.area)

    def as_tuple(self):
        return (self.x, self.y, self.w, self.h, self.total, self.area)


@dataclass
class TemplateApprox:
    """Result of ``precompute_template_approximation`` plus the constants that
    the matching phase precomputes (algorithm steps 3-5 of Section 5)."""

    W: int
    H: int
    segments: List[Segment]
    sigma_used: float          # the threshold the accepted split was made with
    k_before_merge: int        # length(k) tested against K_max
    kbar: float                # Eq. (7)
    c: np.ndarray              # k_i - kbar, float64, one per segment
    area: np.ndarray           # A_i = W_i H_i, int64
    q_k: float                 # sum_i A_i (k_i - kbar)^2 (Eq. (17), area-weighted)
    q_t: float                 # sum over pixels of (t - tbar)^2
    rho_max: float             # NCC between t and k (function output, steps 4-7)
    extra: dict = field(default_factory=dict)

    @property
    def K(self) -> int:
        return len(self.segments)


def std_below(total: int, total_sq: int, area: int, sigma_max) -> bool:
    """Eq. (2): population standard deviation of a segment < sigma_max.

    With S = sum t and S2 = sum t^2 over the segment, sigma_i^2 =
    (A*S2 - S^2) / A^2, so sigma_i < sigma_max  <=>  A*S2 - S^2 < sigma_max^2 A^2
    for sigma_max > 0.  Decided in exact rational arithmetic (``sigma_max`` is
    taken as the exact binary value of the float it is given as).
    """
    sig = Fraction(sigma_max)
    if sig <= 0:
        return False
    lhs = area * total_sq - total * total
    return Fraction(lhs) < sig * sig * area * area


def split_segment(t: np.ndarray, sigma_max, x: int, y: int, w: int, h: int,
                  out: List[Segment]) -> None:
    """``split_segment`` of Section 5: recursive binary split.

    A 1x1 segment is a leaf (step 1).  Otherwise the segment is kept when its
    deviation is below the threshold (steps 2-3); if not, it is cut in half
    across its larger side, width when w > h, else height, the first half
    taking the ceiling (steps 4-5).  Leaves are appended in visiting order.
    """
    block = t[y:y + h, x:x + w].astype(np.int64)
    total = int(block.sum())
    if w == 1 and h == 1:
        out.append(Segment(x, y, 1, 1, total, 1))
        return
    total_sq = int((block * block).sum())
    if std_below(total, total_sq, w * h, sigma_max):
        out.append(Segment(x, y, w, h, total, w * h))
        return
    if w > h:
        first = (w + 1) // 2
        split_segment(t, sigma_max, x, y, first, h, out)
        split_segment(t, sigma_max, x + first, y, w // 2, h, out)
    else:
        first = (h + 1) // 2
        split_segment(t, sigma_max, x, y, w, first, out)
        split_segment(t, sigma_max, x, y + first, w, h // 2, out)


def _same_mean(a: Segment, b: Segment) -> bool:
    # k_a == k_b as rationals: T_a / A_a == T_b / A_b
    return a.total * b.area == b.total * a.area


def _absorb_runs(k: List[Segment], order, follows, grow) -> None:
    """One pass of ``merge_redundant_segments``: sort by ``order``, then walk
    the list keeping the segment that currently heads a run.  A segment that
    ``follows`` the head (adjacent along the pass's axis, same extent across
    it) and has the same exact mean is absorbed by the head (``grow`` adds its
    extent; sums and areas add, so the head's mean is unchanged) and left
    empty; any other segment heads the next run."""
    k.sort(key=order)
    head = None
    for seg in k:
        if head is not None and follows(head, seg) and _same_mean(head, seg):
            grow(head, seg)
            head.total += seg.total
            head.area += seg.area
        else:
            head = seg


def _grow_down(head: Segment, seg: Segment) -> None:
    head.h += seg.h
    seg.h = 0


def _grow_right(head: Segment, seg: Segment) -> None:
    head.w += seg.w
    seg.w = 0


def merge_redundant_segments(segs: List[Segment]) -> List[Segment]:
    """``merge_redundant_segments`` of Section 5, on a copy of the list.

    In the paper's order: sort by (x, y) and join vertically adjacent segments
    with the same x, the same width and equal means; sort by (y, x) and join
    horizontally adjacent ones with the same y, the same height and equal
    means; drop the emptied segments; repeat while the drop removed anything.
    An emptied segment (height or width 0) never matches a live one, since
    their extents across the pass differ.
    """
    k = [Segment(*s.as_tuple()) for s in segs]
    while True:
        _absorb_runs(k, lambda s: (s.x, s.y),
                     lambda a, b: a.x == b.x and a.w == b.w and a.y + a.h == b.y,
                     _grow_down)
        _absorb_runs(k, lambda s: (s.y, s.x),
                     lambda a, b: a.y == b.y and a.h == b.h and a.x + a.w == b.x,
                     _grow_right)
        kept = [s for s in k if s.w != 0 and s.h != 0]
        if len(kept) == len(k):
            return kept
        k = kept


def approximation_image(W: int, H: int, segs: List[Segment]) -> np.ndarray:
    """The piecewise-constant image k of Eq. (3), float64 (H rows, W columns)."""
    img = np.full((H, W), np.nan)
    for s in segs:
        img[s.y:s.y + s.h, s.x:s.x + s.w] = s.total / s.area
    return img


def template_constants(t: np.ndarray, segs: List[Segment]):
    """Algorithm steps 3-4 of Section 5 and steps 4-6 of
    ``precompute_template_approximation``.

    Returns (kbar, c, area, q_k, q_t, rho_max):
      kbar    Eq. (7): sum_i W_i H_i k_i / (W H)
      c       zero-mean variant k_i - kbar
      q_k     sum_i W_i H_i (k_i - kbar)^2   (area-weighted reading of Eq. (17))
      q_t     sum_{x,y} (t - tbar)^2
      rho_max num / denom with num = sum_i (sum_{S_i} t - tbar W_i H_i)(k_i - kbar)
              and denom = sqrt(q_t * q_k), i.e. NCC between t and k.
    """
    H, W = t.shape
    n = W * H
    area = np.array([s.area for s in segs], dtype=np.int64)
    total = np.array([s.total for s in segs], dtype=np.int64)
    k = total.astype(np.float64) / area.astype(np.float64)          # Eq. (4)
    kbar = float((area * k).sum() / n)                              # Eq. (7)
    c = k - kbar
    q_k = float((area * c * c).sum())
    tf = t.astype(np.float64)
    tbar = float(tf.mean())
    q_t = float(((tf - tbar) ** 2).sum())
    num = float(((total - tbar * area) * c).sum())
    denom = float(np.sqrt(q_t * q_k))
    rho_max = num / denom if denom > 0 else float("nan")
    return kbar, c, area, q_k, q_t, rho_max


def precompute_template_approximation(t: np.ndarray, sigma_max, k_max: int = 5000,
                                      merge: bool = True) -> TemplateApprox:
    """``precompute_template_approximation`` of Section 5.

    Repeats the split with sigma_max raised by 1 after every attempt until the
    split produces at most ``k_max`` segments (counted before merging), then
    merges, then computes the template constants.  ``sigma_used`` is the
    threshold of the accepted split.  Raises ValueError when the approximation is
    uniform (q_k == 0): Section 2 puts uniform templates out of scope.
    """
    t = np.asarray(t)
    if t.ndim != 2 or t.shape[0] < 1 or t.shape[1] < 1:
        raise ValueError("template must be a non-empty 2-D array")
    if k_max < 1:
        raise ValueError("k_max must be >= 1")
    H, W = t.shape
    sigma = sigma_max
    while True:
        leaves: List[Segment] = []
        split_segment(t, sigma, 0, 0, W, H, leaves)
        used = sigma
        sigma = sigma + 1
        if len(leaves) <= k_max:
            break
    segs = merge_redundant_segments(leaves) if merge else leaves
    # The approximation is uniform exactly when every segment mean equals the
    # template mean: T_i * n == T * A_i for all i (exact integers).
    n = W * H
    t_sum = sum(s.total for s in segs)
    if all(s.total * n == t_sum * s.area for s in segs):
        raise ValueError("uniform template approximation (q_k == 0)")
    kbar, c, area, q_k, q_t, rho_max = template_constants(t, segs)
    return TemplateApprox(W=W, H=H, segments=segs, sigma_used=used,
                          k_before_merge=len(leaves), kbar=kbar, c=c, area=area,
                          q_k=q_k, q_t=q_t, rho_max=rho_max,
                          extra={"leaves": leaves})
