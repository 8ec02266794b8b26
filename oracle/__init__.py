"""CPU reference (oracle) for segmented NCC template matching.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  The product path
(the HIP library and its Python binding) never imports, calls or links it, and
this package imports nothing from the product path.

Everything here is plain NumPy: integers in int64 (or exact Python integers and
``fractions.Fraction`` where the paper's test is a comparison), floating point in
float64.  Each function cites the part of the paper (Marušić, Popović, Kalafatić,
"Template Matching in Images using Segmented Normalized Cross-Correlation",
arXiv:2502.01286) that it follows.

Readings taken where the paper is silent or inconsistent:

* Eq. (17), step 4 of the matching algorithm and step 6 of
  ``precompute_template_approximation`` print sum_i (k_i - kbar)^2 without the
  segment area; it is read as the area-weighted sum_i W_i H_i (k_i - kbar)^2,
  i.e. sum over pixels of (k - kbar)^2, which is what substituting k for t in
  Eq. (1) gives (Section 4, first paragraph); the unweighted form can exceed
  |rho| = 1, which NCC cannot (Table 1 reports maxima <= 1).
* Sum-table entries at index -1 in Eqs. (11), (13) and (15) are zero; the tables
  are stored zero-padded with one extra leading row and column.
* The standard-deviation test of Eq. (2) is the population deviation with a
  strict ``<``, decided exactly.
* "Equal mean" in merge_redundant_segments is exact rational equality.
* A window whose pixels are all equal gives rho = 0 and is flagged; a template
  whose approximation is uniform is rejected (Section 2 puts both out of scope).

Parity status per function: every public function is pinned by the CPU tests
under ``tests/`` (brute-force Eq. (1), closed forms, invariants, hand-derived
golden fixtures).  ``threshold_match`` is pinned against brute-force Eq. (1)
maps of both approximation images and a planted copy.  ``coarse_fine`` is
pinned against a brute-force walk of steps 7f-i over brute-force Eq. (1) maps
of both approximation images (full sort, Chebyshev test at every offset) and
planted exact ties; ``neighbourhood`` against hand-derived unions at corners
and edges; ``top2_margin`` against hand values and a full sort.  The quality
of the coarse-to-fine heuristic itself (whether it finds the global maximum) has
no reference value: parity unpinned for that property.
"""

from .segmentation import (
    Segment,
    TemplateApprox,
    split_segment,
    merge_redundant_segments,
    precompute_template_approximation,
    approximation_image,
    template_constants,
)
from .ncc import (
    sum_tables,
    window_sums,
    rho_at,
    rho_map,
    brute_ncc_map,
)
from .select import topk, argmax, top2_margin, coarse_fine, paper_sigmas, threshold_match

__all__ = [
    "Segment",
    "TemplateApprox",
    "split_segment",
    "merge_redundant_segments",
    "precompute_template_approximation",
    "approximation_image",
    "template_constants",
    "sum_tables",
    "window_sums",
    "rho_at",
    "rho_map",
    "brute_ncc_map",
    "topk",
    "argmax",
    "top2_margin",
    "coarse_fine",
    "paper_sigmas",
    "threshold_match",
]
