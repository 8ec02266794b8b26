"""Seeded synthetic images and templates for segmented NCC workloads.

This module only draws inputs: it holds none of the matching method's
arithmetic and imports neither the oracle nor the GPU package, so both sides
can take their inputs from it.  Every draw goes through
``numpy.random.default_rng(seed)`` (PCG64) with fixed seeds per workload.

Generators (uint8 grayscale, rows = y):

* ``scene``: value noise (octaves on lattices of spacing 64/32/16 px with
  amplitudes 1, 1/2, 1/4, smoothstep-bilinear), min-max scaled to 0..255, then
  20 flat axis-aligned rectangles of uniform random intensity painted in order
  (w ~ U[M/20, M/4), h ~ U[N/20, N/4)), then N(0, 3^2) noise, rint, clip.
* ``texture``: value noise with 4 octaves (32/16/8/4 px) plus a checker of
  period p ~ U{3..7} and amplitude +-40, then N(0, 3^2) noise, rint, clip.
* templates: a crop plus independent N(0, 2^2) noise, rint, clip.  A crop whose
  population standard deviation is not above ``sigma_max / 0.99`` is drawn
  again, so that no template's approximation collapses to one segment.

Rounding is ``np.rint`` (half to even) followed by clipping to [0, 255].
"""

from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np


def _smoothstep(t):
    return t * t * (3.0 - 2.0 * t)


def value_noise(rng: np.random.Generator, M: int, N: int, spacings, amps):
    """Sum of lattice value-noise octaves, float64 N x M (unscaled)."""
    out = np.zeros((N, M), dtype=np.float64)
    xs = np.arange(M, dtype=np.float64)
    ys = np.arange(N, dtype=np.float64)
    for sp, amp in zip(spacings, amps):
        ny = N // sp + 2
        nx = M // sp + 2
        lat = rng.random((ny, nx))
        ix = (xs // sp).astype(np.int64)
        iy = (ys // sp).astype(np.int64)
        wx = _smoothstep((xs - ix * sp) / sp)
        wy = _smoothstep((ys - iy * sp) / sp)
        rows = lat[:, ix] * (1.0 - wx) + lat[:, ix + 1] * wx          # ny x M
        out += amp * (rows[iy] * (1.0 - wy)[:, None] + rows[iy + 1] * wy[:, None])
    return out


def _to_u8(img):
    return np.clip(np.rint(img), 0, 255).astype(np.uint8)


def _minmax255(img):
    lo, hi = img.min(), img.max()
    return (img - lo) * (255.0 / (hi - lo)) if hi > lo else np.zeros_like(img)


def scene(seed: int, M: int, N: int, n_rects: int = 20, noise: float = 3.0):
    rng = np.random.default_rng(seed)
    img = _minmax255(value_noise(rng, M, N, (64, 32, 16), (1.0, 0.5, 0.25)))
    for _ in range(n_rects):
        w = int(rng.integers(max(1, M // 20), max(2, M // 4)))
        h = int(rng.integers(max(1, N // 20), max(2, N // 4)))
        x = int(rng.integers(0, M - w + 1))
        y = int(rng.integers(0, N - h + 1))
        img[y:y + h, x:x + w] = rng.uniform(0.0, 255.0)
    img = img + rng.normal(0.0, noise, size=img.shape)
    return _to_u8(img)


def texture(seed: int, M: int, N: int, noise: float = 3.0):
    rng = np.random.default_rng(seed)
    img = _minmax255(value_noise(rng, M, N, (32, 16, 8, 4), (1.0, 0.5, 0.25, 0.125)))
    p = int(rng.integers(3, 8))
    yy, xx = np.mgrid[0:N, 0:M]
    img = img + np.where(((xx // p) + (yy // p)) % 2 == 0, 40.0, -40.0)
    img = img + rng.normal(0.0, noise, size=img.shape)
    return _to_u8(img)


def crop_template(rng: np.random.Generator, frame: np.ndarray, W: int, H: int,
                  sigma_max: Optional[float] = None, noise: float = 2.0,
                  max_tries: int = 1000, pos=None):
    """Crop W x H at a random (or given) position, add N(0, noise^2), round.

    Returns (template, x, y).  When ``sigma_max`` is given, draws again until
    the template's population standard deviation exceeds sigma_max / 0.99.
    """
    N, M = frame.shape
    for _ in range(max_tries):
        if pos is None:
            x = int(rng.integers(0, M - W + 1))
            y = int(rng.integers(0, N - H + 1))
        else:
            x, y = pos
        t = frame[y:y + H, x:x + W].astype(np.float64)
        t = _to_u8(t + rng.normal(0.0, noise, size=t.shape))
        if sigma_max is None or float(t.astype(np.float64).std()) > sigma_max / 0.99:
            return t, x, y
        if pos is not None:
            break
    raise RuntimeError("no crop with enough contrast")


@dataclass
class Workload:
    name: str
    frames: List[np.ndarray]
    templates: List[np.ndarray]
    sigmas: List[float]                     # per template (coarse when fine_sigma set)
    pairs: List[tuple]                      # (frame index, template index)
    k: int = 1
    fine_sigma: Optional[float] = None
    k_max: int = 5000
    origin: list = field(default_factory=list)   # (frame, x, y) of each crop
    note: str = ""

    @property
    def M(self):
        return self.frames[0].shape[1]

    @property
    def N(self):
        return self.frames[0].shape[0]


def scene_640x480(scale: float = 1.0) -> Workload:
    """One 640x480 scene, one 32x32 template, sigma_max 8, full map + argmax."""
    M, N = int(640 * scale), int(480 * scale)
    f = scene(0, M, N)
    rng = np.random.default_rng(1)
    t, x, y = crop_template(rng, f, 32, 32, sigma_max=8)
    return Workload("scene_640x480", [f], [t], [8.0], [(0, 0)], k=1, origin=[(0, x, y)])


def scene_1920x1080(sigma: float = 4.0, scale: float = 1.0) -> Workload:
    """One 1920x1080 scene, one 64x64 template, sigma_max in {4, 8, 16}."""
    M, N = int(1920 * scale), int(1080 * scale)
    f = scene(1000, M, N)
    rng = np.random.default_rng(1001)
    t, x, y = crop_template(rng, f, 64, 64, sigma_max=16)
    return Workload(f"scene_1920x1080_s{int(sigma)}", [f], [t], [float(sigma)], [(0, 0)], k=1,
                    origin=[(0, x, y)])


def texture_3840x2160(size: int = 128, scale: float = 1.0, k_max: int = 5000) -> Workload:
    """One 3840x2160 texture, a 128x128 or 256x256 template taken at the
    highest gradient-energy position among 16 seeded candidates, sigma_max 4."""
    M, N = int(3840 * scale), int(2160 * scale)
    f = texture(2000, M, N)
    rng = np.random.default_rng(2001 if size == 128 else 2002)
    best = None
    ff = f.astype(np.float64)
    for _ in range(16):
        x = int(rng.integers(0, M - size + 1))
        y = int(rng.integers(0, N - size + 1))
        blk = ff[y:y + size, x:x + size]
        e = float((np.diff(blk, axis=0) ** 2).sum() + (np.diff(blk, axis=1) ** 2).sum())
        if best is None or e > best[0]:
            best = (e, x, y)
    _, x, y = best
    t, _, _ = crop_template(rng, f, size, size, sigma_max=4, pos=(x, y))
    return Workload(f"texture_3840x2160_t{size}", [f], [t], [4.0], [(0, 0)], k=1, k_max=k_max,
                    origin=[(0, x, y)])


def batch_16x64(n_frames: int = 16, n_templates: int = 64, M: int = 1920, N: int = 1080,
                side_lo: int = 16, side_hi: int = 192, k: int = 5) -> Workload:
    """Batched: frames x templates of sides U{side_lo..side_hi}, sigma_max in
    {4, 8, 12, 16}, every pair scored, top-k per pair."""
    frames = [scene(3000 + i, M, N) for i in range(n_frames)]
    rng = np.random.default_rng(3999)
    temps, sig, origin = [], [], []
    for _ in range(n_templates):
        W = int(rng.integers(side_lo, side_hi + 1))
        H = int(rng.integers(side_lo, side_hi + 1))
        s = float(rng.choice([4, 8, 12, 16]))
        fi = int(rng.integers(0, n_frames))
        t, x, y = crop_template(rng, frames[fi], W, H, sigma_max=s)
        temps.append(t)
        sig.append(s)
        origin.append((fi, x, y))
    pairs = [(fi, ti) for fi in range(n_frames) for ti in range(n_templates)]
    return Workload("batch_16x64", frames, temps, sig, pairs, k=k, origin=origin)


def coarse_fine_256x32(n_frames: int = 256, n_templates: int = 32, M: int = 1280, N: int = 720,
         side_lo: int = 24, side_hi: int = 96, k: int = 32) -> Workload:
    """Batched coarse-fine: coarse sigma_max 16 (top-k), fine sigma_max 4."""
    frames = [scene(4000 + i, M, N) for i in range(n_frames)]
    rng = np.random.default_rng(4999)
    temps, origin = [], []
    for _ in range(n_templates):
        W = int(rng.integers(side_lo, side_hi + 1))
        H = int(rng.integers(side_lo, side_hi + 1))
        fi = int(rng.integers(0, n_frames))
        t, x, y = crop_template(rng, frames[fi], W, H, sigma_max=16)
        temps.append(t)
        origin.append((fi, x, y))
    pairs = [(fi, ti) for fi in range(n_frames) for ti in range(n_templates)]
    return Workload("coarse_fine_256x32", frames, temps, [16.0] * n_templates, pairs, k=k,
                    fine_sigma=4.0, origin=origin)


def threshold_4x4(n_frames: int = 4, n_templates: int = 4, M: int = 1920, N: int = 1080,
                  side: int = 64) -> Workload:
    """The paper's two-threshold search over a small batch: scenes 1920x1080,
    side x side templates cropped from random frames (re-drawn until their
    deviation exceeds 16 / 0.99), every pair scored; the thresholds are taken
    relative to each template (0.99 and 0.1 of its deviation)."""
    frames = [scene(6000 + i, M, N) for i in range(n_frames)]
    rng = np.random.default_rng(6999)
    temps, origin = [], []
    for _ in range(n_templates):
        fi = int(rng.integers(0, n_frames))
        t, x, y = crop_template(rng, frames[fi], side, side, sigma_max=16)
        temps.append(t)
        origin.append((fi, x, y))
    pairs = [(fi, ti) for fi in range(n_frames) for ti in range(n_templates)]
    return Workload("threshold_4x4", frames, temps, [0.0] * n_templates, pairs, k=0,
                    origin=origin, note="relative thresholds")


def prep_1024(n_templates: int = 1024, n_frames: int = 8, M: int = 1920, N: int = 1080,
              side_lo: int = 16, side_hi: int = 192) -> Workload:
    """Templates only, for timing their preparation: crops of sides
    U{side_lo..side_hi} (independently) from seeded scenes, each re-drawn
    until its deviation exceeds 4 / 0.99."""
    frames = [scene(8000 + i, M, N) for i in range(n_frames)]
    rng = np.random.default_rng(8999)
    temps = []
    for _ in range(n_templates):
        W = int(rng.integers(side_lo, side_hi + 1))
        H = int(rng.integers(side_lo, side_hi + 1))
        fi = int(rng.integers(0, n_frames))
        t, _, _ = crop_template(rng, frames[fi], W, H, sigma_max=4)
        temps.append(t)
    return Workload("prep_1024", [], temps, [0.0] * n_templates, [], k=0,
                    note="templates only")


def large_3840x2160(sizes=((640, 480), (384, 384)), sigma: float = 16.0) -> Workload:
    """One 3840x2160 scene and templates beyond a single exact f^2 box
    (n > 66051): a 640x480 crop (too wide for the staged form) and a 384x384
    crop, each at a seeded position; sigma_max 16, top-5 per pair."""
    f = scene(9500, 3840, 2160)
    rng = np.random.default_rng(9501)
    temps, origin = [], []
    for W, H in sizes:
        t, x, y = crop_template(rng, f, W, H, sigma_max=sigma)
        temps.append(t)
        origin.append((0, x, y))
    return Workload("large_3840x2160", [f], temps, [sigma] * len(temps),
                    [(0, i) for i in range(len(temps))], k=5, origin=origin)
