"""Oracle maps at full workload sizes, computed in a pool of processes.

Test infrastructure: the workers run the oracle's rho_map (plain NumPy FP64)
on bands of offset rows.  A band of rows [v0, v1) of a frame's map is the map
of the image rows [v0, v1 + H - 1), since every box sum is the same integer
whichever origin the sum tables have, so the band's values are the values of
the whole map; bands of 16 rows keep each per-segment array in cache.  The
workers import numpy and the oracle only (never torch or the GPU library), and
are started with the spawn method so that nothing of a parent that has
initialised the GPU is inherited.
"""

from __future__ import annotations

import multiprocessing as mp
import os
from concurrent.futures import ProcessPoolExecutor

import numpy as np

import oracle as O

SUB_BAND = 16


def n_workers() -> int:
    return max(1, min(16, len(os.sched_getaffinity(0))))


def _band(job):
    f_rows, ta, nv_band = job
    out = np.empty((nv_band, f_rows.shape[1] - ta.W + 1))
    for a in range(0, nv_band, SUB_BAND):
        b = min(nv_band, a + SUB_BAND)
        out[a:b] = O.rho_map(f_rows[a:b + ta.H - 1], ta)
    return out


class OraclePool:
    def __init__(self, n: int | None = None):
        self.n = n or n_workers()
        self.ex = ProcessPoolExecutor(max_workers=self.n, mp_context=mp.get_context("spawn"))

    def close(self):
        self.ex.shutdown(wait=True, cancel_futures=True)

    def maps(self, jobs):
        """jobs: list of (frame as an N x M uint8 array, TemplateApprox).
        Returns the full FP64 rho map of each job ((N-H+1) x (M-W+1))."""
        tasks, where = [], []
        for j, (f, ta) in enumerate(jobs):
            nv = f.shape[0] - ta.H + 1
            # about four tasks per worker for a single big map, whole maps for many small ones
            rows = max(SUB_BAND, -(-nv // max(1, 4 * self.n // max(1, len(jobs)))))
            for v0 in range(0, nv, rows):
                v1 = min(nv, v0 + rows)
                tasks.append((np.ascontiguousarray(f[v0:v1 + ta.H - 1]), ta, v1 - v0))
                where.append((j, v0))
        out = [np.empty((f.shape[0] - ta.H + 1, f.shape[1] - ta.W + 1)) for f, ta in jobs]
        for (j, v0), m in zip(where, self.ex.map(_band, tasks)):
            out[j][v0:v0 + m.shape[0]] = m
        return out
