"""The banded oracle maps of tests/oracle_pool.py equal the oracle's map of
the whole frame bit for bit (box sums are the same integers from any table
origin, and each offset's arithmetic is the same)."""

import numpy as np

import oracle as O
from oracle_pool import OraclePool
from workloads import synth


def test_banded_maps_equal_whole_maps():
    rng = np.random.default_rng(3)
    frames = [synth.scene(11, 90, 70), synth.texture(12, 75, 64)]
    jobs = []
    for f, (W, H), sg in zip(frames, [(9, 7), (20, 33)], [6, 3]):
        t, _, _ = synth.crop_template(rng, f, W, H, sigma_max=sg)
        jobs.append((f, O.precompute_template_approximation(t, sg)))
    pool = OraclePool(2)
    try:
        got = pool.maps(jobs)
        got1 = pool.maps(jobs[:1])
    finally:
        pool.close()
    for (f, ta), g in zip(jobs, got):
        assert np.array_equal(g, O.rho_map(f, ta))
    assert np.array_equal(got1[0], got[0])
