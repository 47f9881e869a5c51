"""The threaded CPU baseline of bench.py (the oracle's estimator split over
threads by texel runs) gives the oracle's frame bit for bit, multi-resolution
and naive, so its throughput is the oracle's on more cores."""
import os
import sys
from concurrent.futures import ThreadPoolExecutor

import numpy as np

import oracle
import scenegen

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
import bench  # noqa: E402


def test_threaded_oracle_frame_is_bit_identical(scene256):
    s, gb = scene256
    omp = oracle.MaskParams(num_levels=3, level_enable=0b111, sigma2=(0.924, 1.848, 0.0), weight=(100.0, 50.0, 1.0))
    op = oracle.SSAOParams(scenegen.ssao_kernel(16), 0.5, 0.02)
    ref = oracle.frame("ssao", gb.depth, gb.normal, gb.focal, omp, op).out
    ref_plain = oracle.frame("ssao", gb.depth, gb.normal, gb.focal, omp, op, multires=False).out
    with ThreadPoolExecutor(5) as pool:
        got = bench.oracle_ssao_threads(gb.depth, gb.normal, gb.focal, omp, op, pool, 5, True)
        got_plain = bench.oracle_ssao_threads(gb.depth, gb.normal, gb.focal, omp, op, pool, 5, False)
    assert np.array_equal(got, ref)
    assert np.array_equal(got_plain, ref_plain)
