"""The CPU-parallel benchmark baseline agrees with the oracle (it is timed
beside the GPU path, so its output is checked like any other)."""

from __future__ import annotations

import numpy as np
import pytest

import oracle
from oracle import cpu_parallel


@pytest.mark.parametrize("n,U,T", [(0, 5, 3), (1, 1, 1), (1000, 7, 4), (100_003, 65536, 8), (300_000, 1 << 20, 5),
                                   (50_000, 3, 16)])
def test_cpu_parallel_matches_the_oracle(n, U, T):
    rng = np.random.default_rng(n + U + T)
    keys = rng.integers(0, U, n).astype(np.uint32)
    st, H, out = cpu_parallel.sort(keys, U, T)
    st_o, H_o, out_o = oracle.sort(keys, U)
    assert st == 0 and st_o == oracle.OK
    assert np.array_equal(H, H_o) and np.array_equal(out, out_o)
    st, H2, none = cpu_parallel.sort(keys, U, T, out=False)
    assert st == 0 and none is None and np.array_equal(H2, H_o)


def test_cpu_parallel_key_out_of_range():
    keys = np.array([0, 5, 9, 10], dtype=np.uint32)
    st, _, _ = cpu_parallel.sort(keys, 10, 2)
    assert st == 2
