"""The Conflict Resolution Network model (DialSort Sec. 6), no GPU.

Pins: the paper's worked CRN facts (tests/golden/crn_examples.txt), the additive
conservation of Lemma "lem:crn" at every level, ingestion through the CRN equal
to the oracle's histogram, and the counterexample showing that the literal
pairing rule does not make keys unique after ceil(log2 k) levels (which is why
the kernels rely on conservation and additive writes only).
"""

from __future__ import annotations

import math
import os
from collections import Counter

import numpy as np
import pytest
from hypothesis import given, settings
from hypothesis import strategies as st

import oracle
from oracle import crn

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "crn_examples.txt")


def golden():
    d = {}
    for line in open(GOLDEN):
        line = line.strip()
        if line and not line.startswith("#"):
            k, v = (s.strip() for s in line.split("=", 1))
            d[k] = v
    return d


def totals(items):
    c = Counter()
    for k, v in items:
        c[k] += v
    return c


def test_three_arrivals_of_42_become_one_write():
    g = golden()
    lanes = [(int(x), 1) for x in g["lanes_42"].split()]
    final = crn.crn_network(lanes, len(lanes))[-1]
    k, c = g["merged_42"].split(":")
    assert final == [(int(k), int(c))]
    H = crn.crn_ingest([42, 42, 42], 64, 3)
    assert H[42] == 3 and sum(H) == 3


def test_pipeline_depths():
    g = golden()
    assert crn.crn_depth(16) == int(g["depth_16"])
    assert crn.crn_depth(32) == int(g["depth_32"])
    for k in range(1, 200):
        assert crn.crn_depth(k) == math.ceil(math.log2(k)) if k > 1 else crn.crn_depth(k) == 0


def test_odd_residual_forwarded():
    assert crn.crn_level([(1, 1), (1, 2), (5, 1)]) == [(1, 3), (5, 1)]
    assert crn.crn_level([(4, 1)]) == [(4, 1)]
    assert crn.crn_level([(1, 1), (2, 1)]) == [(1, 1), (2, 1)]


@settings(max_examples=300, deadline=None)
@given(st.lists(st.tuples(st.integers(0, 5), st.integers(1, 4)), min_size=1, max_size=40))
def test_conservation_at_every_level(lanes):
    levels = crn.crn_network(lanes, len(lanes))
    assert len(levels) == crn.crn_depth(len(lanes)) + 1
    ref = totals(lanes)
    for lv in levels:
        assert totals(lv) == ref  # Lemma "lem:crn"
        assert len(lv) <= len(lanes)


@pytest.mark.parametrize("k", [1, 2, 3, 8, 16, 32, 64])
@pytest.mark.parametrize("lane_local", [False, True])
def test_crn_ingestion_equals_oracle(k, lane_local):
    rng = np.random.default_rng(k)
    for U in (1, 7, 64):
        keys = rng.integers(0, U, 500).tolist()
        keys += [3 % U] * 40  # a run that lane-local accumulation can merge
        st, H = oracle.histogram(keys, U)
        assert st == oracle.OK
        assert crn.crn_ingest(keys, U, k, lane_local) == H.tolist()


def test_literal_rule_can_leave_duplicates():
    final = crn.crn_network([(7, 1), (9, 1), (7, 1), (9, 1)], 4)[-1]
    assert sorted(final) == [(7, 1), (7, 1), (9, 1), (9, 1)]  # 7 survives twice
    assert totals(final) == {7: 2, 9: 2}  # but nothing is lost


def test_lane_local_accumulation():
    assert crn.lane_local_accumulate([3, 3, 3, 1, 3, 3]) == [(3, 3), (1, 1), (3, 2)]
    assert crn.lane_local_accumulate([]) == []
