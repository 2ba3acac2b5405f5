"""Reference model of the Conflict Resolution Network -- test infrastructure only.

DialSort, Sec. 6 ("Conflict Resolution Network").  Each of k ingestion lanes
carries a pair (key, count) per cycle (Sec. 6.2, lane state).  A CRN node looks
at two pairs: equal keys are merged into one pair whose count is the sum
(Eq. (3) "eq:crn_eq"); unequal keys are both forwarded unchanged (Eq. (4)
"eq:crn_neq").  A level groups adjacent items into consecutive pairs and
forwards an odd residual unchanged (Definition "def:crn_level"); the network
has ceil(log2 k) levels (Theorem "thm:par", Sec. 6.6).  Surviving pairs are
written additively into the histogram, H[key] += count (Sec. 6.4, Lemma
"lem:crn" and Table "tab:crn").

Only equality between keys is evaluated here, never an order comparison
(Definition "def:ordercomp").

Reading (recorded in the design notes): the Definition claims that after the
last level every key appears at most once.  For the literal pairing rule that is
not true in general (lanes [a, b, a, b] never pair the two a's), so only the
conservation property of Lemma "lem:crn" is relied upon, and the final writes are
additive, never plain stores.
"""

from __future__ import annotations

from typing import Iterable, List, Sequence, Tuple

Pair = Tuple[int, int]


def crn_depth(k: int) -> int:
    """Number of CRN levels for k lanes: ceil(log2 k) (0 for a single lane)."""
    if k < 1:
        raise ValueError("k must be >= 1")
    depth = 0
    while (1 << depth) < k:
        depth += 1
    return depth


def crn_level(items: Sequence[Pair]) -> List[Pair]:
    """One level transition (Definition "def:crn_level")."""
    out: List[Pair] = []
    i = 0
    while i + 1 < len(items):
        (a, ca), (b, cb) = items[i], items[i + 1]
        if a == b:  # Eq. (3): merge additively
            out.append((a, ca + cb))
        else:  # Eq. (4): forward both unchanged
            out.append((a, ca))
            out.append((b, cb))
        i += 2
    if i < len(items):  # odd residual, forwarded unchanged
        out.append(items[i])
    return out


def crn_network(lanes: Sequence[Pair], k: int) -> List[List[Pair]]:
    """Run all ceil(log2 k) levels on one cycle's lane states.

    Returns the list of level multisets L^(0), L^(1), ..., L^(L)."""
    levels = [list(lanes)]
    for _ in range(crn_depth(k)):
        levels.append(crn_level(levels[-1]))
    return levels


def lane_local_accumulate(stream: Iterable[int]) -> List[Pair]:
    """Lane-local accumulation (Sec. 6.2): consecutive equal keys in one lane
    are pre-added into a single (key, count) pair.  Equality only."""
    out: List[Pair] = []
    for x in stream:
        if out and out[-1][0] == x:
            out[-1] = (x, out[-1][1] + 1)
        else:
            out.append((x, 1))
    return out


def crn_ingest(keys: Sequence[int], U: int, k: int, lane_local: bool = False) -> List[int]:
    """Ingest keys through k lanes and the CRN into a zeroed histogram.

    Base form: cycle t presents keys[t*k : (t+1)*k], one (key, 1) pair per
    lane.  With lane_local=True the keys are split into k contiguous lane
    streams, each stream is run-length accumulated first, and cycle t presents
    the t-th pair of every lane that still has one.  Either way every surviving
    pair is added into H."""
    H = [0] * U
    if lane_local:
        m = (len(keys) + k - 1) // k if keys else 0
        streams = [lane_local_accumulate(keys[i * m:(i + 1) * m]) for i in range(k)]
        cycles = max((len(s) for s in streams), default=0)
        batches = [[s[t] for s in streams if t < len(s)] for t in range(cycles)]
    else:
        batches = [[(x, 1) for x in keys[t:t + k]] for t in range(0, len(keys), k)]
    for lanes in batches:
        for key, count in crn_network(lanes, k)[-1]:
            H[key] += count
    return H
