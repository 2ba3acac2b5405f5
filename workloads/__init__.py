"""Seeded synthetic inputs for DialSort -- shared by the tests, the oracle side
and the benchmark.  Holds none of the method's arithmetic: it only draws keys.

Every generator returns a 1-D ``torch.int32`` tensor whose bits are the uint32
keys (keys >= 2**31 appear negative when read as int32).  ``device`` selects where
the draw happens: ``"cpu"`` (torch's CPU generator) or ``"cuda"`` (Philox on the
GPU, for the large benchmark inputs).  The same seed on different devices gives
different, equally distributed keys.

Distributions:
  * ``uniform``        i.i.d. uniform on [0, U).
  * ``zipf``           truncated Zipf over ranks 1..U, P(r) proportional to r**-s,
                       sampled through the inverse CDF (float64 table); the key is
                       perm[r - 1] for a seeded permutation perm of [0, U).
  * ``hot_zipf``       exactly round(hot_frac * n) positions (chosen by a seeded
                       shuffle) hold one hot key h drawn uniformly from [0, U); the
                       rest are ``zipf``.  The conflict-stress workload: n = 2**28,
                       U = 2**16, hot_frac = 0.5, s = 1.2.
  * the paper's four distributions (DialSort Sec. 8.2): ``paper_uniform``,
    ``paper_skewed`` (each key independently: with probability 0.8 uniform on
    [0, floor(0.05 U)] inclusive, else uniform on [0, U - 1]),
    ``paper_sorted`` and ``paper_reverse`` (uniform keys in ascending /
    descending order).
Workload tables:
  * ``batch_spec``     the uneven-batch workload: 4096 arrays, n log-uniform in
                       [2**10, 2**22], U = 2**e with e uniform in {10..20}, half
                       uniform and half Zipf(1.1) (exactly count // 2, by a seeded
                       shuffle).
  * ``request_stream`` the served workload: Poisson arrivals, n log-uniform in
                       [2**12, 2**24], U uniform over {2**12, 2**16, 2**20, 2**24},
                       uniform or Zipf(1.2) with probability 1/2 each.
"""

from __future__ import annotations

import math
from dataclasses import dataclass
from typing import List, Optional

import numpy as np
import torch

BASE_SEED = 20260321  # DialSort Sec. 8.1 fixes this seed for its benchmark


def _gen(seed: int, device: str) -> torch.Generator:
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    return g


def _to_key_tensor(x: torch.Tensor) -> torch.Tensor:
    # int64 values in [0, 2**32) -> int32 tensor with the same low 32 bits
    return (x & 0xFFFFFFFF).to(torch.int32) if x.dtype != torch.int32 else x


def uniform(n: int, U: int, seed: int, device: str = "cpu") -> torch.Tensor:
    g = _gen(seed, device)
    if U <= 2**31:
        return torch.randint(0, U, (n,), generator=g, device=device, dtype=torch.int32)
    return _to_key_tensor(torch.randint(0, U, (n,), generator=g, device=device, dtype=torch.int64))


def zipf_table(U: int, s: float, device: str = "cpu") -> torch.Tensor:
    """Normalised float64 CDF of the truncated Zipf law over ranks 1..U."""
    r = torch.arange(1, U + 1, device=device, dtype=torch.float64)
    w = r.pow(-s)
    cdf = torch.cumsum(w, 0)
    return cdf / cdf[-1]


def zipf(n: int, U: int, s: float, seed: int, device: str = "cpu",
         perm: Optional[torch.Tensor] = None) -> torch.Tensor:
    g = _gen(seed, device)
    if perm is None:
        perm = torch.randperm(U, generator=g, device=device)
    cdf = zipf_table(U, s, device)
    u = torch.rand(n, generator=g, device=device, dtype=torch.float64)
    idx = torch.searchsorted(cdf, u, right=True).clamp_(max=U - 1)
    return _to_key_tensor(perm[idx])


def hot_zipf(n: int, U: int, seed: int, device: str = "cpu", hot_frac: float = 0.5,
             s: float = 1.2) -> torch.Tensor:
    g = _gen(seed + 7919, device)
    hot = int(torch.randint(0, U, (1,), generator=g, device=device, dtype=torch.int64).item())
    keys = zipf(n, U, s, seed, device)
    m = int(round(hot_frac * n))
    if m:
        pos = torch.randperm(n, generator=g, device=device)[:m]
        keys[pos] = _to_key_tensor(torch.tensor([hot], dtype=torch.int64, device=device))
    return keys


def paper_uniform(n: int, U: int, seed: int, device: str = "cpu") -> torch.Tensor:
    return uniform(n, U, seed, device)


def paper_skewed(n: int, U: int, seed: int, device: str = "cpu") -> torch.Tensor:
    g = _gen(seed, device)
    hi_small = (5 * U) // 100  # floor(0.05 U), inclusive upper bound
    small = torch.randint(0, hi_small + 1, (n,), generator=g, device=device, dtype=torch.int64)
    wide = torch.randint(0, U, (n,), generator=g, device=device, dtype=torch.int64)
    pick = torch.rand(n, generator=g, device=device) < 0.8
    return _to_key_tensor(torch.where(pick, small, wide))


def paper_sorted(n: int, U: int, seed: int, device: str = "cpu") -> torch.Tensor:
    k = uniform(n, U, seed, device).to(torch.int64) & 0xFFFFFFFF
    return _to_key_tensor(torch.sort(k).values)


def paper_reverse(n: int, U: int, seed: int, device: str = "cpu") -> torch.Tensor:
    k = uniform(n, U, seed, device).to(torch.int64) & 0xFFFFFFFF
    return _to_key_tensor(torch.sort(k, descending=True).values)


PAPER_DISTRIBUTIONS = {
    "uniform": paper_uniform,
    "skewed": paper_skewed,
    "sorted": paper_sorted,
    "reverse": paper_reverse,
}


def as_u32(t: torch.Tensor) -> np.ndarray:
    """Host numpy uint32 view of a key tensor (copies from the device if needed)."""
    return t.detach().to("cpu").contiguous().numpy().view(np.uint32)


@dataclass
class ArraySpec:
    n: int
    U: int
    dist: str  # "uniform" or "zipf"
    s: float
    seed: int

    def keys(self, device: str = "cpu") -> torch.Tensor:
        if self.dist == "uniform":
            return uniform(self.n, self.U, self.seed, device)
        return zipf(self.n, self.U, self.s, self.seed, device)


def batch_spec(count: int = 4096, seed: int = BASE_SEED + 3, n_lo: int = 2**10,
               n_hi: int = 2**22, e_lo: int = 10, e_hi: int = 20, s: float = 1.1) -> List[ArraySpec]:
    rng = np.random.default_rng(seed)
    n = np.rint(np.exp(rng.uniform(math.log(n_lo), math.log(n_hi), count))).astype(np.int64)
    e = rng.integers(e_lo, e_hi + 1, count)
    zipf_sel = np.zeros(count, dtype=bool)
    zipf_sel[rng.permutation(count)[: count // 2]] = True
    return [ArraySpec(int(n[i]), 1 << int(e[i]), "zipf" if zipf_sel[i] else "uniform", s,
                      seed * 7 + 1 + i) for i in range(count)]


@dataclass
class Request:
    rid: int
    arrival: float  # seconds after the stream starts
    spec: ArraySpec


def request_stream(num: int, rate_per_s: float, seed: int = BASE_SEED + 4, n_lo: int = 2**12,
                   n_hi: int = 2**24, s: float = 1.2) -> List[Request]:
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate_per_s, num)
    arrivals = np.cumsum(gaps) - gaps[0]
    n = np.rint(np.exp(rng.uniform(math.log(n_lo), math.log(n_hi), num))).astype(np.int64)
    U = np.array([2**12, 2**16, 2**20, 2**24])[rng.integers(0, 4, num)]
    z = rng.random(num) < 0.5
    return [Request(i, float(arrivals[i]),
                    ArraySpec(int(n[i]), int(U[i]), "zipf" if z[i] else "uniform", s,
                              seed * 11 + 1 + i)) for i in range(num)]
