"""Seeded synthetic inputs for the TT-completion hot path.

This module only draws random numbers and fixes shapes; it holds none of the
method's arithmetic (no gathers, contractions or factorizations), so that it
can feed both the HIP path and the CPU oracle without coupling them.  Every
array is drawn in float64 with ``numpy.random.default_rng`` (PCG64) in a fixed
order and then rounded to float32; the rounded values are the shared input
(the oracle casts them back to float64).

Workloads (all planted-low-rank stand-ins; the paper uses no public dataset):

* ``small_step``  d=4, n=8, r=4, 4096 observed entries (one full completion
  step; CPU-sized).
* ``gather_d10``  d=10, n=10, r=16, 2^20 observed entries (gather + adjoint).
* ``riemann_d10`` d=10, n=10, canonical ranks (1,10,32,...,32,10,1), 2^20
  observed entries with N(0,1) values (tangent projection and rounding).
* ``batched``     256 instances, d=8, n=16, rank per instance in {4,8,16,32},
  lognormal entry counts clipped to [1e4, 2e5].
* ``ttm_layer``   1024x1024 TT-matrix, modes 4^5 x 4^5, r=32, batch 4096.

Draw order inside one workload: point cores (mode 1..d, C order) -> planted
cores -> indices (int32, shape (d, M), uniform with replacement) -> noise /
values.  Targets are t = planted(i) + noise; evaluating planted(i) is a
gather, so this module returns the planted cores and the noise and leaves the
sum to the caller.
"""
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

F32 = np.float32


def canonical_ranks(ns, r):
    """Largest feasible uniform-rank profile: r_k = min(r, prod n_<=k, prod n_>k)."""
    d = len(ns)
    out = [1]
    for k in range(1, d):
        left = int(np.prod(ns[:k], dtype=np.float64))
        right = int(np.prod(ns[k:], dtype=np.float64))
        out.append(int(min(r, left, right)))
    out.append(1)
    return out


def uniform_ranks(d, r):
    return [1] + [r] * (d - 1) + [1]


def random_cores(rng, ns, ranks, std):
    """Cores (r_k, n_k, r_{k+1}) with i.i.d. N(0, std^2) entries, rounded to fp32."""
    return [(std * rng.standard_normal((ranks[k], ns[k], ranks[k + 1]))).astype(F32)
            for k in range(len(ns))]


def random_indices(rng, ns, M):
    """Observed multi-indices, uniform with replacement, int32 SoA (d, M)."""
    d = len(ns)
    idx = np.empty((d, M), dtype=np.int32)
    for k in range(d):
        idx[k] = rng.integers(0, ns[k], size=M, dtype=np.int32)
    return idx


@dataclass
class TTProblem:
    """One TT tensor with an observed index set and per-entry values."""
    ns: List[int]
    ranks: List[int]
    cores: List[np.ndarray]
    idx: np.ndarray
    planted: Optional[List[np.ndarray]] = None   # target TT (None when values are given directly)
    noise: Optional[np.ndarray] = None           # per-observation noise added to planted(i)
    values: Optional[np.ndarray] = None          # per-observation values (sparse gradient)
    meta: dict = field(default_factory=dict)

    @property
    def d(self):
        return len(self.ns)

    @property
    def M(self):
        return int(self.idx.shape[1])


def planted_problem(seed, ns, ranks, std, planted_rank, planted_std, M, noise_std=0.01):
    """A point X, a planted TT, uniform indices and per-observation noise."""
    rng = np.random.default_rng(seed)
    cores = random_cores(rng, ns, ranks, std)
    pr = uniform_ranks(len(ns), planted_rank)
    planted = random_cores(rng, ns, pr, planted_std)
    idx = random_indices(rng, ns, M)
    noise = (noise_std * rng.standard_normal(M)).astype(F32)
    return TTProblem(ns=list(ns), ranks=list(ranks), cores=cores, idx=idx,
                     planted=planted, noise=noise)


def small_step(M=4096):
    """d=4, n=8, r=4; X ~ N(0, 1/4); planted rank 2 ~ N(0, 1/2); 4096 entries."""
    ns = [8] * 4
    return planted_problem(1, ns, canonical_ranks(ns, 4), 0.5, 2, 1 / np.sqrt(2), M)


def gather_d10(M=1 << 20, seed=2):
    """d=10, n=10, uniform r=16; X ~ N(0, 1/16); planted rank 8 ~ N(0, 1/8)."""
    ns = [10] * 10
    return planted_problem(seed, ns, uniform_ranks(10, 16), 0.25, 8, 1 / np.sqrt(8), M)


def riemann_d10(M=1 << 20, seed=3, r=32):
    """d=10, n=10, canonical ranks for r=32; X ~ N(0, 1/32); z ~ N(0, 1)."""
    ns = [10] * 10
    rng = np.random.default_rng(seed)
    ranks = canonical_ranks(ns, r)
    cores = random_cores(rng, ns, ranks, 1 / np.sqrt(r))
    idx = random_indices(rng, ns, M)
    z = rng.standard_normal(M).astype(F32)
    return TTProblem(ns=ns, ranks=ranks, cores=cores, idx=idx, values=z)


def completion_d10(M=1 << 20, M_test=1 << 16, seed=6, r=16):
    """Riemannian completion workload: d=10, n=10, X at canonical ranks for
    r=16, X ~ N(0, 1/16); planted uniform rank 8 ~ N(0, 1/8); M observed and
    M_test held-out uniform indices; noise N(0, 0.01^2) on the observed
    entries.  Targets are formed by the caller (gather of the planted TT)."""
    ns = [10] * 10
    rng = np.random.default_rng(seed)
    ranks = canonical_ranks(ns, r)
    cores = random_cores(rng, ns, ranks, 1 / np.sqrt(r))
    planted = random_cores(rng, ns, uniform_ranks(10, 8), 1 / np.sqrt(8))
    idx = random_indices(rng, ns, M)
    noise = (0.01 * rng.standard_normal(M)).astype(F32)
    idx_test = random_indices(rng, ns, M_test)
    return TTProblem(ns=ns, ranks=ranks, cores=cores, idx=idx, planted=planted, noise=noise,
                     meta={"idx_test": idx_test})


def batched_instance(b, d=8, n=16, seed=4, rank_choices=(4, 8, 16, 32),
                     mu=np.log(50000.0), sigma=0.8, lo=10000, hi=200000):
    """Instance b of the batched workload (its own generator seeded [seed, b])."""
    rng = np.random.default_rng([seed, b])
    r = int(rank_choices[rng.integers(0, len(rank_choices))])
    M = int(np.clip(np.rint(rng.lognormal(mu, sigma)), lo, hi))
    ns = [n] * d
    cores = random_cores(rng, ns, uniform_ranks(d, r), 1 / np.sqrt(r))
    pr = max(2, r // 2)
    planted = random_cores(rng, ns, uniform_ranks(d, pr), 1 / np.sqrt(pr))
    idx = random_indices(rng, ns, M)
    noise = (0.01 * rng.standard_normal(M)).astype(F32)
    return TTProblem(ns=ns, ranks=uniform_ranks(d, r), cores=cores, idx=idx,
                     planted=planted, noise=noise, meta=dict(instance=b, rank=r))


def batched(count=256, **kw):
    return [batched_instance(b, **kw) for b in range(count)]


@dataclass
class TTMProblem:
    row_modes: List[int]
    col_modes: List[int]
    ranks: List[int]
    cores: List[np.ndarray]     # (r_k, m_k, n_k, r_{k+1})
    X: np.ndarray               # (B, prod n)
    dY: np.ndarray              # (B, prod m)


def ttm_layer(B=4096, seed=5, modes=(4, 4, 4, 4, 4), r=32):
    """1024x1024 TT-matrix layer: cores ~ N(0, 1/r); X, dY ~ N(0, 1)."""
    rng = np.random.default_rng(seed)
    d = len(modes)
    ranks = uniform_ranks(d, r)
    std = 1 / np.sqrt(r)
    cores = [(std * rng.standard_normal((ranks[k], modes[k], modes[k], ranks[k + 1]))).astype(F32)
             for k in range(d)]
    N = int(np.prod(modes))
    X = rng.standard_normal((B, N)).astype(F32)
    dY = rng.standard_normal((B, N)).astype(F32)
    return TTMProblem(list(modes), list(modes), ranks, cores, X, dY)


def random_tt(seed, ns, ranks, std=1.0):
    """A generic random TT (fp32-rounded) for tests of any shape."""
    return random_cores(np.random.default_rng(seed), ns, ranks, std)
