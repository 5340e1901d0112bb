"""Seeded synthetic inputs for the Horseshoe Probit sampler.

This module only *generates inputs*: a design matrix X, a coefficient vector
beta_true and binary outcomes y.  It holds none of the sampler's arithmetic
and is shared by the tests, the benchmark, the GPU library's callers and the
oracle's callers alike.

The recipe is the paper's synthetic design (Section 6.1, Eq. 13):
x_ij ~ N(0, 1), y ~ Ber(Phi(X beta)), written as y_i = 1{x_i beta + e_i > 0}
with e_i ~ N(0, 1), which has the same law.  Optionally column 0 is set to 1
(an intercept).  X is drawn in float32; y is computed from the stored float32
X, so the outcomes follow the model for the design the sampler actually sees.

Randomness: numpy's PCG64 generator, one independent stream per block of
rows (SeedSequence.spawn), so the result does not depend on how many threads
generate it.
"""
from __future__ import annotations

import math
import os
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass, field

import numpy as np

ROW_BLOCK = 1 << 16


@dataclass
class Dataset:
    name: str
    X: np.ndarray          # N x p float32, C-contiguous
    y: np.ndarray          # N uint8 in {0, 1}
    beta_true: np.ndarray  # p float64
    seed: int
    intercept: bool
    info: dict = field(default_factory=dict)

    @property
    def N(self) -> int:
        return self.X.shape[0]

    @property
    def p(self) -> int:
        return self.X.shape[1]


def _fill_block(args):
    X, y, beta_true, intercept, ss, r0, r1 = args
    rng = np.random.Generator(np.random.PCG64(ss))
    n = r1 - r0
    xb = rng.standard_normal((n, X.shape[1]), dtype=np.float32)
    if intercept:
        xb[:, 0] = 1.0
    X[r0:r1] = xb
    eps = rng.standard_normal(n)
    eta = xb.astype(np.float64) @ beta_true
    y[r0:r1] = (eta + eps > 0.0).astype(np.uint8)


def probit_design(N: int, p: int, beta_true, seed: int, intercept: bool = True,
                  name: str = "custom", threads: int | None = None) -> Dataset:
    """X (N x p, float32, iid N(0,1), column 0 = 1 if intercept) and probit y."""
    beta_true = np.asarray(beta_true, dtype=np.float64)
    if beta_true.shape != (p,):
        raise ValueError("beta_true must have length p")
    X = np.empty((N, p), dtype=np.float32)
    y = np.empty(N, dtype=np.uint8)
    nblk = max(1, math.ceil(N / ROW_BLOCK))
    seqs = np.random.SeedSequence(seed).spawn(nblk)
    jobs = [(X, y, beta_true, intercept, seqs[b], b * ROW_BLOCK, min(N, (b + 1) * ROW_BLOCK))
            for b in range(nblk)]
    if threads is None:
        threads = min(16, os.cpu_count() or 1)
    if nblk == 1 or threads <= 1:
        for j in jobs:
            _fill_block(j)
    else:
        with ThreadPoolExecutor(max_workers=threads) as ex:
            list(ex.map(_fill_block, jobs))
    return Dataset(name, X, y, beta_true, seed, intercept)


def sparse_beta(p: int, k: int, seed: int, lo: float = -3.0, hi: float = 3.0):
    """k nonzeros ~ U(lo, hi) at indices drawn without replacement from 0..p-1."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, 7])))
    idx = np.sort(rng.choice(p, size=k, replace=False))
    beta = np.zeros(p)
    beta[idx] = rng.uniform(lo, hi, size=k)
    return beta, idx


def leading_beta(p: int, lead) -> np.ndarray:
    beta = np.zeros(p)
    lead = np.asarray(lead, dtype=np.float64)[:p]
    beta[: lead.size] = lead
    return beta


# ---- the named workloads -------------------------------------------------------
C1_LEAD = (1.3, 4.0, -1.0)
EQ13_LEAD = (1.3, 4.0, -1.0, 1.6, 5.0, -2.0)


def config1(seed: int = 11) -> Dataset:
    """N = 1000, p = 10, intercept, beta_true = (1.3, 4, -1, 0, ..., 0)."""
    d = probit_design(1000, 10, leading_beta(10, C1_LEAD), seed, True, "n1000_p10")
    return d


def config2(seed: int = 12) -> Dataset:
    """N = 100,000, p = 100, intercept, 5 nonzeros ~ U(-3, 3) at random indices."""
    beta, idx = sparse_beta(100, 5, seed)
    d = probit_design(100_000, 100, beta, seed, True, "n100000_p100")
    d.info["nonzero_idx"] = idx.tolist()
    return d


def config3(seed: int = 13) -> Dataset:
    """N = 1,000,000, p = 1000 (4 GB float32), intercept, 10 nonzeros ~ U(-3, 3)."""
    beta, idx = sparse_beta(1000, 10, seed)
    d = probit_design(1_000_000, 1000, beta, seed, True, "n1000000_p1000")
    d.info["nonzero_idx"] = idx.tolist()
    return d


def eq13(N: int, p: int, seed: int) -> Dataset:
    """The paper's own synthetic design (no intercept), Eq. (13)."""
    return probit_design(N, p, leading_beta(p, EQ13_LEAD), seed, False, f"eq13_n{N}_p{p}")


RARE_N, RARE_P, RARE_YBAR = 1_295_848, 141, 0.0048


def rare_event(seed: int = 14, N: int = RARE_N, p: int = RARE_P, ybar: float = RARE_YBAR,
               k_nonzero: int = 8) -> Dataset:
    """Shape-matched stand-in for the paper's clinical data set (Section 6.2:
    N = 1,295,848 rows, p = 141 predictors, mean(y) = 0.0048), which is not
    available: an intercept column plus p - 1 iid N(0, 1) covariates,
    k_nonzero covariate effects ~ U(-0.5, 0.5) at random indices, and the
    intercept b0 set so that E[y] = ybar.  With x beta ~ N(0, s^2) over the
    covariates, P(y = 1) = Phi(b0 / sqrt(1 + s^2)), so b0 = Phi^-1(ybar)
    sqrt(1 + s^2), s^2 = sum of the squared effects."""
    from statistics import NormalDist
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, 11])))
    beta = np.zeros(p)
    idx = np.sort(rng.choice(np.arange(1, p), size=k_nonzero, replace=False))
    beta[idx] = rng.uniform(-0.5, 0.5, size=k_nonzero)
    s2 = float(np.sum(beta[1:] ** 2))
    beta[0] = NormalDist().inv_cdf(ybar) * math.sqrt(1.0 + s2)
    d = probit_design(N, p, beta, seed, True, f"rare_n{N}_p{p}")
    d.info["nonzero_idx"] = idx.tolist()
    d.info["target_ybar"] = ybar
    return d


def batch_shapes(n_datasets: int = 64, seed: int = 1000):
    """Uneven dataset shapes: N log-uniform in [1e4, 2e5], p uniform in {50..500}."""
    rng = np.random.Generator(np.random.PCG64(seed))
    Ns = np.rint(np.exp(rng.uniform(math.log(1e4), math.log(2e5), size=n_datasets))).astype(int)
    ps = rng.integers(50, 501, size=n_datasets)
    return [(int(n), int(p)) for n, p in zip(Ns, ps)]


def batch_dataset(d: int, N: int, p: int) -> Dataset:
    """Dataset d of the uneven batch: intercept, beta_true = (1.3, 4, -1, 0, ...)."""
    return probit_design(N, p, leading_beta(p, C1_LEAD), 1000 + d, True, f"batch{d}_n{N}_p{p}")


def bf16_bits(X: np.ndarray) -> np.ndarray:
    """Round float32 to bfloat16 (nearest, ties to even) and return the bits."""
    u = np.ascontiguousarray(X, dtype=np.float32).view(np.uint32)
    if not np.all(np.isfinite(X)):
        raise ValueError("X must be finite")
    lsb = (u >> 16) & 1
    r = (u + np.uint32(0x7FFF) + lsb) >> 16
    return r.astype(np.uint16)


def bf16_to_f32(bits: np.ndarray) -> np.ndarray:
    return (bits.astype(np.uint32) << 16).view(np.float32)
