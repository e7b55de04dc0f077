"""Seeded synthetic workloads for the gapped k-mer kernel.

This module only draws inputs; it holds none of the kernel's arithmetic and
imports nothing from the GPU library or the oracle, so both sides can be fed
the same arrays.  The paper's datasets (ENCODE DNA, SCOP protein, Stanford
Sentiment / WebKB text; Section 3.1, Table 3) are not available, so each
workload draws sequences with the shape of one of them:

* ``dna``      -- N=200, l=100, Sigma=4 iid uniform, g=6, k=4 (ENCODE-like
                  100-bp windows, Table 3; the Fig. 5(c) l=100 setting).
* ``protein``  -- N=3312 (the SCOP 1.34 size, Table 3), l ~ U{50..500},
                  Sigma=20 with a Zipf(s=1.1) symbol composition, g=7, k=4.
* ``text``     -- N=2000, l ~ U{200..1000}, Sigma=36 (26 letters + 10 digits,
                  Section S:3.2) from a first-order Markov chain whose rows are
                  Dirichlet(0.3) draws, g=10, k=4 (M=6).
* ``batched``  -- 64 independent Gram jobs: N ~ U{100..2000},
                  Sigma ~ U{4,20,36}, l ~ U{50..600}, g ~ U{6..10},
                  k ~ U{3..g-2}, iid uniform symbols.
* ``serving``  -- a resident DNA set of 20000 sequences of length 200
                  (Sigma=4, g=10, k=6), dual coefficients ~ N(0,1), bias 0;
                  queries of length U{50..1000} arriving as a Poisson stream.

Every draw uses ``numpy.random.default_rng(seed)``; the default seeds are
fixed so that every run sees the same inputs.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

SEED_BASE = 17040746800


@dataclass
class GramInput:
    name: str
    seqs: np.ndarray  # int8, concatenated symbol codes
    lens: np.ndarray  # int32 [N]
    sigma: int
    g: int
    k: int
    labels: np.ndarray | None = None
    meta: dict = field(default_factory=dict)

    @property
    def N(self) -> int:
        return int(len(self.lens))

    @property
    def M(self) -> int:
        return self.g - self.k

    def seq(self, i: int) -> np.ndarray:
        off = int(np.sum(self.lens[:i], dtype=np.int64))
        return self.seqs[off:off + int(self.lens[i])]

    def subset(self, idx) -> "GramInput":
        idx = list(idx)
        parts = [self.seq(i) for i in idx]
        seqs = np.concatenate(parts) if parts else np.zeros(0, dtype=np.int8)
        lens = np.array([len(p) for p in parts], dtype=np.int32)
        lab = None if self.labels is None else self.labels[idx]
        return GramInput(self.name + "[sub]", seqs.astype(np.int8), lens, self.sigma, self.g,
                         self.k, lab, dict(self.meta))


def _pack(parts) -> tuple[np.ndarray, np.ndarray]:
    lens = np.array([len(p) for p in parts], dtype=np.int32)
    seqs = (np.concatenate(parts) if len(parts) else np.zeros(0)).astype(np.int8)
    return seqs, lens


def iid_uniform(rng, n, lens, sigma):
    return [rng.integers(0, sigma, size=int(l)).astype(np.int8) for l in lens]


def zipf_composition(rng, lens, sigma, s):
    ranks = np.arange(1, sigma + 1, dtype=np.float64)
    p = ranks ** (-s)
    p /= p.sum()
    return [rng.choice(sigma, size=int(l), p=p).astype(np.int8) for l in lens]


def markov_chain(rng, lens, sigma, alpha):
    """First-order chain: one Dirichlet(alpha) transition row per symbol, first
    symbol uniform; all sequences are stepped together."""
    trans = rng.dirichlet(np.full(sigma, alpha), size=sigma)
    cum = np.cumsum(trans, axis=1)
    cum[:, -1] = 1.0
    n = len(lens)
    L = int(max(lens)) if n else 0
    x = np.zeros((n, max(L, 1)), dtype=np.int64)
    if L:
        x[:, 0] = rng.integers(0, sigma, size=n)
        u = rng.random((n, L))
        for i in range(1, L):
            x[:, i] = np.minimum((cum[x[:, i - 1]] <= u[:, i:i + 1]).sum(axis=1), sigma - 1)
    return [x[j, :int(l)].astype(np.int8) for j, l in enumerate(lens)]


def dna(N: int = 200, length: int = 100, g: int = 6, k: int = 4, seed: int = SEED_BASE + 0) -> GramInput:
    rng = np.random.default_rng(seed)
    lens = np.full(N, length, dtype=np.int32)
    seqs, lens = _pack(iid_uniform(rng, N, lens, 4))
    labels = np.array([1] * (N // 2) + [-1] * (N - N // 2), dtype=np.int8)
    rng.shuffle(labels)
    return GramInput("dna", seqs, lens, 4, g, k, labels)


def protein(N: int = 3312, lmin: int = 50, lmax: int = 500, g: int = 7, k: int = 4,
            seed: int = SEED_BASE + 1) -> GramInput:
    rng = np.random.default_rng(seed)
    lens = rng.integers(lmin, lmax + 1, size=N)
    seqs, lens = _pack(zipf_composition(rng, lens, 20, 1.1))
    return GramInput("protein", seqs, lens, 20, g, k)


def text(N: int = 2000, lmin: int = 200, lmax: int = 1000, g: int = 10, k: int = 4,
         seed: int = SEED_BASE + 2) -> GramInput:
    rng = np.random.default_rng(seed)
    lens = rng.integers(lmin, lmax + 1, size=N)
    seqs, lens = _pack(markov_chain(rng, lens, 36, 0.3))
    return GramInput("text", seqs, lens, 36, g, k)


def batched(n_jobs: int = 64, nmin: int = 100, nmax: int = 2000, lmin: int = 50, lmax: int = 600,
            seed: int = SEED_BASE + 3) -> list[GramInput]:
    """Uneven Gram jobs; job j is drawn from its own generator (seed + 1000 * (j + 1))."""
    jobs = []
    for j in range(n_jobs):
        rng = np.random.default_rng(seed + 1000 * (j + 1))
        N = int(rng.integers(nmin, nmax + 1))
        sigma = int(rng.choice([4, 20, 36]))
        g = int(rng.integers(6, 11))
        k = int(rng.integers(3, g - 1))
        lens = rng.integers(lmin, lmax + 1, size=N)
        seqs, lens = _pack(iid_uniform(rng, N, lens, sigma))
        jobs.append(GramInput("job%02d" % j, seqs, lens, sigma, g, k))
    return jobs


@dataclass
class ServingInput:
    sv: GramInput
    alpha: np.ndarray  # float64 [n_sv] dual coefficients (alpha_i * y_i)
    bias: float


def serving_resident(n_sv: int = 20000, length: int = 200, g: int = 10, k: int = 6,
                     seed: int = SEED_BASE + 4) -> ServingInput:
    rng = np.random.default_rng(seed)
    lens = np.full(n_sv, length, dtype=np.int32)
    seqs, lens = _pack(iid_uniform(rng, n_sv, lens, 4))
    alpha = rng.standard_normal(n_sv)
    return ServingInput(GramInput("serving_sv", seqs, lens, 4, g, k), alpha, 0.0)


def serving_queries(n_q: int, lmin: int = 50, lmax: int = 1000, sigma: int = 4,
                    seed: int = SEED_BASE + 5) -> tuple[np.ndarray, np.ndarray]:
    rng = np.random.default_rng(seed)
    lens = rng.integers(lmin, lmax + 1, size=n_q)
    return _pack(iid_uniform(rng, n_q, lens, sigma))


def poisson_arrivals(n: int, rate_per_s: float, seed: int = SEED_BASE + 6) -> np.ndarray:
    """Arrival times (seconds from 0) of a Poisson stream of the given rate."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate_per_s, size=n))


def random_small(rng, N, lmin, lmax, sigma):
    """Tiny iid inputs for brute-force pins and edge cases."""
    lens = rng.integers(lmin, lmax + 1, size=N)
    return _pack(iid_uniform(rng, N, lens, sigma))


CONFIGS = {
    "dna": dna,
    "protein": protein,
    "text": text,
}
