"""Seeded synthetic string collections for the MinJoin workloads.

This module only draws inputs: random symbols, lengths and i.i.d. edits.  It holds
none of MinJoin's arithmetic, so both the GPU library's tests and the CPU oracle can
use it.  All randomness comes from NumPy's PCG64 seeded with the workload's data seed.

A collection is a ``Strings`` tuple: ``chars`` (uint8 symbol codes), ``offsets``
(int64, n+1), ``sigma`` (alphabet size) and ``cluster`` (int32 cluster id per string,
-1 for strings that belong to no cluster).

Workloads (shapes of the paper's datasets, Table 5; the datasets themselves are not
reproduced):
  dna_small  1,000 DNA strings: 100 seeds of length U[800,1200] x 10 copies, per-copy
             edit rate U[2%,10%], insertion/deletion/substitution equally likely.
  dna_long   50,000 DNA strings: 5,000 seeds, lengths N(5000,800) clipped to
             [2000,9000] x 10 copies, rate U[1%,6%], ins .5 / del .3 / sub .2.
  protein    200,000 strings over 25 letters with Zipf(1.1) letter frequencies,
             lengths lognormal(ln 400, 0.8) clipped to [50,5000]; 20% are cluster
             members (seeds x 10 copies, rate U[3%,12%]).
  text       300,000 strings over 37 symbols with Zipf(1.0) frequencies, lengths
             N(1200,300) clipped to [300,3000]; 10% cluster members, rate U[2%,10%].
  dna_index  index of uniform random DNA strings with lengths U[1000,10000], plus a
             query stream: half mutated copies (rate U[5%,15%]) of random indexed
             strings, half fresh random strings, Poisson arrivals.
"""
from __future__ import annotations

from typing import NamedTuple

import numpy as np


class Strings(NamedTuple):
    chars: np.ndarray
    offsets: np.ndarray
    sigma: int
    cluster: np.ndarray

    @property
    def n(self) -> int:
        return len(self.offsets) - 1

    def lengths(self) -> np.ndarray:
        return np.diff(self.offsets)

    def get(self, i: int) -> np.ndarray:
        return self.chars[self.offsets[i]:self.offsets[i + 1]]

    def subset(self, ids) -> "Strings":
        ids = np.asarray(ids, dtype=np.int64)
        parts = [self.get(int(i)) for i in ids]
        return from_list(parts, self.sigma, self.cluster[ids])


def from_list(strings, sigma: int, cluster=None) -> Strings:
    lens = np.array([len(s) for s in strings], dtype=np.int64)
    offsets = np.zeros(len(strings) + 1, dtype=np.int64)
    np.cumsum(lens, out=offsets[1:])
    chars = (np.concatenate([np.asarray(s, dtype=np.uint8) for s in strings])
             if len(strings) and offsets[-1] > 0 else np.zeros(0, dtype=np.uint8))
    if cluster is None:
        cluster = np.full(len(strings), -1, dtype=np.int32)
    return Strings(chars, offsets, int(sigma), np.asarray(cluster, dtype=np.int32))


def zipf_probs(sigma: int, s: float) -> np.ndarray:
    w = np.arange(1, sigma + 1, dtype=np.float64) ** (-s)
    return w / w.sum()


def _random_symbols(rng, n, sigma, probs):
    if probs is None:
        return rng.integers(0, sigma, size=n, dtype=np.uint8)
    return rng.choice(sigma, size=n, p=probs).astype(np.uint8)


def mutate(rng, s: np.ndarray, rate: float, sigma: int, mix=(1 / 3, 1 / 3, 1 / 3),
           probs=None) -> np.ndarray:
    """Apply i.i.d. edits: each position is edited with probability ``rate``; the edit is
    an insertion (a new symbol before it), a deletion or a substitution (a different
    symbol) with probabilities ``mix``."""
    n = len(s)
    hit = rng.random(n) < rate
    kind = rng.choice(3, size=n, p=np.asarray(mix, dtype=np.float64))
    ins = hit & (kind == 0)
    dele = hit & (kind == 1)
    sub = hit & (kind == 2)
    body = s.copy()
    nsub = int(sub.sum())
    if nsub:
        body[sub] = ((body[sub].astype(np.int64) + rng.integers(1, sigma, size=nsub)) % sigma).astype(np.uint8)
    nins = int(ins.sum())
    new = _random_symbols(rng, nins, sigma, probs)
    # each source position emits: [inserted symbol] + [own symbol unless deleted]
    count = (~dele).astype(np.int64) + ins.astype(np.int64)
    out = np.empty(int(count.sum()), dtype=np.uint8)
    start = np.cumsum(count) - count
    own = ~dele
    out[start[own] + ins[own].astype(np.int64)] = body[own]
    out[start[ins]] = new
    return out


def _clustered(rng, n_clusters, copies, seed_lengths, rate_lo, rate_hi, sigma, probs, mix):
    strings, cluster = [], []
    for c in range(n_clusters):
        seed = _random_symbols(rng, int(seed_lengths[c]), sigma, probs)
        for _ in range(copies):
            rate = rng.uniform(rate_lo, rate_hi)
            strings.append(mutate(rng, seed, rate, sigma, mix, probs))
            cluster.append(c)
    return strings, cluster


def dna_small(seed: int = 1, n_clusters: int = 100, copies: int = 10) -> Strings:
    rng = np.random.Generator(np.random.PCG64(seed))
    lens = rng.integers(800, 1201, size=n_clusters)
    s, c = _clustered(rng, n_clusters, copies, lens, 0.02, 0.10, 4, None, (1 / 3, 1 / 3, 1 / 3))
    return from_list(s, 4, c)


def dna_long(seed: int = 2, n_clusters: int = 5000, copies: int = 10) -> Strings:
    rng = np.random.Generator(np.random.PCG64(seed))
    lens = np.clip(np.rint(rng.normal(5000, 800, size=n_clusters)), 2000, 9000).astype(np.int64)
    s, c = _clustered(rng, n_clusters, copies, lens, 0.01, 0.06, 4, None, (0.5, 0.3, 0.2))
    return from_list(s, 4, c)


def _members_and_singletons(rng, n, member_frac, copies, sigma, probs, length_fn, rate_lo,
                            rate_hi):
    n_members = int(round(n * member_frac))
    n_clusters = n_members // copies
    lens = length_fn(n_clusters)
    s, c = _clustered(rng, n_clusters, copies, lens, rate_lo, rate_hi, sigma, probs,
                      (1 / 3, 1 / 3, 1 / 3))
    rest = n - len(s)
    for L in length_fn(rest):
        s.append(_random_symbols(rng, int(L), sigma, probs))
        c.append(-1)
    order = rng.permutation(len(s))
    return from_list([s[i] for i in order], sigma, np.asarray(c, dtype=np.int32)[order])


def protein(seed: int = 3, n: int = 200_000) -> Strings:
    rng = np.random.Generator(np.random.PCG64(seed))
    probs = zipf_probs(25, 1.1)

    def lengths(k):
        return np.clip(np.rint(rng.lognormal(np.log(400), 0.8, size=k)), 50, 5000).astype(np.int64)

    return _members_and_singletons(rng, n, 0.2, 10, 25, probs, lengths, 0.03, 0.12)


def text(seed: int = 4, n: int = 300_000) -> Strings:
    rng = np.random.Generator(np.random.PCG64(seed))
    probs = zipf_probs(37, 1.0)

    def lengths(k):
        return np.clip(np.rint(rng.normal(1200, 300, size=k)), 300, 3000).astype(np.int64)

    return _members_and_singletons(rng, n, 0.1, 10, 37, probs, lengths, 0.02, 0.10)


def random_strings(seed: int, n: int, lo: int, hi: int, sigma: int = 4, probs=None) -> Strings:
    rng = np.random.Generator(np.random.PCG64(seed))
    lens = rng.integers(lo, hi + 1, size=n)
    return from_list([_random_symbols(rng, int(L), sigma, probs) for L in lens], sigma)


def dna_index(seed: int = 5, n: int = 1_000_000, lo: int = 1000, hi: int = 10000) -> Strings:
    """Index strings: uniform random DNA, lengths U[lo,hi].  Built in one draw."""
    rng = np.random.Generator(np.random.PCG64(seed))
    lens = rng.integers(lo, hi + 1, size=n).astype(np.int64)
    offsets = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(lens, out=offsets[1:])
    chars = rng.integers(0, 4, size=int(offsets[-1]), dtype=np.uint8)
    return Strings(chars, offsets, 4, np.full(n, -1, dtype=np.int32))


def dna_queries(index: Strings, seed: int = 50, n: int = 4096, rate_per_s: float = 2000.0,
                lo: int = 1000, hi: int = 10000):
    """Query stream over an index: half mutated copies (rate U[5%,15%]) of uniformly
    chosen indexed strings, half fresh random strings; exponential inter-arrival gaps.
    Returns (queries, source id per query or -1, arrival times in seconds)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    qs, src = [], []
    for _ in range(n):
        if rng.random() < 0.5:
            j = int(rng.integers(0, index.n))
            qs.append(mutate(rng, index.get(j), rng.uniform(0.05, 0.15), 4))
            src.append(j)
        else:
            qs.append(rng.integers(0, 4, size=int(rng.integers(lo, hi + 1)), dtype=np.uint8))
            src.append(-1)
    arrivals = np.cumsum(rng.exponential(1.0 / rate_per_s, size=n))
    return from_list(qs, 4, np.asarray(src, dtype=np.int32)), np.asarray(src), arrivals


def k_fraction(lengths, num: int, den: int) -> np.ndarray:
    """Per-string threshold ceil(num/den * length), in integers (a workload definition)."""
    lengths = np.asarray(lengths, dtype=np.int64)
    return ((lengths * num + den - 1) // den).astype(np.int32)


WORKLOADS = {
    "dna_small": dict(make=dna_small, q=4, k=60, sigma=4),
    "dna_long": dict(make=dna_long, q=5, k=150, sigma=4),
    "protein": dict(make=protein, q=4, k_frac=(8, 100), sigma=25),
    "text": dict(make=text, q=6, k=120, sigma=37),
}
