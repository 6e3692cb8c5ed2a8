"""Writes tests/golden/full_size.json: the oracle's candidate and output pair sets on the
five full-size synthetic workloads, as counts and SHA-256 digests of the sorted
little-endian uint64 arrays (pair = first id << 32 | second id).

Calls only the oracle and the seeded input generators.  Each workload's parameters are
stored beside its digests; the GPU tests read them from the JSON, so the two sides run
the same configuration.  The thresholds T (t_div, reps) are the ones that give 100%
recall against the ground truth, which the script also records: all intra-cluster
pairs within the pair threshold for the joins, and each mutated query against its
source string for search.

Usage:  python tests/golden/make_full_size.py [workload ...]   (a few minutes each)
"""
import hashlib
import itertools
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_1810_08833_amd import datagen as dg  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "full_size.json")

# name -> generator and parameters.  K is uniform ("k") or a fraction of the length
# ("k_frac" = (num, den): K_i = ceil(num/den * m_i)).
JOINS = {
    "dna_small": dict(q=4, sigma=4, k=60, t_div=1, reps=1),
    "dna_long": dict(q=5, sigma=4, k=150, t_div=2, reps=1),
    "protein": dict(q=4, sigma=25, k_frac=[8, 100], t_div=1, reps=7),
    "text": dict(q=6, sigma=37, k=120, t_div=2, reps=4),
}
SEARCH = {
    "dna_index_search": dict(q=5, sigma=4, k_frac=[1, 10], t_div=2, reps=1, index_strings=1_000_000,
                             queries=4096, rate_per_s=2000.0),
}


def digest(a) -> str:
    return hashlib.sha256(np.ascontiguousarray(a, dtype="<u8").tobytes()).hexdigest()


def k_args(cfg, lengths):
    if "k_frac" in cfg:
        return dict(k_per_string=dg.k_fraction(lengths, *cfg["k_frac"]))
    return dict(k=cfg["k"])


def intra_cluster(S):
    cl = S.cluster
    out = []
    for c in np.unique(cl[cl >= 0]):
        ids = np.nonzero(cl == c)[0]
        out += [(int(a) << 32) | int(b) for a, b in itertools.combinations(sorted(ids), 2)]
    return np.array(sorted(out), dtype=np.uint64)


def run_join(name, cfg):
    S = getattr(dg, name)()
    p = oracle.make_params(cfg["q"], cfg["sigma"], t_div=cfg["t_div"], reps=cfg["reps"],
                           **k_args(cfg, S.lengths()))
    t = time.time()
    cand, out, st = oracle.join(S.chars, S.offsets, p)
    secs = time.time() - t
    tp = intra_cluster(S)
    truth = tp[oracle.verify_list(S.chars, S.offsets, p, tp)]
    found = np.intersect1d(truth, out).size
    return dict(cfg, strings=int(S.n), symbols=int(S.offsets[-1]),
                candidates=int(cand.size), candidates_sha256=digest(cand),
                output=int(out.size), output_sha256=digest(out),
                true_pairs=int(truth.size), recall=found / max(1, truth.size),
                oracle_seconds=round(secs, 1), oracle_threads=oracle.max_threads())


def run_search(name, cfg):
    I = dg.dna_index(n=cfg["index_strings"])
    Q, src, _ = dg.dna_queries(I, n=cfg["queries"], rate_per_s=cfg["rate_per_s"])
    ip = oracle.make_params(cfg["q"], cfg["sigma"], t_div=cfg["t_div"], reps=cfg["reps"],
                            **k_args(cfg, I.lengths()))
    qp = oracle.make_params(cfg["q"], cfg["sigma"], t_div=cfg["t_div"], reps=cfg["reps"],
                            **k_args(cfg, Q.lengths()))
    t = time.time()
    cand, out = oracle.search(I.chars, I.offsets, ip, Q.chars, Q.offsets, qp)
    secs = time.time() - t
    kq = dg.k_fraction(Q.lengths(), *cfg["k_frac"])
    truth = [(int(i) << 32) | int(src[i]) for i in np.nonzero(src >= 0)[0]
             if oracle.ed_within(Q.get(int(i)), I.get(int(src[i])), int(kq[i]))]
    found = np.intersect1d(np.array(truth, dtype=np.uint64), out).size
    return dict(cfg, index_symbols=int(I.offsets[-1]), query_symbols=int(Q.offsets[-1]),
                candidates=int(cand.size), candidates_sha256=digest(cand),
                output=int(out.size), output_sha256=digest(out),
                true_pairs=len(truth), recall=found / max(1, len(truth)),
                oracle_seconds=round(secs, 1), oracle_threads=oracle.max_threads())


def main(names):
    oracle.build()
    res = json.load(open(OUT)) if os.path.exists(OUT) else {}
    for name in names or list(JOINS) + list(SEARCH):
        t = time.time()
        res[name] = run_join(name, JOINS[name]) if name in JOINS else run_search(name, SEARCH[name])
        print(name, json.dumps(res[name]), "(%.0f s)" % (time.time() - t), flush=True)
        with open(OUT, "w") as f:
            json.dump(res, f, indent=1, sort_keys=True)
            f.write("\n")


if __name__ == "__main__":
    main(sys.argv[1:])
