"""MinJoin benchmark on one MI355X.

One step = one full join (every stage of the hot path: per-string setup, anchors,
partition records, sort, group and filter, dedup, banded verification, output) over
the long-read DNA workload: 50,000 strings, lengths N(5000, 800) clipped to
[2000, 9000], 5,000 hidden seeds x 10 copies with 1-6% edits (insertions .5,
deletions .3, substitutions .2), K = 150, q = 5, T = ceil(K / 2).  The strings are
resident in HBM before the timed region; the timed region ends when the sorted output
pairs are on the host.

Prints one JSON line: strings joined/s (value), verified candidate pairs/s, recall
against the intra-cluster ground truth, the roofline of the dominant kernel (timed with
HIP events inside the library, on the launching stream) and the CPU oracle timed on a
bounded sample of the same workload.
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "strings joined/s + verified candidate pairs/s at exact recall; batched vs plain GPU"

# MI355X figures used for the roofline.
HBM_PEAK_GBS = 8000.0
CUS, LANES, CLOCK_GHZ = 256, 64, 2.4
INT_PEAK_TOPS = CUS * LANES * CLOCK_GHZ / 1e3  # 39.32 T int32 lane-ops/s
# 32-bit operations of one word-column of the banded bit-vector recurrence (Myers'
# update over 32 rows: 13) plus the match mask for a 2-plane alphabet (2 XNOR + 1 AND):
# 16 operations per 32 band cells.
OPS_PER_WORD_COLUMN = 16

WORKLOADS = {
    "dna_long": dict(q=5, k=150, t_div=2, sigma=4,
                     desc="dna_long: 50,000 DNA strings, lengths N(5000,800) clipped to "
                          "[2000,9000], 5,000 seeds x 10 copies, 1-6% edits "
                          "(ins .5/del .3/sub .2), K=150, q=5, T=ceil(K/2)"),
    "dna_small": dict(q=4, k=60, t_div=1, sigma=4,
                      desc="dna_small: 1,000 DNA strings, 100 seeds x 10 copies, lengths "
                           "U[800,1200], 2-10% edits, K=60, q=4, T=K"),
}


def make(workload, n_clusters=None):
    from paper_1810_08833_amd import datagen as dg
    if workload == "dna_long":
        return dg.dna_long() if n_clusters is None else dg.dna_long(n_clusters=n_clusters)
    return dg.dna_small() if n_clusters is None else dg.dna_small(n_clusters=n_clusters)


def intra_cluster_pairs(S):
    order = np.argsort(S.cluster, kind="stable")
    cl = S.cluster[order]
    out = []
    start = 0
    while start < len(order):
        end = start
        while end < len(order) and cl[end] == cl[start]:
            end += 1
        if cl[start] >= 0:
            ids = np.sort(order[start:end])
            a, b = np.triu_indices(len(ids), 1)
            out.append((ids[a].astype(np.uint64) << np.uint64(32)) | ids[b].astype(np.uint64))
        start = end
    return np.concatenate(out) if out else np.zeros(0, np.uint64)


def file_sha(path):
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def measured_traffic(kernel_src):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it was taken
    on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", "verify_traffic_dna_long.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    if t.get("source_sha256") != file_sha(kernel_src):
        return None
    return t.get("bytes_per_launch")


def cpu_baseline(workload, cfg, clusters):
    import oracle
    S = make(workload, n_clusters=clusters)
    p = oracle.make_params(cfg["q"], cfg["sigma"], k=cfg["k"], t_div=cfg["t_div"])
    threads = oracle.max_threads()
    t0 = time.perf_counter()
    _, out, st = oracle.join(S.chars, S.offsets, p)
    dt = time.perf_counter() - t0
    return {"value": S.n / dt, "unit": "strings/s", "cores": threads, "kind": "oracle",
            "sample": "%s with %d seed clusters (%d strings, %d symbols): full join incl. "
                      "verification of %d candidates in %.1f s"
                      % (workload, clusters, S.n, int(S.offsets[-1]), st["candidates"], dt)}


def copy_calibration(gib):
    """A plain device copy of known size, for scaling rocprofv3 FETCH/WRITE counters."""
    import torch
    n = int(gib * (1 << 30))
    a = torch.empty(n, dtype=torch.uint8, device="cuda").fill_(1)
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": n, "launches": 3}))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="dna_long", choices=sorted(WORKLOADS))
    ap.add_argument("--t-div", type=int, default=None)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-clusters", type=int, default=1000)
    ap.add_argument("--copy-calibration", type=float, default=0.0,
                    help="only run a plain copy of this many GiB (rocprofv3 counter scale)")
    args = ap.parse_args()

    if args.gpus != 1:
        print("bench.py runs on one GPU only: the build has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration > 0:
        copy_calibration(args.copy_calibration)
        return

    import torch
    import paper_1810_08833_amd as mj

    cfg = dict(WORKLOADS[args.workload])
    if args.t_div is not None:
        cfg["t_div"] = args.t_div
    torch.cuda.set_device(0)
    S = make(args.workload)
    print("[bench] workload %s: %d strings, %d symbols" % (args.workload, S.n, S.offsets[-1]),
          file=sys.stderr, flush=True)
    ds = mj.DeviceStrings.from_host(S.chars, S.offsets, S.sigma)
    params = mj.Params(q=cfg["q"], k=cfg["k"], t_div=cfg["t_div"])
    ctx = mj.Context(0)

    # ground truth for recall (outside the timed region): every intra-cluster pair with
    # ED <= K, decided by the verifier; copies of different seeds are unrelated random
    # strings, far beyond K
    truth_pairs = intra_cluster_pairs(S)
    flags = mj.verify(ds, params, truth_pairs, ctx=ctx)
    truth = truth_pairs[flags]

    out = None
    for _ in range(args.warmup):
        out, st = mj.join(ds, params, ctx=ctx)
    torch.cuda.synchronize()
    stats = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        out, st = mj.join(ds, params, ctx=ctx)
        stats.append(st)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms = dt * 1e3 / args.steps
    print("[bench] %d steps in %.3f s" % (args.steps, dt), file=sys.stderr, flush=True)

    recall = float(np.isin(truth, out).mean()) if len(truth) else 1.0
    last = stats[-1]
    verify_ms = np.mean([s["stage_ms"]["verify"] for s in stats])
    kms = {k: float(np.sum([s["kernel_ms"][k] for s in stats])) for k in mj.KERNELS}
    kln = {k: int(np.sum([s["kernel_launches"][k] for s in stats])) for k in mj.KERNELS}
    dominant = max(kms, key=kms.get)

    # roofline of the dominant kernel
    src = os.path.join(ROOT, "paper_1810_08833_amd", "csrc", "verify.hip")
    if dominant == "verify":
        cells = float(np.sum([s["band_cells"] for s in stats]))
        ops = cells / 32.0 * OPS_PER_WORD_COLUMN
        achieved = ops / (kms["verify"] * 1e-3) / 1e12
        traffic = measured_traffic(src)
        roof = {"kernel": "k_verify_bp", "bound": "alu", "achieved": achieved,
                "peak": INT_PEAK_TOPS, "unit": "Tops/s", "frac": achieved / INT_PEAK_TOPS,
                "traffic": traffic,
                "avg_launch_ms": kms["verify"] / max(1, kln["verify"]),
                "band_cells_per_s": cells / (kms["verify"] * 1e-3)}
    else:
        pos = float(np.sum([s["positions"] for s in stats]))
        # the anchor kernel reads each symbol once and writes one bit per position
        byts = pos * (1.0 + 1.0 / 8)
        achieved = byts / (kms[dominant] * 1e-3) / 1e9
        roof = {"kernel": "k_anchor_tiles", "bound": "hbm", "achieved": achieved,
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                "traffic": None, "avg_launch_ms": kms[dominant] / max(1, kln[dominant])}

    line = {
        "metric": METRIC,
        "value": S.n / (ms * 1e-3),
        "unit": "strings/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": cfg["desc"], "strings": S.n, "symbols": int(S.offsets[-1]),
                   "K": cfg["k"], "q": cfg["q"], "t_div": cfg["t_div"], "path": "plain"},
        "verified_pairs_per_s": last["candidates"] / (verify_ms * 1e-3),
        "candidates": last["candidates"],
        "output_pairs": int(len(out)),
        "recall": recall,
        "true_pairs": int(len(truth)),
        "records": last["records"],
        "stage_ms": {k: float(np.mean([s["stage_ms"][k] for s in stats])) for k in mj.STAGES[:7]},
        "kernel_ms_per_step": {k: kms[k] / args.steps for k in kms},
        "roofline": roof,
    }
    if not args.no_cpu_baseline:
        print("[bench] timing the CPU oracle on a sample", file=sys.stderr, flush=True)
        line["cpu_baseline"] = cpu_baseline(args.workload, cfg, args.cpu_clusters)
    else:
        line["cpu_baseline"] = None
    print(json.dumps(line))


if __name__ == "__main__":
    main()
