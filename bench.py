"""MinJoin benchmark on one MI355X.

One step = one full join (every stage of the hot path: per-string setup, anchors,
partition records, sort, group and filter, dedup, banded verification, output) over
the text-shaped workload, the largest join that fits one GPU: 300,000 strings over 37
symbols with Zipf(1.0) frequencies, lengths N(1200, 300) clipped to [300, 3000], 10% in
clusters of 10 near-duplicates at 2-10% edits, K = 120, q = 6, T = ceil(K / 2), four
parallel repetitions.  The strings are resident in HBM before the timed region; the
timed region ends when the sorted output pairs are on the host.  The long-read DNA and
protein joins are measured the same way after it and reported under "workloads".

Prints one JSON line: strings joined/s (value), verified candidate pairs/s, recall
against the intra-cluster ground truth, the plain GPU path beside the batched one, the
roofline of the dominant kernel (timed with HIP events inside the library, on the
launching stream), the HBM rates of the partition and sort stages, and the CPU oracle
timed on a bounded sample of the same workload (all host threads and one thread, with
its stage split).
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
# 32-bit operations of one word-column of the banded bit-vector recurrence: Myers'
# update over 32 rows (13) plus the match mask of a b-bit alphabet (one XOR per bit
# plane against the broadcast query symbol, b - 1 ANDs): 13 + 2b - 1, 16 for DNA.
def ops_per_word_column(bits):
    return 13 + 2 * bits - 1


# Each workload with the T rule (t_div, reps) that gives 100% recall against its ground
# truth; cpu_sample is the bounded sample the CPU oracle is timed on.
WORKLOADS = {
    "dna_long": dict(q=5, k=150, t_div=2, reps=1, sigma=4, cpu_sample=dict(n_clusters=1000),
                     packed=True,
                     desc="dna_long: 50,000 DNA strings, lengths N(5000,800) clipped to "
                          "[2000,9000], 5,000 seeds x 10 copies, 1-6% edits "
                          "(ins .5/del .3/sub .2), K=150, q=5, T=ceil(K/2), 2-bit packed "
                          "storage on device"),
    "dna_small": dict(q=4, k=60, t_div=1, reps=1, sigma=4, cpu_sample=dict(),
                      desc="dna_small: 1,000 DNA strings, 100 seeds x 10 copies, lengths "
                           "U[800,1200], 2-10% edits, K=60, q=4, T=K"),
    "protein": dict(q=4, k_frac=(8, 100), t_div=1, reps=7, sigma=25, cpu_sample=dict(n=20000),
                    desc="protein: 200,000 strings over 25 letters (Zipf 1.1), lengths "
                         "lognormal(ln 400, 0.8) clipped to [50,5000], 20% in clusters of 10 "
                         "at 3-12% edits, K_i=ceil(0.08 m_i), q=4, T=K_i, 7 repetitions"),
    "text": dict(q=6, k=120, t_div=2, reps=4, sigma=37, cpu_sample=dict(n=30000),
                 desc="text: 300,000 strings over 37 symbols (Zipf 1.0), lengths N(1200,300) "
                      "clipped to [300,3000], 10% in clusters of 10 at 2-10% edits, K=120, "
                      "q=6, T=ceil(K/2), 4 repetitions"),
}


def make(workload, **kw):
    from paper_1810_08833_amd import datagen as dg
    return getattr(dg, workload)(**kw)


def k_of(cfg, lengths):
    from paper_1810_08833_amd import datagen as dg
    if "k_frac" in cfg:
        return dict(k_per_string=dg.k_fraction(lengths, *cfg["k_frac"]))
    return dict(k=cfg["k"])


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


def measured_traffic(workload, kernel, kernel_src):
    """HBM bytes per launch of `kernel` (the label the roofline reports) on `workload`, from
    the committed rocprofv3 counter summary, if the counters were taken on the current
    source of that kernel; else None."""
    path = os.path.join(ROOT, "profiles", "traffic_%s.json" % workload)
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    name = os.path.basename(kernel_src)
    if t.get("source_sha256", {}).get(name) != file_sha(kernel_src):
        return None
    return t.get("bytes_per_launch", {}).get(kernel)


def measured_valu(workload, kernel):
    """VALU counters of the dominant kernel on `workload` (rocprofv3 SQ_INSTS_VALU,
    SQ_ACTIVE_INST_VALU, SQ_THREAD_CYCLES_VALU, GRBM_GUI_ACTIVE; profiles/valu_<workload>.md
    gives the commands and definitions), if they were taken on the current sources and
    for this kernel; else None."""
    path = os.path.join(ROOT, "profiles", "valu_%s.json" % workload)
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    csrc = os.path.join(ROOT, "paper_1810_08833_amd", "csrc")
    for name, sha in t.get("source_sha256", {}).items():
        p = os.path.join(csrc, name)
        if not os.path.exists(p) or file_sha(p) != sha:
            return None
    d = t.get("dominant")
    if not d or d.get("kernel") != kernel:
        return None
    return {"valu_busy": d["valu_busy"], "lane_ops_frac_of_peak": d["frac_of_int32_peak"],
            "lane_instr_per_%s" % d["unit"].replace(" ", "_"): d["lane_instr_per_unit"],
            "source": "profiles/valu_%s.md" % workload}


def roofline(kernel, stats, kms, kln, bits, q, workload):
    """Achieved algorithmic rate of `kernel` over the timed steps against its bound.
    Integer ALU kernels count 32-bit operations of the plain algorithm per unit of work:
      verify : 13 + 2b - 1 per 32 band cells (Myers' word update + b-plane match mask)
      anchors: per position, 42 with the 64-bit hash (rolling code 5, SplitMix64 output
               function 23, strict-minimum test on 64-bit values 14), 10 with the rank
               table of small code spaces (code 3, lookup 1, test on 32-bit values 6)
      records: per symbol 17 (one Horner step modulo 2^61 - 1), per record 23 (mixer)
    Emission is memory bound: 32 bytes per pair test (two payloads, two lengths and two
    thresholds)."""
    secs = kms[kernel] * 1e-3
    n_launch = max(1, kln[kernel])
    tot = lambda f: float(np.sum([s[f] for s in stats]))
    csrc = os.path.join(ROOT, "paper_1810_08833_amd", "csrc")
    r = {"kernel": kernel, "avg_launch_ms": kms[kernel] / n_launch, "traffic": None}
    if kernel == "verify":
        cells = tot("band_cells")
        ops = cells / 32.0 * ops_per_word_column(bits)
        last = stats[-1]
        planes = {1: 2, 2: 2, 3: 4, 4: 4, 5: 6, 6: 6}.get(bits, 8)
        if last["verify_group"] == -2:  # two lanes per pair, split by text columns
            kname, vcfg = "k_verify_bidir", "<%d, %d>" % (last["verify_words"], planes)
        elif last["verify_group"] == -3:  # each pair's window by its band class
            kname, vcfg = "k_verify_classes", "<%d>" % planes
        else:
            kname = "k_verify_persist"
            vcfg = "<%d, %d, %d>" % (last["verify_words"], last["verify_group"], planes)
        r.update(kernel=kname + vcfg, bound="alu", unit="Tops/s",
                 achieved=ops / secs / 1e12, peak=INT_PEAK_TOPS,
                 band_cells_per_s=cells / secs)
        r["traffic"] = measured_traffic(workload, r["kernel"], os.path.join(csrc, "verify_lg.hip"))
    elif kernel == "anchors":
        per_pos = 10 if q * bits <= 12 else 42
        r.update(kernel="k_anchor_tiles<%s>" % ("uint32_t" if per_pos == 10 else "uint64_t"),
                 bound="alu", unit="Tops/s", achieved=tot("positions") * per_pos / secs / 1e12,
                 peak=INT_PEAK_TOPS, ops_per_position=per_pos)
        r["traffic"] = measured_traffic(workload, r["kernel"], os.path.join(csrc, "partition.hip"))
    elif kernel == "records":
        ops = tot("positions") * 17 + tot("records") * 23
        r.update(kernel="k_records", bound="alu", unit="Tops/s", achieved=ops / secs / 1e12,
                 peak=INT_PEAK_TOPS)
    else:
        byts = tot("pair_tests") * 32.0
        r.update(kernel="k_emit", bound="hbm", unit="GB/s", achieved=byts / secs / 1e9,
                 peak=HBM_PEAK_GBS)
    r["frac"] = r["achieved"] / r["peak"]
    r["counters"] = measured_valu(workload, r["kernel"])
    return r


def cpu_baseline(workload, cfg, one_thread=True):
    """The oracle as it stands on the host cores: all threads (partition and verification
    run over strings and pairs in parallel, the bucket join on one thread), then one
    thread, on the same bounded sample; with the stage split of the paper's Fig. 5 (the
    input is already in memory, so there is no read stage)."""
    import oracle
    S = make(workload, **cfg["cpu_sample"])
    res = {}
    for threads in ([oracle.max_threads(), 1] if one_thread else [oracle.max_threads()]):
        p = oracle.make_params(cfg["q"], cfg["sigma"], t_div=cfg["t_div"], reps=cfg["reps"],
                               threads=threads, **k_of(cfg, S.lengths()))
        t0 = time.perf_counter()
        _, out, st = oracle.join(S.chars, S.offsets, p)
        dt = time.perf_counter() - t0
        res[threads] = (dt, st)
    threads = max(res)
    dt, st = res[threads]
    line = {"value": S.n / dt, "unit": "strings/s", "cores": threads, "kind": "oracle",
            "sample": "%s generator with %s (%d strings, %d symbols): full join incl. "
                      "verification of %d candidates in %.1f s on %d threads"
                      % (workload, cfg["cpu_sample"] or "its full size", S.n,
                         int(S.offsets[-1]), st["candidates"], dt, threads),
            "stage_s": st["stage_s"]}
    if 1 in res and threads != 1:
        dt1, st1 = res[1]
        line["one_thread"] = {"value": S.n / dt1, "unit": "strings/s", "seconds": dt1,
                              "stage_s": st1["stage_s"]}
    return line


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


def serve(args):
    """Serving: a resident index over uniform random DNA strings (lengths U[1000,10000]),
    queries replayed at their Poisson arrival times into the continuous-batching server, at
    each offered rate of the sweep.  Prints one JSON line: the capacity (the highest offered
    rate served at 90% or more with p99 within the bound), its latency, every rate's figures,
    and each batch's admission estimate against the device memory it used."""
    import torch
    import paper_1810_08833_amd as mj
    from paper_1810_08833_amd import datagen as dg
    torch.cuda.set_device(0)
    t_gen = time.perf_counter()
    S = dg.dna_index(n=args.serve_strings)
    Q, src, arrivals = dg.dna_queries(S, n=args.serve_queries, rate_per_s=args.serve_rate)
    print("[serve] index %d strings (%d symbols), %d queries, generated in %.1f s"
          % (S.n, S.offsets[-1], Q.n, time.perf_counter() - t_gen), file=sys.stderr, flush=True)
    ds = mj.DeviceStrings.from_host(S.chars, S.offsets, 4, packing=mj.PACK_2BIT)
    ki = torch.from_numpy(dg.k_fraction(S.lengths(), 1, 10)).cuda()
    torch.cuda.synchronize()
    t_b = time.perf_counter()
    index = mj.Index(ds, mj.Params(q=5, k_per_string=ki, t_div=args.serve_t_div))
    torch.cuda.synchronize()
    build_s = time.perf_counter() - t_b
    del ds
    kq = dg.k_fraction(Q.lengths(), 1, 10)
    # ground truth: each mutated query against its source, threshold K_query
    mut = np.nonzero(src >= 0)[0]
    pairs_c = dg.from_list([x for i in mut for x in (Q.get(int(i)), S.get(int(src[i])))], 4)
    kc = np.repeat(kq[mut], 2).astype(np.int32)
    pc = mj.DeviceStrings.from_host(pairs_c.chars, pairs_c.offsets, 4)
    pl = (np.arange(len(mut), dtype=np.uint64) * 2 << np.uint64(32)) | (np.arange(len(mut), dtype=np.uint64) * 2 + 1)
    within = mj.verify(pc, mj.Params(q=5, k_per_string=torch.from_numpy(kc).cuda()), pl)
    truth = {int(mut[i]): int(src[mut[i]]) for i in range(len(mut)) if within[i]}
    server = mj.Server(index, workers=args.serve_workers, max_batch=4096,
                       memory_budget=args.serve_budget_gib << 30)
    # warm-up (workspaces, verifier tuning) outside the measured replays
    for t in range(min(64, Q.n)):
        server.submit(Q.get(t), int(kq[t]), 1 << 40 | t)
    got = 0
    while got < min(64, Q.n):
        got += len(server.poll(timeout_ms=60000))
    rates = [int(r) for r in (args.serve_rates or str(args.serve_rate)).split(",")]
    p99_bound = args.serve_p99_ms

    def replay(rate):
        """The queries submitted at their Poisson arrival times, scaled to `rate`."""
        arr = (arrivals - arrivals[0]) * (args.serve_rate / rate)
        replies = []
        t0 = time.perf_counter()
        for i in range(Q.n):
            target = t0 + arr[i]
            while True:
                now = time.perf_counter()
                if now >= target:
                    break
                replies += server.poll(timeout_ms=0)
                if target - now > 0.0003:
                    time.sleep(min(0.0005, target - now - 0.0002))
            server.submit(Q.get(i), int(kq[i]), i)
        while len(replies) < Q.n:
            replies += server.poll(timeout_ms=60000)
        lat = np.array([r["done_ms"] - r["submit_ms"] for r in replies])
        first = min(r["submit_ms"] for r in replies)
        last = max(r["done_ms"] for r in replies)
        found = sum(1 for r in replies if r["tag"] in truth and truth[r["tag"]] in set(r["ids"].tolist()))
        # batches: (worker, start); their estimate against the device memory they used, and
        # the largest sum over batches in flight together
        batches = {}
        for r in replies:
            batches[(r["worker"], r["start_ms"])] = (r["done_ms"], r["batch_estimate"], r["batch_device"])
        events = sorted([(st, 1, e, d) for (w, st), (dn, e, d) in batches.items()] +
                        [(dn, -1, e, d) for (w, st), (dn, e, d) in batches.items()],
                        key=lambda x: (x[0], x[1]))
        cur_e = cur_d = peak_e = peak_d = 0
        for _, sign, e, d in events:
            cur_e += sign * e
            cur_d += sign * d
            peak_e, peak_d = max(peak_e, cur_e), max(peak_d, cur_d)
        ratio = max(d / e for (_, e, d) in batches.values())
        # the batches' query symbols and device bytes: a least-squares line
        # device = a + b * symbols
        qlen = Q.lengths()
        symd = {}
        for r in replies:
            k = (r["worker"], r["start_ms"])
            symd[k] = symd.get(k, 0) + int(qlen[r["tag"]])
        sym = np.array([symd[k] for k in batches], dtype=np.float64)
        dev = np.array([d for (_, _, d) in batches.values()], dtype=np.float64)
        fit_b, fit_a = np.polyfit(sym, dev, 1) if len(sym) > 1 else (0.0, float(dev[0]))
        return {"offered_qps": rate, "qps": Q.n / ((last - first) * 1e-3),
                "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
                "mean_batch": float(np.mean([r["batch_size"] for r in replies])),
                "max_batch": int(max(r["batch_size"] for r in replies)),
                "recall": found / max(1, len(truth)),
                "batches": len(batches),
                "max_device_over_estimate": float(ratio),
                "device_fit_bytes": {"per_batch": float(fit_a), "per_symbol": float(fit_b),
                                     "max_residual": float(np.max(dev - (fit_a + fit_b * sym)))},
                "batch_symbols_max": int(sym.max()),
                "peak_inflight_estimate_bytes": int(peak_e),
                "peak_inflight_device_bytes": int(peak_d)}

    sweep = []
    for rate in rates:
        m = replay(rate)
        sweep.append(m)
        print("[serve] offered %d q/s: %.0f q/s, p50 %.1f ms, p99 %.1f ms, mean batch %.1f, "
              "device/estimate <= %.2f" % (rate, m["qps"], m["p50_ms"], m["p99_ms"], m["mean_batch"],
                                           m["max_device_over_estimate"]),
              file=sys.stderr, flush=True)
    server.close()
    # capacity: the highest offered rate served at 90% or more of it with p99 within the bound
    ok = [m for m in sweep if m["qps"] >= 0.9 * m["offered_qps"] and m["p99_ms"] <= p99_bound]
    best = max(ok, key=lambda m: m["offered_qps"]) if ok else sweep[0]
    line = {
        "metric": "serving: queries/s with p50/p99 latency (continuous batching)",
        "value": best["qps"],
        "unit": "queries/s",
        "n_gpus": 1,
        "higher_is_better": True,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": "dna_index: %d uniform DNA strings, lengths U[1000,10000]; %d queries "
                               "(half mutated copies at 5-15%%, half random), Poisson arrivals, "
                               "K=ceil(0.1|q|), q=5, T=ceil(K/%d)" % (S.n, Q.n, args.serve_t_div),
                   "workers": args.serve_workers, "memory_budget_gib": args.serve_budget_gib},
        "capacity_qps": best["offered_qps"] if ok else None,
        "p99_bound_ms": p99_bound,
        "p50_ms": best["p50_ms"],
        "p99_ms": best["p99_ms"],
        "recall": best["recall"],
        "true_pairs": len(truth),
        "sweep": sweep,
        "admission_estimate": "8 MiB per batch + 96 bytes per query symbol + 4 KiB per query",
        "index_records": index.records,
        "index_device_bytes": index.device_bytes,
        "index_build_s": build_s,
    }
    print(json.dumps(line))


def characterise(args):
    """Synthetic analogues of the paper's characterisation (Sec. 5): the distribution of
    partitions per string around T (Fig. 2, T = 100 on long DNA, T = 25 on protein), the
    T sweep of recall and time (Figs. 3-4, T = K/5 .. K) and the stage split as K grows
    (Fig. 5), all on the GPU path.  One JSON line per measurement."""
    import torch
    import paper_1810_08833_amd as mj
    from paper_1810_08833_amd import datagen as dg
    torch.cuda.set_device(0)

    def emit(kind, **kw):
        print(json.dumps(dict(kind=kind, **kw)), flush=True)

    # Fig. 2: partitions per string at a fixed T
    for name, make_s, q, T in (("dna_long", dg.dna_long, 5, 100), ("protein", dg.protein, 4, 25)):
        S = make_s()
        ds = mj.DeviceStrings.from_host(S.chars, S.offsets, S.sigma)
        rec = mj.partition(ds, mj.Params(q=q, k=1, t_fixed=T))
        per = np.bincount(rec["sid"], minlength=S.n)
        # only strings whose radius formula gives r >= 1 (shorter ones are clamped)
        long_enough = S.lengths() - q + 1 >= 3 * T + 2
        c = per[long_enough]
        emit("partitions_per_string", workload=name, T=T, strings=int(c.size),
             excluded_short=int(S.n - c.size),
             mean=float(c.mean()), std=float(c.std()),
             quantiles={str(p): float(np.percentile(c, p)) for p in (1, 5, 25, 50, 75, 95, 99)},
             within_20pct=float(np.mean(np.abs(c - T) <= 0.2 * T)),
             cdf={str(f): float(np.mean(c <= f * T)) for f in (0.5, 0.75, 0.9, 1.0, 1.1, 1.25, 1.5)})
        del ds

    # Figs. 3-5: recall, time and stage split on long DNA for several K and T = K/t_div
    S = dg.dna_long()
    ds = mj.DeviceStrings.from_host(S.chars, S.offsets, S.sigma)
    tp = intra_cluster_pairs(S)
    for K in (100, 150, 200, 250):
        truth_ctx = mj.Context(0)
        truth = tp[mj.verify(ds, mj.Params(q=5, k=K), tp, ctx=truth_ctx)]
        for t_div in (5, 4, 3, 2, 1):
            params = mj.Params(q=5, k=K, t_div=t_div)
            ctx = mj.Context(0)
            for _ in range(2):
                out, st = mj.join(ds, params, ctx=ctx)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            stats = []
            for _ in range(3):
                out, st = mj.join(ds, params, ctx=ctx)
                stats.append(st)
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t0) * 1e3 / 3
            emit("t_sweep", workload="dna_long", K=K, t_div=t_div, T=int(-(-K // t_div)),
                 recall=float(np.isin(truth, out).mean()) if len(truth) else 1.0,
                 true_pairs=int(len(truth)), candidates=int(st["candidates"]),
                 output=int(len(out)), ms_per_join=ms,
                 stage_ms={k: float(np.mean([x["stage_ms"][k] for x in stats]))
                           for k in mj.STAGES[:7]})


def stage_hbm(workload, stats, reps, sym_bytes):
    """HBM rates of the partition and sort stages over their stage times (HIP events on the
    call's stream).  Algorithmic bytes are the least traffic the stage needs: partitioning
    reads the symbols once per repetition and writes a 16-byte record (key, string id and
    position) per partition; the sort reads and writes every record once.  Measured bytes
    are FETCH_SIZE + WRITE_SIZE of the stage's kernels in one join (rocprofv3, calibrated),
    used only when the counters were taken on the current sources."""
    total = float(np.mean([s["positions"] for s in stats])) / reps
    R = float(np.mean([s["records"] for s in stats]))
    alg = {"partition": reps * total * sym_bytes + 16.0 * R, "sort": 32.0 * R}
    meas = {}
    path = os.path.join(ROOT, "profiles", "traffic_%s.json" % workload)
    if os.path.exists(path):
        with open(path) as f:
            t = json.load(f)
        csrc = os.path.join(ROOT, "paper_1810_08833_amd", "csrc")
        fresh = all(t.get("source_sha256", {}).get(n) == file_sha(os.path.join(csrc, n))
                    for n in os.listdir(csrc) if n.endswith(".hip") or n.endswith(".h"))
        if fresh:
            meas = t.get("bytes_per_join_by_stage", {})
    out = {}
    for st in ("partition", "sort"):
        secs = float(np.mean([s["stage_ms"][st] for s in stats])) * 1e-3
        m = meas.get(st)
        out[st] = {"ms": secs * 1e3, "algorithmic_bytes": alg[st],
                   "algorithmic_GBps": alg[st] / secs / 1e9,
                   "measured_bytes": m, "measured_GBps": (m / secs / 1e9) if m else None,
                   "frac_of_hbm_peak": ((m or alg[st]) / secs / 1e9) / HBM_PEAK_GBS}
    return out


def measure_join(workload, args, steps, warmup):
    """Times `steps` joins of `workload` (after `warmup`) on the plain and the batched path
    and returns the measurement as a dict (no CPU baseline)."""
    import torch
    import paper_1810_08833_amd as mj

    cfg = dict(WORKLOADS[workload])
    if args.t_div is not None:
        cfg["t_div"] = args.t_div
    S = make(workload)
    print("[bench] workload %s: %d strings, %d symbols" % (workload, S.n, S.offsets[-1]),
          file=sys.stderr, flush=True)
    packing = mj.PACK_2BIT if cfg.get("packed") else mj.PACK_U8
    ds = mj.DeviceStrings.from_host(S.chars, S.offsets, S.sigma, packing=packing)
    kw = k_of(cfg, S.lengths())
    if "k_per_string" in kw:
        kw["k_per_string"] = torch.from_numpy(kw["k_per_string"]).cuda()
    params = mj.Params(q=cfg["q"], t_div=cfg["t_div"], reps=cfg["reps"], **kw)
    ctx = mj.Context(0)
    # the same join with the strings uploaded from pageable host memory inside the timing
    # (held on the host 2 bits per symbol when the device stores them so)
    host_words = mj.pack_2bit(S.chars) if packing == mj.PACK_2BIT else None
    torch.cuda.synchronize()
    t_up = time.perf_counter()
    for _ in range(3):
        if host_words is not None:
            du = mj.DeviceStrings.from_packed_host(host_words, S.offsets, S.sigma)
        else:
            du = mj.DeviceStrings.from_host(S.chars, S.offsets, S.sigma)
        torch.cuda.synchronize()
    upload_ms = (time.perf_counter() - t_up) * 1e3 / 3
    del du

    # ground truth for recall (outside the timed region): every intra-cluster pair with
    # ED <= K, decided by the verifier; copies of different seeds are unrelated random
    # strings, far beyond K
    # (its own context: the verifier's one-time configuration timing belongs to the join)
    truth_pairs = intra_cluster_pairs(S)
    flags = mj.verify(ds, params, truth_pairs, ctx=mj.Context(0))
    truth = truth_pairs[flags]

    def timed(verifier, streaming=True):
        params.verifier = verifier
        ctx.set_streaming(streaming)
        out = None
        for _ in range(warmup):
            out, st = mj.join(ds, params, ctx=ctx)
        torch.cuda.synchronize()
        stats = []
        t0 = time.perf_counter()
        for _ in range(steps):
            out, st = mj.join(ds, params, ctx=ctx)
            stats.append(st)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        return out, stats, dt * 1e3 / steps

    plain_out, plain_stats, plain_ms = timed(mj.VERIFY_PLAIN)
    print("[bench] %s plain: %.3f ms/step" % (workload, plain_ms), file=sys.stderr, flush=True)
    sbs_out, sbs_stats, sbs_ms = timed(mj.VERIFY_BATCHED, streaming=False)
    print("[bench] %s batched, stage by stage: %.3f ms/step" % (workload, sbs_ms), file=sys.stderr,
          flush=True)
    cap_ms, cap_joins = None, 0
    if not args.no_capture:
        cap_out, cap_stats, cap_ms = timed(mj.VERIFY_BATCHED, streaming=2)
        cap_joins = int(sum(1 for s in cap_stats if s["streamed"] == 2))
        print("[bench] %s batched, captured in HIP graphs: %.3f ms/step (%d of %d joins replayed)"
              % (workload, cap_ms, cap_joins, len(cap_stats)), file=sys.stderr, flush=True)
        assert np.array_equal(cap_out, plain_out), "captured and plain joins disagree"
    out, stats, ms = timed(mj.VERIFY_BATCHED)
    st_ms, st_joins = ms, int(sum(s["streamed"] for s in stats))
    print("[bench] %s batched, streamed: %.3f ms/step (%d of %d joins streamed)"
          % (workload, ms, st_joins, len(stats)), file=sys.stderr, flush=True)
    assert np.array_equal(out, plain_out), "batched and plain verifiers disagree"
    assert np.array_equal(sbs_out, plain_out), "stage-by-stage and plain joins disagree"
    # the headline is the faster of the batched path's two modes (both exact); the other
    # is reported beside it
    mode = "streamed"
    if sbs_ms < ms:
        out, stats, ms, mode = sbs_out, sbs_stats, sbs_ms, "stage by stage"

    recall = float(np.isin(truth, out).mean()) if len(truth) else 1.0
    last = stats[-1]
    verify_ms = np.mean([s["stage_ms"]["verify"] for s in stats])
    kms = {k: float(np.sum([s["kernel_ms"][k] for s in stats])) for k in mj.KERNELS}
    kln = {k: int(np.sum([s["kernel_launches"][k] for s in stats])) for k in mj.KERNELS}
    dominant = max(kms, key=kms.get)
    bits = int(np.ceil(np.log2(S.sigma)))
    roof = roofline(dominant, stats, kms, kln, bits, cfg["q"], workload)
    return {
        "cfg": cfg,
        "value": S.n / (ms * 1e-3),
        "ms_per_step": ms,
        "config": {"workload": cfg["desc"], "strings": S.n, "symbols": int(S.offsets[-1]),
                   "K": cfg.get("k", "ceil(%d/%d m_i)" % tuple(cfg.get("k_frac", (0, 1)))),
                   "q": cfg["q"], "t_div": cfg["t_div"], "reps": cfg["reps"], "path": "batched",
                   "storage": "2-bit packed" if cfg.get("packed") else "uint8",
                   "verify_lanes_per_pair": last["verify_group"],
                   "verify_words_per_lane": last["verify_words"],
                   "verify_workgroups": last["verify_blocks"]},
        "plain": {"value": S.n / (plain_ms * 1e-3), "ms_per_step": plain_ms,
                  "verify_kernel_ms": float(np.mean([s["kernel_ms"]["verify"] for s in plain_stats]))},
        "batched_vs_plain": plain_ms / ms,
        "batched_modes": {"streamed_ms_per_step": st_ms, "streamed_joins": st_joins,
                          "stage_by_stage_ms_per_step": sbs_ms,
                          "captured_ms_per_step": cap_ms, "captured_replays": cap_joins,
                          "headline_mode": mode,
                          "note": "the headline is the faster mode whose kernels the library "
                                  "times (captured graphs carry no kernel timers)"},
        "with_upload": {"value": S.n / ((ms + upload_ms) * 1e-3), "upload_ms": upload_ms,
                        "note": "strings uploaded from pageable host memory inside the timing"},
        "verified_pairs_per_s": last["candidates"] / (verify_ms * 1e-3),
        "candidates": last["candidates"],
        "output_pairs": int(len(out)),
        "recall": recall,
        "true_pairs": int(len(truth)),
        "records": last["records"],
        "members": last["members"],
        "member_filter": last["member_filter"],
        "pair_tests": last["pair_tests"],
        "stage_ms": {k: float(np.mean([s["stage_ms"][k] for s in stats])) for k in mj.STAGES[:7]},
        "stage_hbm": stage_hbm(workload, stats, cfg["reps"], 0.25 if cfg.get("packed") else 1.0),
        "kernel_ms_per_step": {k: kms[k] / steps for k in kms},
        "roofline": roof,
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="text", choices=sorted(WORKLOADS))
    ap.add_argument("--also", default=None,
                    help="comma-separated workloads measured after the main one (default: "
                         "dna_long,protein when the main workload is text, else none)")
    ap.add_argument("--t-div", type=int, default=None)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-capture", action="store_true",
                    help="skip the captured (HIP graph) mode, e.g. under counter collection")
    ap.add_argument("--serve", action="store_true", help="run the serving benchmark instead")
    ap.add_argument("--serve-strings", type=int, default=1_000_000)
    ap.add_argument("--serve-queries", type=int, default=4096)
    ap.add_argument("--serve-rate", type=int, default=2000)
    ap.add_argument("--serve-rates", default=None,
                    help="comma-separated offered rates (q/s) swept in turn; default --serve-rate")
    ap.add_argument("--serve-p99-ms", type=float, default=50.0,
                    help="p99 latency bound of the capacity figure")
    ap.add_argument("--serve-t-div", type=int, default=2)
    ap.add_argument("--serve-workers", type=int, default=4)
    ap.add_argument("--serve-budget-gib", type=int, default=32)
    ap.add_argument("--characterise", action="store_true",
                    help="partition counts around T, T sweep and stage split (JSON lines)")
    ap.add_argument("--copy-calibration", type=float, default=0.0,
                    help="only run a plain copy of this many GiB (rocprofv3 counter scale)")
    args = ap.parse_args()

    if args.gpus != 1:
        print("bench.py runs on one GPU only: there is no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration > 0:
        copy_calibration(args.copy_calibration)
        return
    if args.serve:
        serve(args)
        return
    if args.characterise:
        characterise(args)
        return

    import torch
    torch.cuda.set_device(0)
    also = args.also
    if also is None:
        also = "dna_long,protein" if args.workload == "text" else ""
    also = [w for w in also.split(",") if w and w != args.workload]

    m = measure_join(args.workload, args, args.steps, args.warmup)
    cfg = m.pop("cfg")
    line = {
        "metric": METRIC,
        "value": m.pop("value"),
        "unit": "strings/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": m.pop("ms_per_step"),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": m.pop("config"),
    }
    line.update(m)
    if also:
        line["workloads"] = {}
        for w in also:
            mw = measure_join(w, args, min(args.steps, 10), min(args.warmup, 3))
            mw.pop("cfg")
            line["workloads"][w] = mw
    if not args.no_cpu_baseline:
        print("[bench] timing the CPU oracle on a sample", file=sys.stderr, flush=True)
        line["cpu_baseline"] = cpu_baseline(args.workload, cfg)
    else:
        line["cpu_baseline"] = None
    print(json.dumps(line))


if __name__ == "__main__":
    main()
