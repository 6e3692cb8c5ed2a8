"""GPU parity at full size: the five synthetic workloads at the sizes and in the launch
configuration the benchmark uses, against the oracle's candidate and output pair sets.

The oracle's results are stored as counts and SHA-256 digests of the sorted uint64
pair arrays (tests/golden/full_size.json, written by tests/golden/make_full_size.py,
which calls only the oracle).  Integer work: the bar is bit-exact equality."""
import hashlib
import json
import os
import sys

import numpy as np
import pytest

from paper_1810_08833_amd import datagen as dg

pytestmark = pytest.mark.gpu

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "full_size.json")))
JOINS = [n for n in ("dna_small", "dna_long", "protein", "text") if n in GOLDEN]


def say(*a):
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


def digest(a) -> str:
    return hashlib.sha256(np.ascontiguousarray(a, dtype="<u8").tobytes()).hexdigest()


@pytest.fixture(scope="module")
def mj():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1810_08833_amd as mj
    mj.load_library()
    return mj


def params(mj, g, lengths, **kw):
    import torch
    if "k_frac" in g:
        kp = torch.from_numpy(dg.k_fraction(lengths, *g["k_frac"])).cuda()
        return mj.Params(q=g["q"], k_per_string=kp, t_div=g["t_div"], reps=g["reps"], **kw)
    return mj.Params(q=g["q"], k=g["k"], t_div=g["t_div"], reps=g["reps"], **kw)


@pytest.mark.parametrize("name", JOINS)
def test_join_full_size_identical(mj, name):
    g = GOLDEN[name]
    say(name, "full size: %d strings, t_div=%d, reps=%d" % (g["strings"], g["t_div"], g["reps"]))
    S = getattr(dg, name)()
    assert S.n == g["strings"] and int(S.offsets[-1]) == g["symbols"]
    ds = mj.DeviceStrings.from_host(S.chars, S.offsets, S.sigma)
    cand, _ = mj.candidates(ds, params(mj, g, S.lengths()))
    assert cand.size == g["candidates"]
    assert digest(cand) == g["candidates_sha256"]
    ctx = mj.Context()
    for verifier in (mj.VERIFY_BATCHED, mj.VERIFY_PLAIN, mj.VERIFY_BATCHED):
        # the second batched join is streamed (stages sized on the device)
        out, st = mj.join(ds, params(mj, g, S.lengths(), verifier=verifier), ctx=ctx)
        assert st["candidates"] == g["candidates"]
        assert out.size == g["output"], verifier
        assert digest(out) == g["output_sha256"], verifier
    assert st["streamed"] == 1
    ctx.close()


@pytest.mark.parametrize("name", [n for n in JOINS if GOLDEN[n]["sigma"] <= 4])
def test_join_full_size_identical_from_packed_input(mj, name):
    """The DNA joins with the strings stored 2 bits per symbol on the device (the layout the
    benchmark times for them)."""
    g = GOLDEN[name]
    say(name, "full size, 2-bit packed input")
    S = getattr(dg, name)()
    ds = mj.DeviceStrings.from_host(S.chars, S.offsets, S.sigma, packing=mj.PACK_2BIT)
    cand, _ = mj.candidates(ds, params(mj, g, S.lengths()))
    assert cand.size == g["candidates"] and digest(cand) == g["candidates_sha256"]
    ctx = mj.Context()
    for _ in range(2):
        out, st = mj.join(ds, params(mj, g, S.lengths()), ctx=ctx)
        assert out.size == g["output"] and digest(out) == g["output_sha256"]
    assert st["streamed"] == 1
    ctx.set_streaming(2)  # captured into HIP graphs, then replayed
    for _ in range(2):
        out, st = mj.join(ds, params(mj, g, S.lengths()), ctx=ctx)
        assert out.size == g["output"] and digest(out) == g["output_sha256"]
    assert st["streamed"] == 2
    ctx.close()


@pytest.mark.skipif("dna_index_search" not in GOLDEN, reason="no stored search result")
def test_search_full_size_identical_direct_and_served(mj):
    """1M-string index, 4096 queries: one mj_search call over all queries, and the same
    queries through the continuous-batching server, both equal the oracle's pairs."""
    import torch
    g = GOLDEN["dna_index_search"]
    say("dna_index search full size: %d index strings, %d queries" % (g["index_strings"], g["queries"]))
    I = dg.dna_index(n=g["index_strings"])
    Q, _, _ = dg.dna_queries(I, n=g["queries"], rate_per_s=g["rate_per_s"])
    assert int(I.offsets[-1]) == g["index_symbols"] and int(Q.offsets[-1]) == g["query_symbols"]
    # the index is built from the strings stored 2 bits per symbol (1.4 GB) and keeps no
    # copy of them, only the verifier's planes, lengths, thresholds and sorted records
    ds = mj.DeviceStrings.from_host(I.chars, I.offsets, 4, packing=mj.PACK_2BIT)
    index = mj.Index(ds, params(mj, g, I.lengths()))
    say("index holds %.2f GB of device memory" % (index.device_bytes / 1e9))
    assert index.device_bytes <= 6.1e9  # 1.4 GB of planes + 16 B per record, no symbols
    del ds
    torch.cuda.empty_cache()
    kq = dg.k_fraction(Q.lengths(), *g["k_frac"])
    qd = mj.DeviceStrings.from_host(Q.chars, Q.offsets, 4, packing=mj.PACK_2BIT)
    for verifier in (mj.VERIFY_BATCHED, mj.VERIFY_PLAIN):
        out, st = index.search(qd, k_per_query=torch.from_numpy(kq).cuda(), verifier=verifier)
        assert st["candidates"] == g["candidates"]
        assert out.size == g["output"] and digest(out) == g["output_sha256"], verifier
    say("served")
    srv = mj.Server(index, workers=4, max_batch=512, memory_budget=8 << 30)
    for t in range(Q.n):
        srv.submit(Q.get(t), int(kq[t]), t)
    replies = []
    while len(replies) < Q.n:
        replies += srv.poll(timeout_ms=60000)
    srv.close()
    assert all(r["status"] == 0 for r in replies)
    served = np.sort(np.concatenate(
        [(np.uint64(r["tag"]) << np.uint64(32)) | r["ids"].astype(np.uint64) for r in replies]))
    assert served.size == g["output"] and digest(served) == g["output_sha256"]
    assert max(r["batch_size"] for r in replies) > 1
