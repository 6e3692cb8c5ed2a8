"""GPU parity: the HIP path (through the C-ABI) against the CPU oracle, element by
element on the same seeded inputs.  Everything here is integer work, so the bar is
bit-exact equality."""
import sys

import numpy as np
import pytest

import oracle
from paper_1810_08833_amd import datagen as dg
from tests import worked_example as wex

pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def mj():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1810_08833_amd as mj
    mj.load_library()
    return mj


def dev(mj, S):
    return mj.DeviceStrings.from_host(S.chars, S.offsets, S.sigma)


def sort_records(keys, sids, poss, lens):
    order = np.lexsort((lens, poss, sids, keys))
    return keys[order], sids[order], poss[order], lens[order]


def assert_records_equal(got, want):
    a = sort_records(got["key"], got["sid"], got["pos"], got["len"])
    b = sort_records(want["key"], want["sid"], want["pos"], want["len"])
    assert len(a[0]) == len(b[0])
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


def mixed_collection(seed):
    """Ragged lengths: empty strings, strings shorter than q, a homopolymer run,
    duplicates, and clustered copies."""
    rng = np.random.default_rng(seed)
    base = dg.dna_small(seed=seed, n_clusters=30, copies=6)
    extra = [np.zeros(0, np.uint8), np.array([1, 2], np.uint8), np.zeros(700, np.uint8),
             np.full(64, 3, np.uint8), rng.integers(0, 4, 3).astype(np.uint8)]
    strs = [base.get(i) for i in range(base.n)] + extra + [base.get(0), base.get(5)]
    order = rng.permutation(len(strs))
    return dg.from_list([strs[i] for i in order], 4)


def heavy_cluster_collection(seed):
    """Two bases with 60 near-copies each (1% edits): groups of ~60 records, so the pair
    tests outnumber the records many times over (the emission path that builds the (m, K)
    words of every record first)."""
    rng = np.random.default_rng(seed)
    strs = []
    for c in range(2):
        base = rng.integers(0, 4, 500).astype(np.uint8)
        strs += [dg.mutate(np.random.default_rng(seed * 1000 + c * 100 + i), base, 0.01, 4)
                 for i in range(60)]
    return dg.from_list(strs, 4)


def big_group_collection(seed, sigma):
    """Near-copy clusters of 64, 65, 100, 129 and 200 strings (0.5% edits), strings of
    tandem repeats of three units at random phases and lengths, and unrelated strings:
    groups of 64 records and more, whose tests the join takes by 64 x 64 tile pairs, with
    ragged last tiles, records of one string several times in a group, and pairs that the
    length and position filter rejects."""
    rng = np.random.default_rng(seed)
    strs = []
    for c, copies in enumerate([64, 65, 100, 129, 200]):
        base = rng.integers(0, sigma, int(rng.integers(300, 600))).astype(np.uint8)
        strs += [dg.mutate(np.random.default_rng(seed * 10000 + c * 1000 + i), base, 0.005, sigma)
                 for i in range(copies)]
    units = [rng.integers(0, sigma, int(rng.integers(3, 30))).astype(np.uint8) for _ in range(3)]
    for i in range(60):
        unit, m = units[i % 3], int(rng.integers(300, 600))
        ph = int(rng.integers(0, len(unit)))
        strs.append(np.tile(unit, m // len(unit) + 2)[ph:ph + m])
    strs += [rng.integers(0, sigma, int(rng.integers(300, 600))).astype(np.uint8) for _ in range(100)]
    order = np.random.default_rng(seed + 1).permutation(len(strs))
    return dg.from_list([strs[i] for i in order], sigma)


def lazy_big_group_collection(seed, copies):
    """One cluster of near-copies (0.5% edits) among 3,000 unrelated strings: a few groups
    of 64 records or more, but fewer pair tests than records, so emission gathers each
    record's (m, K) by string id (with 70 copies from the length and K arrays, with 80
    from one packed word per string)."""
    rng = np.random.default_rng(seed)
    base = rng.integers(0, 4, 400).astype(np.uint8)
    strs = [dg.mutate(np.random.default_rng(seed * 1000 + i), base, 0.005, 4) for i in range(copies)]
    strs += [rng.integers(0, 4, int(rng.integers(600, 1000))).astype(np.uint8) for _ in range(3000)]
    order = np.random.default_rng(seed + 1).permutation(len(strs))
    return dg.from_list([strs[i] for i in order], 4)


def wide_radius_collection(seed, sigma, n=60):
    """Lengths 50..6000 at T = 2: radii from 7 to ~1000 (regions of 4096 positions, window
    blocks of 8 and 16), plus a homopolymer run (equal q-grams across whole windows)."""
    rng = np.random.default_rng(seed)
    strs = [rng.integers(0, sigma, int(rng.integers(50, 6000))).astype(np.uint8) for _ in range(n)]
    strs.insert(n // 2, np.full(3000, 1, np.uint8))
    return dg.from_list(strs, sigma)


def long_T1_collection(seed, sigma, n_bases=6, copies=3):
    """Strings of 8,000-11,000 symbols at T = 1: radii of 2,000-2,750, past what a tile
    region's halo holds (the wide anchor path), in clusters of near-copies (0.02% edits:
    with about three partitions per string, a candidate needs an unedited one), a
    homopolymer of 9,000 (no strict minimum anywhere) and shorter strings whose radii the
    tile kernel takes, in the same collection."""
    rng = np.random.default_rng(seed)
    strs = []
    for c in range(n_bases):
        base = rng.integers(0, sigma, int(rng.integers(8000, 11000))).astype(np.uint8)
        strs += [base] + [dg.mutate(np.random.default_rng(seed * 100 + 10 * c + i), base, 0.0002,
                                    sigma) for i in range(copies - 1)]
    strs.append(np.full(9000, 2, np.uint8))
    strs += [rng.integers(0, sigma, L).astype(np.uint8) for L in (0, 3, 40, 500, 3000, 7700)]
    order = rng.permutation(len(strs))
    return dg.from_list([strs[i] for i in order], sigma)


# ---------------------------------------------------------------- worked example
def test_worked_example_end_to_end(mj):
    import torch
    say("worked example")
    g, table, strings, chars, offsets = wex.load()
    ds = mj.DeviceStrings.from_host(chars, offsets, 4)
    tab = torch.from_numpy(table.view(np.int64)).cuda()
    p = mj.Params(q=3, k=4, t_fixed=3, pi_table=tab)
    rec = mj.partition(ds, p)
    parts = [[] for _ in range(5)]
    for r in sorted(rec.tolist(), key=lambda r: (r[1], r[2])):
        parts[r[1]].append(g["strings"][r[1]][r[2]:r[2] + r[3]])
    assert parts == g["partitions"]
    cand, _ = mj.candidates(ds, p)
    assert wex.pairs_1based(cand) == g["candidates_1based"]
    out, st = mj.join(ds, p)
    assert wex.pairs_1based(out) == g["output_1based"]
    assert st["candidates"] == 4 and st["output"] == 3


# ---------------------------------------------------------------- stage parity
CASES = {
    "dna_mixed_T_from_K": dict(make=lambda: mixed_collection(3), q=4, k=60, t_div=1),
    "dna_mixed_t_div3": dict(make=lambda: mixed_collection(4), q=4, k=60, t_div=3),
    "dna_reps3": dict(make=lambda: mixed_collection(5), q=5, k=40, t_div=4, reps=3),
    "dna_small_fixedT": dict(make=lambda: dg.dna_small(seed=8, n_clusters=20, copies=5), q=4,
                             k=70, t_fixed=7),
    "protein_per_string_K": dict(make=lambda: dg.protein(seed=6, n=1500), q=4, k_frac=(8, 100),
                                 t_div=1),
    "text_q6": dict(make=lambda: dg.text(seed=7, n=1500), q=6, k=120, t_div=2),
    "dna_heavy_clusters": dict(make=lambda: heavy_cluster_collection(77), q=4, k=20, t_div=1),
    "dna_big_groups": dict(make=lambda: big_group_collection(91, 4), q=4, k=20, t_div=1),
    "protein_big_groups": dict(make=lambda: big_group_collection(92, 20), q=3, k_frac=(5, 100),
                               t_div=2),
    "dna_lazy_big_group": dict(make=lambda: lazy_big_group_collection(93, 70), q=4, k=20, t_div=1),
    "dna_lazy_big_group_lk": dict(make=lambda: lazy_big_group_collection(93, 80), q=4, k=20,
                                  t_div=1),
    "dna_wide_radius": dict(make=lambda: wide_radius_collection(31, 4), q=4, k=60, t_fixed=2),
    "text_wide_radius_hashed": dict(make=lambda: wide_radius_collection(32, 37), q=6, k=60,
                                    t_fixed=2),
    "dna_T1_long_reps2": dict(make=lambda: long_T1_collection(41, 4), q=6, k=60, t_fixed=1,
                              reps=2),
    "text_T1_long_hashed": dict(make=lambda: long_T1_collection(42, 37), q=6, k=40, t_div=40),
    "alphabet12_q4": dict(make=lambda: dg.from_list(
        [dg.mutate(np.random.default_rng(900 + i), base, 0.02, 12)
         for base in [np.random.default_rng(80 + c).integers(0, 12, 600 + 37 * c).astype(np.uint8)
                      for c in range(40)] for i in range(5)], 12), q=4, k=50, t_div=2, reps=2),
}


def run_case(mj, name):
    return params_for(mj, CASES[name], CASES[name]["make"]())


def params_for(mj, c, S):
    import torch
    kw = dict(t_div=c.get("t_div", 1), t_fixed=c.get("t_fixed", 0), reps=c.get("reps", 1))
    if "k_frac" in c:
        kq = dg.k_fraction(S.lengths(), *c["k_frac"])
        op = oracle.make_params(c["q"], S.sigma, k_per_string=kq, **kw)
        gp = mj.Params(q=c["q"], k_per_string=torch.from_numpy(kq).cuda(), **kw)
    else:
        op = oracle.make_params(c["q"], S.sigma, k=c["k"], **kw)
        gp = mj.Params(q=c["q"], k=c["k"], **kw)
    return S, op, gp


@pytest.mark.parametrize("name", sorted(CASES))
def test_partition_records_identical(mj, name):
    say("partition", name)
    S, op, gp = run_case(mj, name)
    got = mj.partition(dev(mj, S), gp)
    want = oracle.partition_all(S.chars, S.offsets, op)
    assert len(got) > S.n  # several tiles' worth of partitions
    assert_records_equal(got, want)


@pytest.mark.parametrize("t_div", [1, 4])
def test_partition_hashed_path_with_top_half_collisions(mj, t_div):
    """q * b = 14 bits: the anchor test runs on 64-bit hashes, not ranks.  A table whose
    values share only 8 distinct top halves (distinct low halves) makes nearly every window
    minimum tie on the top half, so every comparison must use the full values; lengths from
    40 to 2500 give radii on both sides of the block test's limit."""
    import torch
    say("partition hashed path, top-half ties, t_div=%d" % t_div)
    rng = np.random.default_rng(4242 + t_div)
    q, ncodes = 7, 1 << 14
    low = rng.permutation(ncodes).astype(np.uint64) * np.uint64(2654435761) + np.uint64(12345)
    table = (rng.integers(0, 8, ncodes).astype(np.uint64) << np.uint64(32)) | (low & np.uint64(0xFFFFFFFF))
    assert len(np.unique(table)) == ncodes
    strs = [rng.integers(0, 4, int(rng.integers(40, 2500))).astype(np.uint8) for _ in range(160)]
    S = dg.from_list(strs, 4)
    tab = torch.from_numpy(table.view(np.int64)).cuda()
    got = mj.partition(dev(mj, S), mj.Params(q=q, k=30, t_div=t_div, pi_table=tab))
    want = oracle.partition_all(S.chars, S.offsets,
                                oracle.make_params(q, 4, k=30, t_div=t_div, pi_table=table))
    assert len(got) > S.n
    assert_records_equal(got, want)


@pytest.mark.parametrize("name", sorted(CASES))
def test_candidates_and_output_identical(mj, name):
    say("join", name)
    S, op, gp = run_case(mj, name)
    cand_w, out_w, st_w = oracle.join(S.chars, S.offsets, op)
    ds = dev(mj, S)
    cand_g, st_c = mj.candidates(ds, gp)
    assert np.array_equal(cand_g, cand_w)
    out_g, st = mj.join(ds, gp)
    assert np.array_equal(out_g, out_w)
    assert st["candidates"] == len(cand_w) and st["output"] == len(out_w)
    gp.verifier = mj.VERIFY_PLAIN
    out_p, _ = mj.join(ds, gp)
    assert np.array_equal(out_p, out_w)


def test_kernel_launch_counts_per_repetition(mj):
    """The join reports one anchor launch and one record bracket, each covering all
    repetitions (Sec. 3), and its device times."""
    say("launch counts", "dna_reps3")
    S, op, gp = run_case(mj, "dna_reps3")
    _, st = mj.join(dev(mj, S), gp)
    n = st["kernel_launches"]
    assert n["anchors"] == 1 and n["records"] == 1
    assert st["candidates"] > 0
    assert n["emit"] == 1 and n["verify"] >= 1
    assert all(st["kernel_ms"][k] > 0 for k in n)


def test_empty_and_degenerate_collections(mj):
    say("degenerate collections")
    for strs in ([], [np.zeros(0, np.uint8)], [np.zeros(0, np.uint8)] * 3,
                 [np.array([1], np.uint8)], [np.array([1, 2, 3], np.uint8)] * 2):
        S = dg.from_list(strs, 4)
        ds = dev(mj, S)
        p = mj.Params(q=4, k=2, t_div=1)
        want_c, want_o, _ = oracle.join(S.chars, S.offsets, oracle.make_params(4, 4, k=2, t_div=1))
        got_o, st = mj.join(ds, p)
        assert np.array_equal(got_o, want_o)
        assert len(mj.partition(ds, p)) == len(
            oracle.partition_all(S.chars, S.offsets, oracle.make_params(4, 4, k=2, t_div=1)))


# ---------------------------------------------------------------- verification
def near_threshold_pairs(rng, K, count, sigma=4):
    strs, pairs = [], []
    for t in range(count):
        L = int(rng.integers(max(1, K // 2), 4 * K + 40))
        x = rng.integers(0, sigma, L).astype(np.uint8)
        rate = min(0.9, rng.uniform(0.6, 1.4) * (K + 1) / L)
        y = dg.mutate(rng, x, rate, sigma)
        a, b = len(strs), len(strs) + 1
        strs += [x, y]
        pairs.append((a << 32) | b if t % 2 == 0 else (b << 32) | a)
    # paths along the edges of the band: y drops a symbols at one end of x and gains b
    # random symbols at the other, so the cheapest alignment runs along diagonal a (or
    # -b) with a + b in {K-1, K, K+1} and length difference d = a - b
    for d in sorted({0, 1, K // 3, max(0, K - 1), K}):
        for total in (K - 1, K, K + 1):
            if total < d or (total - d) % 2:
                continue
            a_, b_ = (total + d) // 2, (total - d) // 2
            L = int(rng.integers(a_ + 8, a_ + 3 * K + 40))
            x = rng.integers(0, sigma, L).astype(np.uint8)
            extra = rng.integers(0, sigma, b_).astype(np.uint8)
            for y in (np.concatenate([x[a_:], extra]), np.concatenate([extra, x[:L - a_]])):
                i0 = len(strs)
                strs += [x, y]
                pairs.append((i0 << 32) | (i0 + 1))
    # a few degenerate ones: empty strings and length gaps at the limit
    e = len(strs)
    strs += [np.zeros(0, np.uint8), rng.integers(0, sigma, K).astype(np.uint8),
             rng.integers(0, sigma, K + 1).astype(np.uint8)]
    pairs += [(e << 32) | (e + 1), (e << 32) | (e + 2), ((e + 1) << 32) | (e + 2)]
    return dg.from_list(strs, sigma), np.array(pairs, dtype=np.uint64)


@pytest.mark.parametrize("verifier", ["batched", "plain"])
@pytest.mark.parametrize("K", [0, 1, 7, 31, 32, 33, 60, 150, 255, 256, 257, 400])
def test_verify_matches_banded_oracle(mj, K, verifier):
    say("verify K=%d %s" % (K, verifier))
    rng = np.random.default_rng(1000 + K)
    S, pairs = near_threshold_pairs(rng, K, 120 if K < 300 else 40)
    v = mj.VERIFY_BATCHED if verifier == "batched" else mj.VERIFY_PLAIN
    got = mj.verify(dev(mj, S), mj.Params(q=4, k=K, t_div=1, verifier=v), pairs)
    want = oracle.verify_list(S.chars, S.offsets, oracle.make_params(4, 4, k=K), pairs)
    assert np.array_equal(got, want)
    assert 0 < want.sum() < len(want)


@pytest.mark.parametrize("lanes", [1, 2, 4, 8, -2])
@pytest.mark.parametrize("K", [0, 1, 31, 33, 60, 150, 257])
def test_verify_each_lane_layout_matches_banded_oracle(mj, K, lanes):
    """Every fixed layout of the batched verifier (1-8 lanes splitting the band words, or
    two lanes splitting the text columns) decides like the oracle; texts under 64 columns
    exercise the column split's one-lane fallback, longer ones its meeting step."""
    say("verify K=%d lanes=%d" % (K, lanes))
    rng = np.random.default_rng(2000 + K)
    S, pairs = near_threshold_pairs(rng, K, 120)
    got = mj.verify(dev(mj, S), mj.Params(q=4, k=K, t_div=1, verify_lanes=lanes), pairs)
    want = oracle.verify_list(S.chars, S.offsets, oracle.make_params(4, 4, k=K), pairs)
    assert np.array_equal(got, want)
    assert 0 < want.sum() < len(want)


@pytest.mark.parametrize("verifier", ["batched", "plain", "classes"])
def test_verify_per_pair_thresholds_across_bins(mj, verifier):
    """Per-string K from 3 to 520 (band windows of 2 to 18 words): the batched verifier in
    its small-call layout, the band classes (each pair in the window of its own class:
    2, 4, 8, 16 or 32 words) and the plain verifier all decide like the oracle."""
    import torch
    say("verify mixed K bins", verifier)
    rng = np.random.default_rng(77)
    strs, pairs, ks = [], [], []
    for t in range(300):
        K = int(rng.choice([3, 20, 45, 90, 130, 200, 250, 300, 520]))
        L = int(rng.integers(K + 5, 5 * K + 50))
        x = rng.integers(0, 25, L).astype(np.uint8)
        y = dg.mutate(rng, x, min(0.9, rng.uniform(0.6, 1.4) * (K + 1) / L), 25)
        a = len(strs)
        strs += [x, y]
        ks += [K, int(rng.integers(0, K + 1))]
        pairs.append((a << 32) | (a + 1))
    S = dg.from_list(strs, 25)
    kq = np.array(ks, dtype=np.int32)
    pairs = np.array(pairs, dtype=np.uint64)
    v = mj.VERIFY_PLAIN if verifier == "plain" else mj.VERIFY_BATCHED
    lanes = -3 if verifier == "classes" else 0
    got = mj.verify(dev(mj, S), mj.Params(q=3, k_per_string=torch.from_numpy(kq).cuda(), verifier=v,
                                          verify_lanes=lanes), pairs)
    want = oracle.verify_list(S.chars, S.offsets, oracle.make_params(3, 25, k_per_string=kq), pairs)
    assert np.array_equal(got, want)


@pytest.mark.parametrize("name", ["protein_per_string_K", "dna_mixed_T_from_K"])
def test_join_with_band_classes(mj, name):
    """The batched verifier with the band classes fixed (verify_lanes -3), stage by stage and
    streamed: the output equals the oracle's; a uniform K puts every pair in one class."""
    say("band classes", name)
    S, op, gp = run_case(mj, name)
    _, out_w, _ = oracle.join(S.chars, S.offsets, op)
    gp.verify_lanes = -3
    ctx = mj.Context()
    ds = dev(mj, S)
    for streamed in (0, 1):
        out, st = mj.join(ds, gp, ctx=ctx)
        assert np.array_equal(out, out_w)
        assert st["verify_group"] == -3 and st["streamed"] == streamed
    ctx.set_streaming(2)  # captured into HIP graphs, then replayed
    for _ in range(2):
        out, st = mj.join(ds, gp, ctx=ctx)
        assert np.array_equal(out, out_w)
    assert st["streamed"] == 2
    ctx.close()


# ---------------------------------------------------------------- search
def test_search_matches_oracle(mj):
    import torch
    say("search")
    S = dg.dna_small(seed=21, n_clusters=25, copies=6)
    ids = np.arange(S.n)
    I, Q = S.subset(ids[ids % 3 != 0]), S.subset(ids[ids % 3 == 0])
    kq = dg.k_fraction(Q.lengths(), 1, 10)
    ki = dg.k_fraction(I.lengths(), 1, 10)
    index = mj.Index(dev(mj, I), mj.Params(q=4, k_per_string=torch.from_numpy(ki).cuda(), t_div=1))
    got, st = index.search(dev(mj, Q), k_per_query=torch.from_numpy(kq).cuda())
    _, want = oracle.search(I.chars, I.offsets, oracle.make_params(4, 4, k_per_string=ki, t_div=1),
                            Q.chars, Q.offsets, oracle.make_params(4, 4, k_per_string=kq, t_div=1))
    assert len(want) > 0
    assert np.array_equal(got, want)
    # a second batch on the same resident index gives the same answer
    got2, _ = index.search(dev(mj, Q), k_per_query=torch.from_numpy(kq).cuda())
    assert np.array_equal(got2, want)
    # and so does the plain verifier (a pair per lane, one launch per band size)
    got3, st3 = index.search(dev(mj, Q), k_per_query=torch.from_numpy(kq).cuda(),
                             verifier=mj.VERIFY_PLAIN)
    assert np.array_equal(got3, want) and st3["verify_group"] == 0
    # and so do the band classes (per-query K: windows sized per pair)
    got4, st4 = index.search(dev(mj, Q), k_per_query=torch.from_numpy(kq).cuda(), verify_lanes=-3)
    assert np.array_equal(got4, want) and st4["verify_group"] == -3
    index.close()


def test_search_with_wide_radii(mj):
    """An index and queries of 8,000-11,000 symbols at T = 1 (radii above the tile halo, on
    both sides of the search) against the oracle, with both verifiers."""
    import torch
    say("search, wide radii")
    S = long_T1_collection(43, 4, n_bases=5, copies=3)
    ids = np.arange(S.n)
    I, Q = S.subset(ids[ids % 3 != 0]), S.subset(ids[ids % 3 == 0])
    op = oracle.make_params(6, 4, k=60, t_fixed=1)
    _, want = oracle.search(I.chars, I.offsets, op, Q.chars, Q.offsets, op)
    assert len(want) > 0
    index = mj.Index(dev(mj, I), mj.Params(q=6, k=60, t_fixed=1))
    kq = torch.full((Q.n,), 60, dtype=torch.int32).cuda()
    for verifier in (mj.VERIFY_BATCHED, mj.VERIFY_PLAIN):
        got, _ = index.search(dev(mj, Q), k_per_query=kq, verifier=verifier)
        assert np.array_equal(got, want)
    index.close()


def test_search_few_queries_large_index(mj):
    """Query ids span far fewer bits than index ids (3 queries, 6,000 index strings):
    the candidate pairs must still be deduplicated over the full index id range."""
    import torch
    say("search: 3 queries against 6,000 strings")
    S = dg.dna_small(seed=22, n_clusters=600, copies=10)
    rng = np.random.default_rng(5)
    qids = rng.choice(S.n, size=3, replace=False)
    mask = np.ones(S.n, bool)
    mask[qids] = False
    I, Q = S.subset(np.nonzero(mask)[0]), S.subset(np.sort(qids))
    kq = dg.k_fraction(Q.lengths(), 1, 10)
    ki = dg.k_fraction(I.lengths(), 1, 10)
    index = mj.Index(dev(mj, I), mj.Params(q=4, k_per_string=torch.from_numpy(ki).cuda(), t_div=1))
    got, st = index.search(dev(mj, Q), k_per_query=torch.from_numpy(kq).cuda())
    cand, want = oracle.search(I.chars, I.offsets, oracle.make_params(4, 4, k_per_string=ki, t_div=1),
                               Q.chars, Q.offsets, oracle.make_params(4, 4, k_per_string=kq, t_div=1))
    assert st["candidates"] == len(cand)
    assert len(want) > 0 and np.array_equal(got, want)
    index.close()


# ---------------------------------------------------------------- full workloads
def test_dna_small_workload_identical(mj):
    say("dna_small full (1,000 strings, K=60)")
    S = dg.dna_small()
    op = oracle.make_params(4, 4, k=60, t_div=1)
    cand_w, out_w, _ = oracle.join(S.chars, S.offsets, op)
    out_g, st = mj.join(dev(mj, S), mj.Params(q=4, k=60, t_div=1))
    assert st["candidates"] == len(cand_w)
    assert np.array_equal(out_g, out_w)


def test_dna_long_workload_sampled(mj):
    """The 50,000-string long-read workload in the configuration the benchmark times:
    candidates compared in full, the verification on a sample of candidates, records
    on a sample of strings."""
    say("dna_long full size (50,000 strings, K=150, t_div=2)")
    S = dg.dna_long()
    op = oracle.make_params(5, 4, k=150, t_div=2)
    ds = dev(mj, S)
    gp = mj.Params(q=5, k=150, t_div=2)
    cand_w, _, _ = oracle.join(S.chars, S.offsets, op, verify=False)
    cand_g, _ = mj.candidates(ds, gp)
    assert np.array_equal(cand_g, cand_w)
    out_g, st = mj.join(ds, gp)
    gp.verifier = mj.VERIFY_PLAIN
    out_p, _ = mj.join(ds, gp)
    assert np.array_equal(out_p, out_g)  # batched and plain verifiers agree at full size
    rng = np.random.default_rng(0)
    sample = np.sort(rng.choice(len(cand_w), size=min(1500, len(cand_w)), replace=False))
    flags = oracle.verify_list(S.chars, S.offsets, op, cand_w[sample])
    in_out = np.isin(cand_w[sample], out_g)
    assert np.array_equal(in_out, flags)
    assert np.all(np.isin(out_g, cand_w))
    ids = np.sort(rng.choice(S.n, size=300, replace=False))
    sub = S.subset(ids)
    want = oracle.partition_all(sub.chars, sub.offsets, op)
    got = mj.partition(ds, gp)
    sel = np.isin(got["sid"], ids)
    got = got[sel]
    got["sid"] = np.searchsorted(ids, got["sid"])
    assert_records_equal(got, want)


# ---------------------------------------------------------------- serving
def test_server_answers_equal_alone_and_in_the_mix(mj):
    """Continuous batching: each request's answer in the mix equals its answer alone
    (and the oracle's), while batches of several requests and several workers run."""
    import torch
    say("server")
    rng = np.random.default_rng(90)
    I = dg.random_strings(91, 300, 300, 1500)
    Ikq = dg.k_fraction(I.lengths(), 1, 10)
    index = mj.Index(dev(mj, I), mj.Params(q=4, k_per_string=torch.from_numpy(Ikq).cuda(), t_div=1))
    queries = []
    for t in range(120):
        if t % 2 == 0:
            src = I.get(int(rng.integers(0, I.n)))
            queries.append(dg.mutate(rng, src, rng.uniform(0.01, 0.12), 4))
        else:
            queries.append(rng.integers(0, 4, int(rng.integers(1, 1500))).astype(np.uint8))
    ks = [int(v) for v in dg.k_fraction([len(q) for q in queries], 1, 10)]
    alone = []
    for q, k in zip(queries, ks):
        Q = dg.from_list([q], 4)
        got, _ = index.search(dev(mj, Q), k=k)
        alone.append(np.sort((got & np.uint64(0xFFFFFFFF)).astype(np.uint32)))
    Q = dg.from_list(queries, 4)
    _, want = oracle.search(I.chars, I.offsets, oracle.make_params(4, 4, k_per_string=Ikq, t_div=1),
                            Q.chars, Q.offsets, oracle.make_params(4, 4, k_per_string=np.array(ks, np.int32), t_div=1))
    srv = mj.Server(index, workers=3, max_batch=16, memory_budget=1 << 26)
    for t, (q, k) in enumerate(zip(queries, ks)):
        srv.submit(q, k, t)
    replies = []
    while len(replies) < len(queries):
        replies += srv.poll(timeout_ms=10000)
    srv.close()
    by_tag = {r["tag"]: r for r in replies}
    assert sorted(by_tag) == list(range(len(queries)))
    for t in range(len(queries)):
        r = by_tag[t]
        assert r["status"] == 0
        assert np.array_equal(r["ids"], alone[t])
        ref = np.sort((want[(want >> np.uint64(32)) == t] & np.uint64(0xFFFFFFFF)).astype(np.uint32))
        assert np.array_equal(r["ids"], ref)
    assert max(r["batch_size"] for r in replies) > 1
    assert sum(len(a) for a in alone) > 0
    index.close()


# ---------------------------------------------------------------- streamed join
@pytest.mark.parametrize("name", sorted(CASES))
def test_streamed_join_identical(mj, name):
    """A second batched join with the same parameters on a context sizes its stages on the
    device (two host reads); its output equals the oracle's, and so does a join of another
    collection through the same context (streamed, or stage by stage when the candidates
    outgrow the room the first join left)."""
    say("streamed", name)
    S, op, gp = run_case(mj, name)
    _, out_w, _ = oracle.join(S.chars, S.offsets, op)
    ctx = mj.Context()
    ds = dev(mj, S)
    out1, st1 = mj.join(ds, gp, ctx=ctx)
    out2, st2 = mj.join(ds, gp, ctx=ctx)
    assert st1["streamed"] == 0 and st2["streamed"] == 1 and st2["host_reads"] == 2
    assert np.array_equal(out1, out_w) and np.array_equal(out2, out_w)
    assert st2["candidates"] == st1["candidates"] and st2["records"] == st1["records"]
    assert st2["pair_tests"] == st1["pair_tests"] and st2["groups"] == st1["groups"]
    # another collection (every other string) through the same context
    T = S.subset(np.arange(0, S.n, 2))
    _, op_t, gp_t = params_for(mj, CASES[name], T)
    _, out_t, _ = oracle.join(T.chars, T.offsets, op_t)
    out3, _ = mj.join(dev(mj, T), gp_t, ctx=ctx)
    assert np.array_equal(out3, out_t)
    ctx.close()


def test_streamed_join_falls_back_when_candidates_outgrow_the_room(mj):
    """Hints from a join with few candidates per record leave too little room for a
    collection of near-copies: the streamed join notices and the result is still exact."""
    say("streamed fallback")
    sparse = dg.dna_small(seed=81, n_clusters=40, copies=2)
    dense = heavy_cluster_collection(82)
    p = mj.Params(q=4, k=20, t_div=1)
    ctx = mj.Context()
    mj.join(dev(mj, sparse), p, ctx=ctx)
    _, want, _ = oracle.join(dense.chars, dense.offsets, oracle.make_params(4, 4, k=20, t_div=1))
    out, st = mj.join(dev(mj, dense), p, ctx=ctx)
    assert np.array_equal(out, want) and len(want) > 0
    ctx.close()


@pytest.mark.parametrize("name", ["dna_mixed_T_from_K", "protein_per_string_K", "text_q6", "dna_reps3",
                                  "dna_T1_long_reps2", "protein_big_groups"])
def test_captured_join_identical(mj, name):
    """Streamed joins captured into HIP graphs (mj_ctx_set_streaming 2) and replayed: each
    replay equals the oracle, also after the strings' content changes in place (same
    pointers and lengths: the graphs replay, or the join runs again stage by stage)."""
    import torch
    say("captured", name)
    S, op, gp = run_case(mj, name)
    _, out_w, _ = oracle.join(S.chars, S.offsets, op)
    ctx = mj.Context()
    ctx.set_streaming(2)
    ds = dev(mj, S)
    modes = []
    for _ in range(3):
        out, st = mj.join(ds, gp, ctx=ctx)
        assert np.array_equal(out, out_w)
        modes.append(st["streamed"])
    assert modes == [0, 2, 2]
    # new content, same lengths, same device buffers: every string reversed
    rev = np.concatenate([S.get(i)[::-1] for i in range(S.n)]) if S.n else S.chars
    T = dg.from_list([S.get(i)[::-1] for i in range(S.n)], S.sigma)
    assert np.array_equal(T.offsets, S.offsets)
    ds.chars.copy_(torch.from_numpy(np.ascontiguousarray(rev, dtype=np.uint8)).cuda()[:ds.chars.numel()])
    torch.cuda.synchronize()
    _, out_t, _ = oracle.join(T.chars, T.offsets, op)
    out, st = mj.join(ds, gp, ctx=ctx)
    assert np.array_equal(out, out_t)
    ctx.set_streaming(1)
    out, st = mj.join(ds, gp, ctx=ctx)
    assert np.array_equal(out, out_t) and st["streamed"] == 1
    ctx.close()


@pytest.mark.parametrize("bucket_limit", [0, 1])
@pytest.mark.parametrize("name", sorted(CASES))
def test_member_filter_identical(mj, name, bucket_limit):
    """The member filter forced on (every join; with bucket_limit 1 every bucket of two or
    more records is kept whole): candidates and output equal the oracle's, stage by stage
    and streamed, with the same groups and pair tests as without the filter."""
    say("member filter", name, bucket_limit)
    S, op, gp = run_case(mj, name)
    cand_w, out_w, _ = oracle.join(S.chars, S.offsets, op)
    ds = dev(mj, S)
    ctx0 = mj.Context()
    ctx0.set_member_filter(-1)
    _, st0 = mj.join(ds, gp, ctx=ctx0)
    assert st0["member_filter"] == 0 and st0["members"] == st0["records"]
    ctx0.close()
    ctx = mj.Context()
    ctx.set_member_filter(0, bucket_limit)
    cand, stc = mj.candidates(ds, gp, ctx=ctx)
    assert np.array_equal(cand, cand_w) and stc["member_filter"] == 1
    for streamed in (0, 1):
        out, st = mj.join(ds, gp, ctx=ctx)
        assert np.array_equal(out, out_w)
        assert st["streamed"] == streamed and st["member_filter"] == 1
        assert st["groups"] == st0["groups"] and st["pair_tests"] == st0["pair_tests"]
        assert st["records"] == st0["records"] and st["members"] <= st["records"]
    ctx.set_streaming(2)  # captured into HIP graphs, then replayed
    for _ in range(2):
        out, st = mj.join(ds, gp, ctx=ctx)
        assert np.array_equal(out, out_w)
    assert st["streamed"] == 2
    ctx.close()


@pytest.mark.parametrize("tile_min", [0, -1])
@pytest.mark.parametrize("name", ["dna_big_groups", "protein_big_groups", "dna_heavy_clusters",
                                  "text_q6", "dna_lazy_big_group", "dna_lazy_big_group_lk"])
def test_tile_emission_identical(mj, name, tile_min):
    """Candidate emission with the groups of 64 records or more tested by 64 x 64 tile
    pairs (mj_ctx_set_tile_emission 0: whenever there is one) or every group test by test
    (-1): candidates and output equal the oracle's, stage by stage, streamed and captured."""
    say("tile emission", name, tile_min)
    S, op, gp = run_case(mj, name)
    cand_w, out_w, st_w = oracle.join(S.chars, S.offsets, op)
    ctx = mj.Context()
    ctx.set_tile_emission(tile_min)
    ds = dev(mj, S)
    cand, st = mj.candidates(ds, gp, ctx=ctx)
    assert np.array_equal(cand, cand_w) and st["pair_tests"] == st_w["pair_tests"]
    modes = []
    for _ in range(2):
        out, st = mj.join(ds, gp, ctx=ctx)
        assert np.array_equal(out, out_w) and st["pair_tests"] == st_w["pair_tests"]
        modes.append(st["streamed"])
    assert modes == [0, 1]
    ctx.set_streaming(2)
    for _ in range(2):
        out, st = mj.join(ds, gp, ctx=ctx)
        assert np.array_equal(out, out_w)
    assert st["streamed"] == 2
    ctx.close()


def test_tile_emission_over_2_29_symbols(mj):
    """At 2^29 symbols or more both emission kernels take the 64-bit filter: 500 random
    strings of 1,074,000 symbols (K = 2,000) and a cluster of 70 near-copies of 400
    symbols (K = 20, groups of 64 records and more); candidates and output equal the
    oracle's with the tile-pair path forced on and off."""
    import torch
    say("tile emission over 2^29 symbols")
    rng = np.random.default_rng(97)
    strs = [rng.integers(0, 4, 1_074_000, dtype=np.uint8) for _ in range(500)]
    base = rng.integers(0, 4, 400).astype(np.uint8)
    strs += [dg.mutate(np.random.default_rng(97000 + i), base, 0.005, 4) for i in range(70)]
    S = dg.from_list(strs, 4)
    del strs
    assert int(S.offsets[-1]) >= 1 << 29
    kq = np.where(S.lengths() > 100_000, 2000, 20).astype(np.int32)
    op = oracle.make_params(4, 4, k_per_string=kq, t_div=1)
    cand_w, out_w, _ = oracle.join(S.chars, S.offsets, op)
    assert len(out_w) > 0
    ds = dev(mj, S)
    gp = mj.Params(q=4, k_per_string=torch.from_numpy(kq).cuda(), t_div=1)
    for tile_min in (0, -1):
        ctx = mj.Context()
        ctx.set_tile_emission(tile_min)
        cand, _ = mj.candidates(ds, gp, ctx=ctx)
        assert np.array_equal(cand, cand_w), tile_min
        out, _ = mj.join(ds, gp, ctx=ctx)
        assert np.array_equal(out, out_w), tile_min
        ctx.close()


@pytest.mark.parametrize("name", ["dna_heavy_clusters", "protein_per_string_K", "dna_big_groups"])
def test_join_in_emission_passes(mj, name):
    """A join whose record-pair tests exceed one emission pass (here forced down to 1,024
    tests per pass) emits and deduplicates them in passes: candidates and output equal the
    oracle's, for the stage-by-stage and the streamed path."""
    say("emission passes", name)
    S, op, gp = run_case(mj, name)
    cand_w, out_w, st_w = oracle.join(S.chars, S.offsets, op)
    assert st_w["pair_tests"] > 8 * 1024
    ctx = mj.Context()
    ctx.set_pair_test_pass(1024)
    ds = dev(mj, S)
    cand, st = mj.candidates(ds, gp, ctx=ctx)
    assert np.array_equal(cand, cand_w) and st["pair_tests"] > 8 * 1024
    for _ in range(2):
        out, st = mj.join(ds, gp, ctx=ctx)
        assert np.array_equal(out, out_w)
    ctx.close()
