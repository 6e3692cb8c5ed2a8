"""Pins for the CPU oracle: each test checks it against something the paper or the
mathematics fixes, not against a retyped copy of its own formulas."""
import itertools
import math

import numpy as np
import pytest

import oracle
from paper_1810_08833_amd import datagen as dg
from tests import worked_example as wex

GAMMA = 0x9E3779B97F4A7C15
M64 = (1 << 64) - 1


# ---------------------------------------------------------------- hash Pi
def test_mixer_matches_published_splitmix64_outputs():
    # SplitMix64 seeded with 0 outputs M(k * gamma) for k = 1, 2, 3 (Steele, Lea & Flood
    # 2014; these are the generator's published first outputs for seed 0).
    assert oracle.mix64(GAMMA) == 0xE220A8397B1DCDAF
    assert oracle.mix64((2 * GAMMA) & M64) == 0x6E789E6AA1B965F4
    assert oracle.mix64((3 * GAMMA) & M64) == 0x06C45D188009454F


def test_pi_is_injective_on_a_full_code_space():
    # every DNA 5-gram occurs once in this de Bruijn-like enumeration string set
    grams = np.array(list(itertools.product(range(4), repeat=5)), dtype=np.uint8)
    vals = set()
    for g in grams:
        vals.add(int(oracle.qgram_hashes(g, 5, 4, seed=0)[0]))
    assert len(vals) == 4 ** 5


def test_pi_depends_only_on_qgram_content():
    rng = np.random.default_rng(7)
    s = rng.integers(0, 4, 400).astype(np.uint8)
    h = oracle.qgram_hashes(s, 4, 4, seed=3)
    # equal q-grams <=> equal hash values (Pi is a function of the q-gram and injective)
    for i in range(0, 380, 7):
        for j in range(i + 1, 397, 11):
            assert (h[i] == h[j]) == bool(np.array_equal(s[i:i + 4], s[j:j + 4]))
    assert not np.array_equal(h, oracle.qgram_hashes(s, 4, 4, seed=4))


# ---------------------------------------------------------------- r and T
def test_radius_rule_and_clamp():
    # r = floor((|s| - q + 1 - T) / (2T + 2)) (Alg. 2), clamped to >= 1
    assert oracle.radius(21, 3, 3) == 2          # Table 4: r = 2 for |s| = 21
    assert oracle.radius(22, 3, 3) == 2
    assert oracle.radius(1000, 4, 12) == (1000 - 4 + 1 - 12) // 26
    assert oracle.radius(5000, 5, 150) == (5000 - 5 + 1 - 150) // 302
    assert oracle.radius(300, 6, 120) == 1       # numerator 175 < 242: clamped
    assert oracle.radius(10, 6, 120) == 1        # negative numerator: clamped
    assert oracle.target_partitions(60, 5) == 12
    assert oracle.target_partitions(61, 5) == 13
    assert oracle.target_partitions(3, 5) == 1
    assert oracle.target_partitions(60, 1, t_fixed=3) == 3


# ---------------------------------------------------------------- worked example
def test_worked_example_partitions_match_table_4():
    g, table, strings, _, _ = wex.load()
    for s, want_parts, want_r, text in zip(strings, g["partitions"], g["radius"], g["strings"]):
        assert oracle.radius(len(s), g["q"], g["T"]) == want_r
        a = oracle.find_anchors(s, g["q"], 4, g["T"], pi_table=table)
        got = [text[a[k]:a[k + 1]] for k in range(len(a) - 1)]
        assert got == want_parts
    a1 = oracle.find_anchors(strings[0], 3, 4, 3, pi_table=table)
    assert list(a1[:-1] + 1) == [1, 6, 14]  # the 6th and 14th 3-grams of s1 (1-based)


def test_worked_example_join_candidates_and_output():
    g, table, _, chars, offsets = wex.load()
    p = oracle.make_params(g["q"], 4, k=g["K"], t_fixed=g["T"], pi_table=table)
    cand, out, st = oracle.join(chars, offsets, p)
    assert wex.pairs_1based(cand) == g["candidates_1based"]
    assert wex.pairs_1based(out) == g["output_1based"]
    # any other Pi ATC value of Table 2 (0.77) gives the same result
    t2 = table.copy()
    t2[(0 << 4) | (3 << 2) | 1] = np.uint64(77)
    p2 = oracle.make_params(g["q"], 4, k=g["K"], t_fixed=g["T"], pi_table=t2)
    cand2, out2, _ = oracle.join(chars, offsets, p2)
    assert np.array_equal(cand, cand2) and np.array_equal(out, out2)


# ---------------------------------------------------------------- edit distance
def _ed_by_search(x, y):
    """Brute force: breadth-first search over single edits from x until y appears."""
    x, y = tuple(x), tuple(y)
    alphabet = sorted(set(x) | set(y)) or [0]
    seen, frontier, d = {x}, {x}, 0
    while y not in frontier:
        nxt = set()
        for s in frontier:
            for i in range(len(s) + 1):
                for c in alphabet:
                    nxt.add(s[:i] + (c,) + s[i:])
                if i < len(s):
                    nxt.add(s[:i] + s[i + 1:])
                    for c in alphabet:
                        nxt.add(s[:i] + (c,) + s[i + 1:])
        frontier = nxt - seen
        seen |= nxt
        d += 1
    return d


def test_edit_distance_textbook_values():
    enc = {c: i for i, c in enumerate("abcdefghijklmnopqrstuvwxyz")}
    e = lambda s: np.array([enc[c] for c in s], dtype=np.uint8)  # noqa: E731
    assert oracle.edit_distance(e("kitten"), e("sitting")) == 3
    assert oracle.edit_distance(e("flaw"), e("lawn")) == 2
    assert oracle.edit_distance(e(""), e("abc")) == 3
    assert oracle.edit_distance(e("abc"), e("abc")) == 0


def test_edit_distance_equals_brute_force_search():
    rng = np.random.default_rng(11)
    for _ in range(60):
        x = rng.integers(0, 2, rng.integers(0, 5)).astype(np.uint8)
        y = rng.integers(0, 2, rng.integers(0, 5)).astype(np.uint8)
        assert oracle.edit_distance(x, y) == _ed_by_search(x, y)


def test_worked_example_pair_decisions():
    g, _, strings, _, _ = wex.load()
    want = {tuple(p) for p in g["output_1based"]}
    for i in range(5):
        for j in range(i + 1, 5):
            within = (i + 1, j + 1) in want
            # (4,5) is a candidate that the verification rejects
            assert oracle.ed_within(strings[i], strings[j], g["K"]) == within
            if (i + 1, j + 1) in want:
                assert oracle.edit_distance(strings[i], strings[j]) <= g["K"]


@pytest.mark.parametrize("K", [0, 1, 2, 5, 13, 40])
def test_banded_decision_equals_full_dp(K):
    # Ukkonen: deciding ED <= K only needs the band |i - j| <= K (stress ED near K)
    rng = np.random.default_rng(100 + K)
    hits = {K - 1: 0, K: 0, K + 1: 0}
    for _ in range(200):
        L = int(rng.integers(0, 6 * K + 12))
        x = rng.integers(0, 4, L).astype(np.uint8)
        rate = min(0.9, rng.uniform(0.5, 1.5) * (K + 1) / max(L, 1))
        y = dg.mutate(rng, x, rate, 4)
        d = oracle.edit_distance(x, y)
        if d in hits:
            hits[d] += 1
        assert oracle.ed_within(x, y, K) == (d <= K)
        assert oracle.ed_within(y, x, K) == (d <= K)
    if K >= 2:
        assert all(v > 0 for v in hits.values()), hits


# ---------------------------------------------------------------- anchors
def test_anchors_are_exactly_the_strict_local_minima():
    rng = np.random.default_rng(5)
    for trial in range(40):
        sigma = [2, 4, 25][trial % 3]
        q = [3, 4, 2][trial % 3]
        m = int(rng.integers(0, 300))
        T = int(rng.integers(1, 20))
        s = rng.integers(0, sigma, m).astype(np.uint8)
        a = oracle.find_anchors(s, q, sigma, T, seed=trial)
        if m == 0:
            assert len(a) == 0
            continue
        assert a[0] == 0 and a[-1] == m and np.all(np.diff(a) > 0)
        npos = m - q + 1
        if npos <= 0:
            assert list(a) == [0, m]
            continue
        h = oracle.qgram_hashes(s, q, sigma, seed=trial)
        r = oracle.radius(m, q, T)
        want = [0]
        for i in range(r, npos - r):
            win = np.concatenate([h[i - r:i], h[i + 1:i + r + 1]])
            if np.all(h[i] < win):
                want.append(i)
        want.append(m)
        assert list(a) == want


def test_strictness_suppresses_periodic_runs():
    # "AAAA..." repeats one q-gram: equal neighbours forbid anchors (Sec. 2.1, Discussions)
    s = np.zeros(500, dtype=np.uint8)
    assert list(oracle.find_anchors(s, 4, 4, 10)) == [0, 500]


def test_lemma1_anchor_count_concentrates_around_T():
    # Lemma 1: with distinct values in every window, E[X] = w / (2r + 1) with
    # w = |s| - q + 1 - 2r, and Var[X] < T.  q = 16 on DNA makes repeats negligible.
    rng = np.random.default_rng(2024)
    m, q, T = 4000, 16, 40
    r = oracle.radius(m, q, T)
    w = m - q + 1 - 2 * r
    xs = []
    for t in range(300):
        s = rng.integers(0, 4, m).astype(np.uint8)
        xs.append(len(oracle.find_anchors(s, q, 4, T, seed=t)) - 2)
    xs = np.array(xs, dtype=np.float64)
    mean_expected = w / (2 * r + 1)
    assert abs(xs.mean() - mean_expected) < 4 * math.sqrt(T / len(xs))
    assert xs.var(ddof=1) < T


def test_lemma2_similar_strings_share_a_partition():
    # Lemma 2: T = 120K and |s| >> Kq: at least 98% of pairs with ED <= K share a
    # partition.  Each trial applies K random edits to a random string.
    rng = np.random.default_rng(77)
    q = 12
    shared = trials = 0
    for K in (1, 2):
        T = 120 * K
        for t in range(60):
            m = int(rng.integers(30000, 40000))
            s = rng.integers(0, 4, m).astype(np.uint8)
            u = s.copy()
            for _ in range(K):
                i = int(rng.integers(0, len(u)))
                op = int(rng.integers(0, 3))
                if op == 0:
                    u = np.insert(u, i, rng.integers(0, 4))
                elif op == 1:
                    u = np.delete(u, i)
                else:
                    u[i] = (u[i] + 1) % 4
            pa = oracle.find_anchors(s, q, 4, T, seed=t)
            pb = oracle.find_anchors(u, q, 4, T, seed=t)
            parts_a = {s[pa[k]:pa[k + 1]].tobytes() for k in range(len(pa) - 1)}
            parts_b = {u[pb[k]:pb[k + 1]].tobytes() for k in range(len(pb) - 1)}
            shared += bool(parts_a & parts_b)
            trials += 1
    assert shared / trials >= 0.98


# ---------------------------------------------------------------- partition key
def test_partition_key_closed_form():
    # Phi = L * B^L + sum_k (x_k + 1) B^(L-1-k) mod 2^61-1, evaluated as a power sum
    P = (1 << 61) - 1
    B = oracle.lib().orc_phi_base(0)
    assert 2 <= B <= P - 2
    rng = np.random.default_rng(3)
    for L in [0, 1, 2, 7, 64, 333]:
        x = rng.integers(0, 37, L).astype(np.uint8)
        want = (L * pow(B, L, P) + sum((int(x[k]) + 1) * pow(B, L - 1 - k, P) for k in range(L))) % P
        assert oracle.partition_phi(x, 0) == want


def test_partition_key_separates_contents_and_lengths():
    rng = np.random.default_rng(9)
    keys = {}
    for _ in range(3000):
        L = int(rng.integers(0, 12))
        x = rng.integers(0, 4, L).astype(np.uint8)
        k = oracle.partition_key(x, 0)
        prev = keys.setdefault(k, x.tobytes())
        assert prev == x.tobytes()
    # a zero-padded string is a different partition
    assert oracle.partition_key(np.zeros(3, np.uint8)) != oracle.partition_key(np.zeros(4, np.uint8))


# ---------------------------------------------------------------- join
def _bruteforce_candidates(S, params, K_of):
    """Definition of the candidate set, by brute force over all record pairs: ids i != j
    holding partitions with the same bucket key that pass both filters."""
    rec = oracle.partition_all(S.chars, S.offsets, params)
    lens = S.lengths()
    out = set()
    for a in range(len(rec)):
        for b in range(a + 1, len(rec)):
            if rec[a]["key"] != rec[b]["key"]:
                continue
            i, j = int(rec[a]["sid"]), int(rec[b]["sid"])
            if i == j:
                continue
            mi, mj = int(lens[i]), int(lens[j])
            pi, pj = int(rec[a]["pos"]), int(rec[b]["pos"])
            K = max(K_of(i), K_of(j))
            if abs(mi - mj) <= K and abs(pi - pj) + abs((mi - pi) - (mj - pj)) <= K:
                out.add((min(i, j) << 32) | max(i, j))
    return out


@pytest.mark.parametrize("case", range(4))
def test_join_candidates_equal_definition(case):
    rng_seed = 300 + case
    S = dg.dna_small(seed=rng_seed, n_clusters=6, copies=5)
    K = [20, 40, 60, 80][case]
    p = oracle.make_params(4, 4, k=K, t_div=[1, 2, 3, 1][case], reps=[1, 1, 1, 2][case])
    cand, out, _ = oracle.join(S.chars, S.offsets, p)
    want = _bruteforce_candidates(S, p, lambda i: K)
    assert set(cand.tolist()) == want
    # precision: every output pair is within K under the full DP, and every candidate
    # within K is output
    for v in cand.tolist():
        i, j = v >> 32, v & 0xFFFFFFFF
        d = oracle.edit_distance(S.get(i), S.get(j))
        assert (v in set(out.tolist())) == (d <= K)


def test_join_per_string_threshold_matches_definition():
    S = dg.protein(seed=12, n=120)
    kq = dg.k_fraction(S.lengths(), 8, 100)
    p = oracle.make_params(4, 25, k_per_string=kq, t_div=1)
    cand, out, _ = oracle.join(S.chars, S.offsets, p)
    assert set(cand.tolist()) == _bruteforce_candidates(S, p, lambda i: int(kq[i]))
    for v in cand.tolist():
        i, j = v >> 32, v & 0xFFFFFFFF
        d = oracle.edit_distance(S.get(i), S.get(j))
        assert (v in set(out.tolist())) == (d <= max(kq[i], kq[j]))


def test_join_handles_empty_short_and_duplicate_strings():
    strings = [np.zeros(0, np.uint8), np.array([1, 2], np.uint8), np.array([1, 2], np.uint8),
               np.array([3], np.uint8), np.zeros(0, np.uint8), np.arange(4, dtype=np.uint8)]
    S = dg.from_list(strings, 4)
    p = oracle.make_params(3, 4, k=1, t_div=1)
    rec = oracle.partition_all(S.chars, S.offsets, p)
    assert sorted(rec["sid"].tolist()) == [1, 2, 3, 5]  # empty strings have no partition
    cand, out, _ = oracle.join(S.chars, S.offsets, p)
    # identical strings with different ids share their single partition (ED 0)
    assert (1 << 32 | 2) in set(out.tolist())


def test_search_equals_join_restricted_to_query_index_pairs():
    S = dg.dna_small(seed=41, n_clusters=8, copies=4)
    ids = np.arange(S.n)
    q_ids, i_ids = ids[ids % 4 == 0], ids[ids % 4 != 0]
    Q, I = S.subset(q_ids), S.subset(i_ids)
    K = 70
    pj = oracle.make_params(4, 4, k=K, t_div=1)
    _, out, _ = oracle.join(S.chars, S.offsets, pj)
    want = set()
    qpos = {int(g): k for k, g in enumerate(q_ids)}
    ipos = {int(g): k for k, g in enumerate(i_ids)}
    for v in out.tolist():
        a, b = v >> 32, v & 0xFFFFFFFF
        for x, y in ((a, b), (b, a)):
            if x in qpos and y in ipos:
                want.add((qpos[x] << 32) | ipos[y])
    _, got = oracle.search(I.chars, I.offsets, oracle.make_params(4, 4, k=K, t_div=1),
                           Q.chars, Q.offsets, oracle.make_params(4, 4, k=K, t_div=1))
    assert set(got.tolist()) == want


def test_parallel_repetition_only_adds_candidates():
    S = dg.dna_small(seed=55, n_clusters=10, copies=4)
    c1, o1, _ = oracle.join(S.chars, S.offsets, oracle.make_params(4, 4, k=60, t_div=3, reps=1))
    c3, o3, _ = oracle.join(S.chars, S.offsets, oracle.make_params(4, 4, k=60, t_div=3, reps=3))
    assert set(c1.tolist()) <= set(c3.tolist())
    assert set(o1.tolist()) <= set(o3.tolist())


def test_deterministic_for_a_fixed_seed():
    S = dg.dna_small(seed=9, n_clusters=10, copies=4)
    a = oracle.join(S.chars, S.offsets, oracle.make_params(4, 4, k=60, t_div=2, seed=1))
    b = oracle.join(S.chars, S.offsets, oracle.make_params(4, 4, k=60, t_div=2, seed=1, threads=1))
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


# ---------------------------------------------------------------- pins added for the
# repetition schedule, per-query thresholds and larger alphabets
@pytest.mark.parametrize("sigma", [25, 37])
def test_pi_is_injective_for_larger_alphabets(sigma):
    # b = ceil(log2 sigma) = 5 or 6 bits per symbol: every one of the sigma^3 3-grams gets
    # its own hash (a too-narrow packing would make codes >= 2^(b-1) collide)
    grams = np.array(list(itertools.product(range(sigma), repeat=3)), dtype=np.uint8)
    h = oracle.qgram_hashes(grams.reshape(-1), 3, sigma, seed=0)[::3]
    assert len(h) == sigma ** 3
    assert len(np.unique(h)) == sigma ** 3


def _content_partitions(S, q, T_of, reps, seed=0):
    """Each repetition rho cuts every string at the anchors that Find-Anchor gives with
    seed + rho (Sec. 3, parallel repetition); a partition is (content bytes, sid, pos)."""
    parts = []
    for i in range(S.n):
        s = S.get(i)
        for rho in range(reps):
            a = oracle.find_anchors(s, q, S.sigma, T_of(i), seed=seed + rho)
            parts += [(s[a[k]:a[k + 1]].tobytes(), i, int(a[k])) for k in range(len(a) - 1)]
    return parts


def _content_candidates(S, parts, K_of):
    """Candidates by brute force on partition content (not on the bucket key): distinct
    strings holding a partition with the same symbols that pass both filters."""
    lens = S.lengths()
    by = {}
    for c, i, p in parts:
        by.setdefault(c, []).append((i, p))
    out = set()
    for group in by.values():
        for a in range(len(group)):
            for b in range(a + 1, len(group)):
                (i, pi), (j, pj) = group[a], group[b]
                if i == j:
                    continue
                mi, mj = int(lens[i]), int(lens[j])
                K = max(K_of(i), K_of(j))
                if abs(mi - mj) <= K and abs(pi - pj) + abs((mi - pi) - (mj - pj)) <= K:
                    out.add((min(i, j) << 32) | max(i, j))
    return out


def test_repetition_rho_uses_seed_plus_rho():
    # the records of repetition rho are exactly the partitions at Find-Anchor's anchors
    # for seed + rho, with the bucket key of the base seed
    S = dg.dna_small(seed=61, n_clusters=5, copies=4)
    K, t_div, reps, seed = 60, 3, 3, 11
    p = oracle.make_params(4, 4, k=K, t_div=t_div, reps=reps, seed=seed)
    rec = oracle.partition_all(S.chars, S.offsets, p)
    T = oracle.target_partitions(K, t_div)
    for i in range(S.n):
        s = S.get(i)
        for rho in range(reps):
            mine = np.sort(rec[(rec["sid"] == i) & (rec["rep"] == rho)], order="pos")
            a = oracle.find_anchors(s, 4, 4, T, seed=seed + rho)
            assert mine["pos"].tolist() == a[:-1].tolist()
            assert mine["len"].tolist() == np.diff(a).tolist()
            keys = [oracle.partition_key(s[a[k]:a[k + 1]], seed) for k in range(len(a) - 1)]
            assert mine["key"].tolist() == keys
        # the repetitions really cut differently
        a0 = oracle.find_anchors(s, 4, 4, T, seed=seed)
        a1 = oracle.find_anchors(s, 4, 4, T, seed=seed + 1)
        assert not np.array_equal(a0, a1)


@pytest.mark.parametrize("reps", [1, 2, 3])
def test_join_with_repetitions_equals_content_brute_force(reps):
    # the union of all repetitions' partitions is joined: partitions of different
    # repetitions with the same content share a bucket
    S = dg.dna_small(seed=62, n_clusters=6, copies=4)
    K, t_div = 60, 3
    p = oracle.make_params(4, 4, k=K, t_div=t_div, reps=reps)
    cand, _, _ = oracle.join(S.chars, S.offsets, p, verify=False)
    T = oracle.target_partitions(K, t_div)
    want = _content_candidates(S, _content_partitions(S, 4, lambda i: T, reps), lambda i: K)
    assert set(cand.tolist()) == want


def test_second_repetition_finds_a_pair_the_first_misses():
    # at T = K/4 on these copies one repetition misses a true pair that a second finds
    S = dg.dna_small(seed=57, n_clusters=10, copies=4)
    c1, o1, _ = oracle.join(S.chars, S.offsets, oracle.make_params(4, 4, k=60, t_div=4, reps=1))
    c2, o2, _ = oracle.join(S.chars, S.offsets, oracle.make_params(4, 4, k=60, t_div=4, reps=2))
    new = set(o2.tolist()) - set(o1.tolist())
    assert new and set(o1.tolist()) < set(o2.tolist())
    for v in new:
        assert oracle.edit_distance(S.get(v >> 32), S.get(v & 0xFFFFFFFF)) <= 60


def _split_search_fixture(seed=43):
    S = dg.dna_small(seed=seed, n_clusters=8, copies=4)
    ids = np.arange(S.n)
    return S.subset(ids[ids % 4 != 0]), S.subset(ids[ids % 4 == 0])


def test_search_per_query_threshold_matches_definition():
    # search(index, queries, K): query q partitions with the T rule at its own K_q, and
    # both the filters and the verification use K_q (not max(K_q, K_s)).  The index
    # strings hold K = 140 for their T rule, above every query's K, so a threshold of
    # max(K_q, K_s) would accept more pairs.
    I, Q = _split_search_fixture(47)
    rng = np.random.default_rng(3)
    kq = rng.integers(40, 100, Q.n).astype(np.int32)
    KI, t_div = 140, 1
    ip = oracle.make_params(4, 4, k=KI, t_div=t_div)
    qp = oracle.make_params(4, 4, k_per_string=kq, t_div=t_div)
    cand, got = oracle.search(I.chars, I.offsets, ip, Q.chars, Q.offsets, qp)
    TI = oracle.target_partitions(KI, t_div)
    iparts = _content_partitions(I, 4, lambda i: TI, 1)
    by = {}
    for c, s, p in iparts:
        by.setdefault(c, []).append((s, p))
    want_c, want_o, wider = set(), set(), 0
    for qi in range(Q.n):
        x, mq, K = Q.get(qi), Q.lengths()[qi], int(kq[qi])
        a = oracle.find_anchors(x, 4, 4, oracle.target_partitions(K, t_div))
        for k in range(len(a) - 1):
            pq = int(a[k])
            for s, ps in by.get(x[a[k]:a[k + 1]].tobytes(), []):
                ms = int(I.lengths()[s])
                if abs(mq - ms) <= K and abs(pq - ps) + abs((mq - pq) - (ms - ps)) <= K:
                    want_c.add((qi << 32) | s)
    for v in want_c:
        d = oracle.edit_distance(Q.get(v >> 32), I.get(v & 0xFFFFFFFF))
        if d <= int(kq[v >> 32]):
            want_o.add(v)
        elif d <= KI:
            wider += 1
    assert set(cand.tolist()) == want_c
    assert set(got.tolist()) == want_o
    assert want_o and wider > 0  # the case distinguishes K_q from max(K_q, K_s)


def test_search_per_query_threshold_is_the_union_of_single_query_searches():
    I, Q = _split_search_fixture(44)
    rng = np.random.default_rng(4)
    kq = rng.integers(30, 80, Q.n).astype(np.int32)
    ip = oracle.make_params(4, 4, k=70, t_div=1)
    _, got = oracle.search(I.chars, I.offsets, ip, Q.chars, Q.offsets,
                           oracle.make_params(4, 4, k_per_string=kq, t_div=1))
    want = set()
    for qi in range(Q.n):
        one = dg.from_list([Q.get(qi)], 4)
        _, o = oracle.search(I.chars, I.offsets, ip, one.chars, one.offsets,
                             oracle.make_params(4, 4, k=int(kq[qi]), t_div=1))
        want |= {(qi << 32) | (int(v) & 0xFFFFFFFF) for v in o.tolist()}
    assert set(got.tolist()) == want and want
