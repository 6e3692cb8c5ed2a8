"""Error paths of the C-ABI on the GPU: arguments the entry points must refuse (and the
message they give), inputs that name out-of-range symbols, limits of the server's
admission, and an index that must not depend on its caller's buffers after the build.
Every failing call is refused by a host check or a bounds-checked device pass; no
kernel is made to fault."""
import ctypes
import sys

import numpy as np
import pytest

import oracle
from paper_1810_08833_amd import datagen as dg

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


def status_of(fn):
    import paper_1810_08833_amd as mj
    with pytest.raises(mj.MinJoinError) as e:
        fn()
    return e.value.status


@pytest.mark.parametrize("bad", [dict(q=0), dict(q=33), dict(t_div=0), dict(k=-2), dict(reps=-1),
                                 dict(verifier=7), dict(verify_lanes=3), dict(verify_lanes=16)])
def test_join_rejects_bad_parameters(mj, bad):
    say("join rejects", bad)
    S = dg.dna_small(seed=3, n_clusters=3, copies=3)
    kw = dict(q=4, k=20, t_div=1)
    kw.update(bad)
    p = mj.Params(**kw)
    assert status_of(lambda: mj.join(dev(mj, S), p)) == mj.MJ_EINVAL


def test_search_rejects_bad_verifier_arguments(mj):
    say("search rejects verify_lanes 3 and 16, verifier 5")
    S = dg.dna_small(seed=4, n_clusters=4, copies=3)
    index = mj.Index(dev(mj, S), mj.Params(q=4, k=40, t_div=1))
    Q = dg.from_list([S.get(0), S.get(4)], 4)
    for kw in (dict(verify_lanes=3), dict(verify_lanes=16), dict(verifier=5)):
        assert status_of(lambda: index.search(dev(mj, Q), k=40, **kw)) == mj.MJ_EINVAL
    got, _ = index.search(dev(mj, Q), k=40)  # the index still answers
    assert len(got) > 0
    index.close()


def test_band_classes_refuse_bands_wider_than_their_widest_window(mj):
    """verify_lanes -3 holds bands of up to 32 window words (K <= 992): a call with K = 1500
    fails with ECAPACITY; the same call with the timed layout verifies."""
    say("band classes, K = 1500")
    rng = np.random.default_rng(9)
    x = rng.integers(0, 4, 3000).astype(np.uint8)
    S = dg.from_list([x, dg.mutate(rng, x, 0.2, 4)], 4)
    pairs = np.array([1], dtype=np.uint64)  # (0, 1)
    p = mj.Params(q=4, k=1500, t_div=1, verify_lanes=-3)
    assert status_of(lambda: mj.verify(dev(mj, S), p, pairs)) == mj.MJ_ECAPACITY
    p.verify_lanes = 0
    assert mj.verify(dev(mj, S), p, pairs).tolist() == [1]


def test_out_of_range_symbols_are_rejected(mj):
    say("symbol codes >= sigma")
    S = dg.dna_small(seed=5, n_clusters=3, copies=3)
    chars = S.chars.copy()
    chars[len(chars) // 2] = 4  # sigma is 4
    bad = mj.DeviceStrings.from_host(chars, S.offsets, 4)
    p = mj.Params(q=4, k=30, t_div=1)
    assert status_of(lambda: mj.join(bad, p)) == mj.MJ_EINVAL
    assert status_of(lambda: mj.candidates(bad, p)) == mj.MJ_EINVAL
    assert status_of(lambda: mj.partition(bad, p)) == mj.MJ_EINVAL
    assert status_of(lambda: mj.verify(bad, p, np.array([1], np.uint64))) == mj.MJ_EINVAL
    assert status_of(lambda: mj.Index(bad, p)) == mj.MJ_EINVAL
    # the same collection as 37 symbols is valid
    ok, _ = mj.join(mj.DeviceStrings.from_host(chars, S.offsets, 37), mj.Params(q=4, k=30, t_div=1))
    assert ok.dtype == np.uint64


def test_server_refuses_requests_it_cannot_admit(mj):
    say("server admission limits")
    S = dg.random_strings(92, 50, 200, 400)
    index = mj.Index(dev(mj, S), mj.Params(q=4, k=20, t_div=1))
    srv = mj.Server(index, workers=1, max_batch=4, memory_budget=(8 << 20) + 8192)
    # a batch's estimate is 8 MiB plus 96 bytes per symbol + 4 KiB per query: one query of
    # 100 symbols (8 MiB + 13.4 KiB) exceeds the budget
    assert status_of(lambda: srv.submit(S.get(0)[:100], 10, 1)) == mj.MJ_EINVAL
    assert status_of(lambda: srv.submit(np.array([0, 1, 9], np.uint8), 1, 2)) == mj.MJ_EINVAL
    assert status_of(lambda: srv.submit(S.get(0)[:10], 4000, 3)) == mj.MJ_EINVAL
    srv.submit(S.get(0)[:20], 2, 4)  # 20 symbols: 8 MiB + 5.9 KiB fits
    rep = []
    while not rep:
        rep = srv.poll(timeout_ms=10000)
    assert rep[0]["tag"] == 4 and rep[0]["status"] == 0
    srv.close()
    index.close()


def test_index_keeps_its_own_pi_table(mj):
    """An index built with an injected Pi table still partitions its queries with that
    table after the caller's tensor is gone and its memory is reused."""
    import torch
    say("index with pi_table, caller's table freed")
    rng = np.random.default_rng(12)
    q = 5
    table = rng.permutation(1 << (2 * q)).astype(np.uint64) * np.uint64(0x9E3779B1)
    S = dg.dna_small(seed=13, n_clusters=12, copies=4)
    ids = np.arange(S.n)
    I, Q = S.subset(ids[ids % 4 != 0]), S.subset(ids[ids % 4 == 0])
    tab = torch.from_numpy(table.view(np.int64)).cuda()
    index = mj.Index(dev(mj, I), mj.Params(q=q, k=80, t_div=1, pi_table=tab))
    del tab
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    junk = [torch.full((1 << 14,), -1, dtype=torch.int64, device="cuda") for _ in range(64)]
    torch.cuda.synchronize()
    got, _ = index.search(dev(mj, Q), k=80)
    _, want = oracle.search(I.chars, I.offsets, oracle.make_params(q, 4, k=80, t_div=1, pi_table=table),
                            Q.chars, Q.offsets, oracle.make_params(q, 4, k=80, t_div=1, pi_table=table))
    assert len(want) > 0 and np.array_equal(got, want)
    del junk
    index.close()


def test_context_settings_reject_bad_values(mj):
    """The context's tuning switches reject out-of-range values with EINVAL and keep
    working afterwards."""
    say("context settings")
    ctx = mj.Context()
    assert status_of(lambda: ctx.set_tile_emission(-2)) == mj.MJ_EINVAL
    assert status_of(lambda: ctx.set_pair_test_pass(1023)) == mj.MJ_EINVAL
    assert status_of(lambda: ctx.set_member_filter(-2)) == mj.MJ_EINVAL
    ctx.set_tile_emission(-1)
    ctx.set_tile_emission(0)
    S = dg.dna_small(seed=5, n_clusters=4, copies=3)
    out, st = mj.join(dev(mj, S), mj.Params(q=4, k=20, t_div=1), ctx=ctx)
    assert st["candidates"] >= out.size
    ctx.close()

