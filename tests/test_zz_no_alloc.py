"""The allocation-free verification entry point (mj_verify_noalloc), called through the
C-ABI, against mj_verify on the same inputs: two calls in a row, the second smaller, and
a call larger than its fixed scratch, which must fail before writing any flag."""
import ctypes
import sys

import numpy as np
import pytest

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


def pair_set(seed, n_pairs, sigma, kmax):
    """Pairs of a random string and a mutated copy near its threshold, plus random
    cross pairs; per-string thresholds up to kmax."""
    rng = np.random.default_rng(seed)
    strs, ks = [], []
    for _ in range(n_pairs):
        K = int(rng.integers(0, kmax + 1))
        L = int(rng.integers(max(1, K // 2), 4 * K + 60))
        x = rng.integers(0, sigma, L).astype(np.uint8)
        y = dg.mutate(rng, x, min(0.9, rng.uniform(0.5, 1.5) * (K + 1) / L), sigma)
        strs += [x, y]
        ks += [K, int(rng.integers(0, K + 1))]
    S = dg.from_list(strs, sigma)
    idx = np.arange(0, 2 * n_pairs, 2, dtype=np.uint64)
    pairs = np.concatenate([(idx << np.uint64(32)) | (idx + np.uint64(1)),
                            (rng.integers(0, 2 * n_pairs, n_pairs).astype(np.uint64) << np.uint64(32))
                            | rng.integers(0, 2 * n_pairs, n_pairs).astype(np.uint64)])
    return S, np.array(ks, np.int32), pairs


def call_noalloc(mj, ds, params, pairs_t, flags_t):
    import torch
    L = mj.load_library()
    s, p = ds.struct(), params.struct()
    st = L.mj_verify_noalloc(ctypes.byref(s), ctypes.byref(p), ctypes.c_void_p(pairs_t.data_ptr()),
                             int(pairs_t.numel()), ctypes.c_void_p(flags_t.data_ptr()),
                             ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    return st


@pytest.mark.parametrize("sigma", [4, 25])
def test_noalloc_verify_equals_verify_twice_then_smaller(mj, sigma):
    import torch
    for call, (n_pairs, kmax) in enumerate([(3000, 300), (700, 60)]):
        say("noalloc verify sigma=%d call %d: %d pairs, K <= %d" % (sigma, call, n_pairs, kmax))
        S, ks, pairs = pair_set(100 * sigma + call, n_pairs, sigma, kmax)
        ds = mj.DeviceStrings.from_host(S.chars, S.offsets, sigma)
        params = mj.Params(q=4, k_per_string=torch.from_numpy(ks).cuda())
        want = mj.verify(ds, params, pairs)
        pt = torch.from_numpy(pairs.view(np.int64)).cuda()
        flags = torch.full((len(pairs),), 7, dtype=torch.uint8, device="cuda")
        assert call_noalloc(mj, ds, params, pt, flags) == mj.MJ_OK, mj.load_library().mj_last_error()
        got = flags.cpu().numpy()
        assert set(np.unique(got).tolist()) <= {0, 1}
        assert np.array_equal(got.astype(bool), want)
        assert 0 < want.sum() < len(want)


def test_noalloc_rejects_a_call_beyond_its_scratch(mj):
    import torch
    say("noalloc verify beyond the scratch size")
    S = dg.from_list([np.arange(100, dtype=np.uint8) % 4, np.arange(90, dtype=np.uint8) % 4], 4)
    ds = mj.DeviceStrings.from_host(S.chars, S.offsets, 4)
    n = 9_000_000  # 72 MB of longest-first order alone
    pt = torch.ones(n, dtype=torch.int64, device="cuda")  # pair (0, 1)
    flags = torch.full((n,), 7, dtype=torch.uint8, device="cuda")
    st = call_noalloc(mj, ds, mj.Params(q=4, k=20), pt, flags)
    assert st == mj.MJ_ECAPACITY
    assert b"scratch" in mj.load_library().mj_last_error()
    torch.cuda.synchronize()
    assert int(flags.min()) == 7 and int(flags.max()) == 7
    # and the next call works
    small = torch.ones(5, dtype=torch.int64, device="cuda")
    f2 = torch.zeros(5, dtype=torch.uint8, device="cuda")
    assert call_noalloc(mj, ds, mj.Params(q=4, k=20), small, f2) == mj.MJ_OK
    assert np.array_equal(f2.cpu().numpy().astype(bool), mj.verify(ds, mj.Params(q=4, k=20), np.ones(5, np.uint64)))
