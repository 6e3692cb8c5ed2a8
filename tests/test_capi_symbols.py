"""The C-ABI library loads on the CPU host and exports every function that
include/minjoin.h declares (no compute call: there may be no GPU here)."""
import ctypes
import os
import re

import paper_1810_08833_amd as mj

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "minjoin.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mj_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("mj_join", "mj_search", "mj_index_build", "mj_partition", "mj_candidates",
                 "mj_verify", "mj_ctx_create", "mj_last_error"):
        assert must in names


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(mj.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    assert set(mj.EXPORTS) == set(declared_functions())


def test_version_and_error_strings_without_a_device():
    lib = mj.load_library()
    assert b"gfx950" in lib.mj_version()
    assert isinstance(lib.mj_last_error(), bytes)


def test_null_arguments_are_rejected_before_any_device_work():
    lib = mj.load_library()
    out = ctypes.c_void_p()
    assert lib.mj_join(None, None, None, None, ctypes.byref(out), None) == mj.MJ_EINVAL
    assert lib.mj_ctx_create(0, None, None) == mj.MJ_EINVAL
    bad = mj.MjAllocator()  # an allocator without alloc/free
    assert lib.mj_ctx_create(0, ctypes.byref(bad), ctypes.byref(out)) == mj.MJ_EINVAL
    assert lib.mj_pairs_copy_to_host(None, None, 0) == mj.MJ_EINVAL
    assert lib.mj_ctx_set_pair_test_pass(None, 1 << 20) == mj.MJ_EINVAL
    assert lib.mj_ctx_set_member_filter(None, 0, 0) == mj.MJ_EINVAL
    assert lib.mj_ctx_set_tile_emission(None, 0) == mj.MJ_EINVAL
    assert lib.mj_pairs_count(None) == 0
    assert lib.mj_records_count(None) == 0
    lib.mj_pairs_free(None)
    lib.mj_records_free(None)
    lib.mj_index_free(None)
    lib.mj_ctx_destroy(None)


def test_two_bit_packing_layout():
    """MJ_PACK_2BIT: four symbols per byte, the first in the low bits, whole 32-bit words."""
    import numpy as np
    rng = np.random.default_rng(1)
    for n in (0, 1, 15, 16, 17, 1000):
        c = rng.integers(0, 4, n).astype(np.uint8)
        w = mj.pack_2bit(c)
        assert w.dtype == np.dtype("<u4") and len(w) == -(-n // 16)
        bits = np.unpackbits(w.view(np.uint8), bitorder="little").reshape(-1, 2)
        back = (bits[:, 0] | (bits[:, 1] << 1)).astype(np.uint8)
        assert np.array_equal(back[:n], c) and not back[n:].any()
