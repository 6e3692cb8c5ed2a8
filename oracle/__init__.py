"""MinJoin oracle -- TEST INFRASTRUCTURE ONLY.

A ctypes front end to ``minjoin_oracle.c``: a plain CPU implementation of MinJoin
(Zhang & Zhang, arXiv:1810.08833, Algorithms 1-3) that the GPU library is checked
against.  Only the tests, the smoke check and the benchmark's CPU-baseline leg may
import this package; the product path never does and shares no code with it.

Strings are passed as one ``uint8`` array of symbol codes plus ``int64`` offsets
(``n + 1`` entries).  Pairs come back as sorted ``uint64`` values ``lo << 32 | hi``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "minjoin_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (building the checker is not using it)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=gnu11", "-fopenmp", "-shared", "-fPIC",
                               "-Wall", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


class Params(ctypes.Structure):
    _fields_ = [("q", ctypes.c_int32), ("sigma", ctypes.c_int32), ("seed", ctypes.c_uint64),
                ("t_div", ctypes.c_int32), ("t_fixed", ctypes.c_int32), ("reps", ctypes.c_int32),
                ("threads", ctypes.c_int32), ("k", ctypes.c_int64),
                ("k_per_string", ctypes.c_void_p), ("pi_table", ctypes.c_void_p)]


class Record(ctypes.Structure):
    _fields_ = [("key", ctypes.c_uint64), ("sid", ctypes.c_int32), ("pos", ctypes.c_int32),
                ("len", ctypes.c_int32), ("rep", ctypes.c_int32)]


class Stats(ctypes.Structure):
    _fields_ = [("records", ctypes.c_int64), ("candidates", ctypes.c_int64),
                ("output", ctypes.c_int64), ("pair_tests", ctypes.c_int64),
                ("partition_s", ctypes.c_double), ("join_s", ctypes.c_double),
                ("dedup_s", ctypes.c_double), ("verify_s", ctypes.c_double)]


RECORD_DTYPE = np.dtype([("key", "<u8"), ("sid", "<i4"), ("pos", "<i4"), ("len", "<i4"),
                         ("rep", "<i4")])

_lib = None
P = ctypes.POINTER
VP = ctypes.c_void_p


def lib():
    global _lib
    if _lib is None:
        _lib = ctypes.CDLL(build())
        L = _lib
        L.orc_mix64.restype = ctypes.c_uint64
        L.orc_mix64.argtypes = [ctypes.c_uint64]
        L.orc_symbol_bits.restype = ctypes.c_int
        L.orc_pi_salt.restype = ctypes.c_uint64
        L.orc_pi_salt.argtypes = [ctypes.c_uint64]
        L.orc_phi_base.restype = ctypes.c_uint64
        L.orc_phi_base.argtypes = [ctypes.c_uint64]
        L.orc_radius.restype = ctypes.c_int64
        L.orc_radius.argtypes = [ctypes.c_int64, ctypes.c_int, ctypes.c_int64]
        L.orc_target_partitions.restype = ctypes.c_int64
        L.orc_target_partitions.argtypes = [ctypes.c_int64, ctypes.c_int, ctypes.c_int]
        L.orc_qgram_hashes.restype = None
        L.orc_qgram_hashes.argtypes = [VP, ctypes.c_int64, ctypes.c_int, ctypes.c_int,
                                       ctypes.c_uint64, VP, VP]
        L.orc_find_anchors.restype = ctypes.c_int64
        L.orc_find_anchors.argtypes = [VP, ctypes.c_int64, ctypes.c_int, ctypes.c_int,
                                       ctypes.c_int64, ctypes.c_uint64, VP, VP]
        L.orc_partition_phi.restype = ctypes.c_uint64
        L.orc_partition_phi.argtypes = [VP, ctypes.c_int64, ctypes.c_uint64]
        L.orc_partition_key.restype = ctypes.c_uint64
        L.orc_partition_key.argtypes = [VP, ctypes.c_int64, ctypes.c_uint64]
        L.orc_partition_all.restype = ctypes.c_int64
        L.orc_partition_all.argtypes = [VP, VP, ctypes.c_int32, P(Params), P(VP)]
        L.orc_edit_distance.restype = ctypes.c_int64
        L.orc_edit_distance.argtypes = [VP, ctypes.c_int64, VP, ctypes.c_int64]
        L.orc_ed_within.restype = ctypes.c_int
        L.orc_ed_within.argtypes = [VP, ctypes.c_int64, VP, ctypes.c_int64, ctypes.c_int64]
        L.orc_join.restype = ctypes.c_int
        L.orc_join.argtypes = [VP, VP, ctypes.c_int32, P(Params), P(VP), P(ctypes.c_int64),
                               P(VP), P(ctypes.c_int64), P(Stats)]
        L.orc_join_candidates.restype = ctypes.c_int
        L.orc_join_candidates.argtypes = L.orc_join.argtypes
        L.orc_search.restype = ctypes.c_int
        L.orc_search.argtypes = [VP, VP, ctypes.c_int32, P(Params), VP, VP, ctypes.c_int32,
                                 P(Params), P(VP), P(ctypes.c_int64), P(VP), P(ctypes.c_int64)]
        L.orc_verify_list.restype = None
        L.orc_verify_list.argtypes = [VP, VP, P(Params), VP, ctypes.c_int64, VP]
        L.orc_max_threads.restype = ctypes.c_int
        L.orc_free.restype = None
        L.orc_free.argtypes = [VP]
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _u8(a):
    return np.ascontiguousarray(a, dtype=np.uint8)


def make_params(q, sigma, k=None, k_per_string=None, seed=0, t_div=5, t_fixed=0, reps=1,
                threads=None, pi_table=None):
    """Build a Params struct; keeps referenced arrays alive on the returned object."""
    p = Params()
    p.q, p.sigma, p.seed = int(q), int(sigma), int(seed)
    p.t_div, p.t_fixed, p.reps = int(t_div), int(t_fixed), int(reps)
    p.threads = int(threads if threads is not None else lib().orc_max_threads())
    keep = []
    if k_per_string is not None:
        kp = np.ascontiguousarray(k_per_string, dtype=np.int32)
        keep.append(kp)
        p.k, p.k_per_string = -1, kp.ctypes.data
    else:
        p.k, p.k_per_string = int(k), None
    if pi_table is not None:
        tb = np.ascontiguousarray(pi_table, dtype=np.uint64)
        keep.append(tb)
        p.pi_table = tb.ctypes.data
    else:
        p.pi_table = None
    p._keep = keep
    return p


def mix64(z: int) -> int:
    return lib().orc_mix64(z & 0xFFFFFFFFFFFFFFFF)


def symbol_bits(sigma: int) -> int:
    return lib().orc_symbol_bits(int(sigma))


def radius(m: int, q: int, T: int) -> int:
    return lib().orc_radius(m, q, T)


def target_partitions(K: int, t_div: int, t_fixed: int = 0) -> int:
    return lib().orc_target_partitions(K, t_div, t_fixed)


def qgram_hashes(s, q, sigma, seed=0, pi_table=None):
    s = _u8(s)
    n = max(0, len(s) - q + 1)
    out = np.zeros(n, dtype=np.uint64)
    tb = None if pi_table is None else np.ascontiguousarray(pi_table, dtype=np.uint64)
    lib().orc_qgram_hashes(_ptr(s), len(s), q, symbol_bits(sigma), seed, _ptr(tb), _ptr(out))
    return out


def find_anchors(s, q, sigma, T, seed=0, pi_table=None):
    s = _u8(s)
    out = np.zeros(len(s) + 2, dtype=np.int64)
    tb = None if pi_table is None else np.ascontiguousarray(pi_table, dtype=np.uint64)
    na = lib().orc_find_anchors(_ptr(s), len(s), q, symbol_bits(sigma), T, seed, _ptr(tb),
                                _ptr(out))
    return out[:na].copy()


def partition_phi(x, seed=0) -> int:
    x = _u8(x)
    return lib().orc_partition_phi(_ptr(x), len(x), seed)


def partition_key(x, seed=0) -> int:
    x = _u8(x)
    return lib().orc_partition_key(_ptr(x), len(x), seed)


def partition_all(chars, offsets, params):
    """All partition records (key, sid, pos, len, rep) in string order."""
    chars = _u8(chars)
    offsets = np.ascontiguousarray(offsets, dtype=np.int64)
    n = len(offsets) - 1
    out = ctypes.c_void_p()
    R = lib().orc_partition_all(_ptr(chars), _ptr(offsets), n, ctypes.byref(params),
                                ctypes.byref(out))
    if R:
        res = np.frombuffer(ctypes.string_at(out, R * RECORD_DTYPE.itemsize), dtype=RECORD_DTYPE).copy()
    else:
        res = np.zeros(0, RECORD_DTYPE)
    lib().orc_free(out)
    return res


def _take_u64(ptr, n):
    if n == 0:
        lib().orc_free(ptr)
        return np.zeros(0, dtype=np.uint64)
    a = np.ctypeslib.as_array(ctypes.cast(ptr, P(ctypes.c_uint64)), shape=(n,)).copy()
    lib().orc_free(ptr)
    return a


def join(chars, offsets, params, verify=True):
    """Returns (candidates, pairs, stats): sorted uint64 arrays lo<<32|hi and a dict.
    With verify=False the verification stage is skipped and pairs is empty."""
    chars = _u8(chars)
    offsets = np.ascontiguousarray(offsets, dtype=np.int64)
    n = len(offsets) - 1
    cp, pp = ctypes.c_void_p(), ctypes.c_void_p()
    nc, npairs = ctypes.c_int64(), ctypes.c_int64()
    st = Stats()
    fn = lib().orc_join if verify else lib().orc_join_candidates
    fn(_ptr(chars), _ptr(offsets), n, ctypes.byref(params), ctypes.byref(cp),
       ctypes.byref(nc), ctypes.byref(pp), ctypes.byref(npairs), ctypes.byref(st))
    cand = _take_u64(cp, nc.value)
    pairs = _take_u64(pp, npairs.value)
    return cand, pairs, {"records": st.records, "candidates": st.candidates,
                         "output": st.output, "pair_tests": st.pair_tests,
                         "stage_s": {"partition": st.partition_s, "join": st.join_s,
                                     "dedup": st.dedup_s, "verify": st.verify_s}}


def search(ichars, ioffsets, iparams, qchars, qoffsets, qparams):
    """Returns (candidates, pairs): sorted uint64 arrays qid<<32|sid."""
    ichars, qchars = _u8(ichars), _u8(qchars)
    ioffsets = np.ascontiguousarray(ioffsets, dtype=np.int64)
    qoffsets = np.ascontiguousarray(qoffsets, dtype=np.int64)
    cp, pp = ctypes.c_void_p(), ctypes.c_void_p()
    nc, npairs = ctypes.c_int64(), ctypes.c_int64()
    lib().orc_search(_ptr(ichars), _ptr(ioffsets), len(ioffsets) - 1, ctypes.byref(iparams),
                     _ptr(qchars), _ptr(qoffsets), len(qoffsets) - 1, ctypes.byref(qparams),
                     ctypes.byref(cp), ctypes.byref(nc), ctypes.byref(pp), ctypes.byref(npairs))
    return _take_u64(cp, nc.value), _take_u64(pp, npairs.value)


def edit_distance(x, y) -> int:
    x, y = _u8(x), _u8(y)
    return lib().orc_edit_distance(_ptr(x), len(x), _ptr(y), len(y))


def ed_within(x, y, K) -> bool:
    x, y = _u8(x), _u8(y)
    return bool(lib().orc_ed_within(_ptr(x), len(x), _ptr(y), len(y), K))


def verify_list(chars, offsets, params, pairs):
    chars = _u8(chars)
    offsets = np.ascontiguousarray(offsets, dtype=np.int64)
    pairs = np.ascontiguousarray(pairs, dtype=np.uint64)
    flags = np.zeros(len(pairs), dtype=np.uint8)
    lib().orc_verify_list(_ptr(chars), _ptr(offsets), ctypes.byref(params), _ptr(pairs),
                          len(pairs), _ptr(flags))
    return flags.astype(bool)


def max_threads() -> int:
    return lib().orc_max_threads()
