"""MinJoin on MI355X: Python binding of libminjoin.so (C-ABI in include/minjoin.h).

The binding only marshals arguments: strings live in torch tensors on the GPU
(``chars``: uint8 symbol codes, ``offsets``: int64, n + 1 entries), the stream is
torch's current HIP stream, and every step of the method runs in the library's HIP
kernels.  Pair results are uint64 values ``a << 32 | b`` copied to host NumPy arrays.

If the library is not built (``python -m paper_1810_08833_amd.build``) every call raises
``RuntimeError``: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libminjoin.so")

MJ_OK, MJ_EINVAL, MJ_ENOMEM, MJ_EDEVICE, MJ_ECAPACITY = 0, 1, 2, 3, 4
VERIFY_BATCHED, VERIFY_PLAIN = 0, 1
STATUS_NAMES = {0: "MJ_OK", 1: "MJ_EINVAL", 2: "MJ_ENOMEM", 3: "MJ_EDEVICE", 4: "MJ_ECAPACITY"}
KERNELS = ["anchors", "records", "emit", "verify"]
STAGES = ["setup", "partition", "sort", "group_filter", "dedup", "verify", "output", "unused"]


PACK_U8, PACK_2BIT = 0, 1


class MjStrings(ctypes.Structure):
    _fields_ = [("chars", ctypes.c_void_p), ("offsets", ctypes.c_void_p), ("n", ctypes.c_int32),
                ("sigma", ctypes.c_int32), ("packing", ctypes.c_int32), ("reserved", ctypes.c_int32)]


ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)


class MjAllocator(ctypes.Structure):
    _fields_ = [("alloc", ALLOC_FN), ("free", FREE_FN), ("user", ctypes.c_void_p)]


class MjParams(ctypes.Structure):
    _fields_ = [("q", ctypes.c_int32), ("t_div", ctypes.c_int32), ("t_fixed", ctypes.c_int32),
                ("reps", ctypes.c_int32), ("seed", ctypes.c_uint64), ("k", ctypes.c_int64),
                ("k_per_string", ctypes.c_void_p), ("pi_table", ctypes.c_void_p),
                ("verifier", ctypes.c_int32), ("verify_lanes", ctypes.c_int32)]


class MjStats(ctypes.Structure):
    _fields_ = [("records", ctypes.c_int64), ("groups", ctypes.c_int64),
                ("pair_tests", ctypes.c_int64), ("candidates", ctypes.c_int64),
                ("output", ctypes.c_int64), ("band_cells", ctypes.c_int64),
                ("stage_ms", ctypes.c_float * 8), ("kernel_ms", ctypes.c_float * 4),
                ("kernel_launches", ctypes.c_int32 * 4), ("positions", ctypes.c_int64),
                ("verify_group", ctypes.c_int32), ("verify_words", ctypes.c_int32),
                ("verify_blocks", ctypes.c_int32), ("streamed", ctypes.c_int32),
                ("host_reads", ctypes.c_int32), ("member_filter", ctypes.c_int32),
                ("members", ctypes.c_int64)]

    def as_dict(self):
        d = {k: getattr(self, k) for k in ("records", "groups", "pair_tests", "candidates",
                                           "output", "band_cells", "positions", "verify_group",
                                           "verify_words", "verify_blocks", "streamed",
                                           "host_reads", "member_filter", "members")}
        d["stage_ms"] = {STAGES[i]: float(self.stage_ms[i]) for i in range(7)}
        d["kernel_ms"] = {KERNELS[i]: float(self.kernel_ms[i]) for i in range(4)}
        d["kernel_launches"] = {KERNELS[i]: int(self.kernel_launches[i]) for i in range(4)}
        return d


class MjServerConfig(ctypes.Structure):
    _fields_ = [("workers", ctypes.c_int32), ("max_batch", ctypes.c_int32),
                ("memory_budget", ctypes.c_int64)]


class MjReply(ctypes.Structure):
    _fields_ = [("tag", ctypes.c_uint64), ("status", ctypes.c_int32), ("count", ctypes.c_int32),
                ("offset", ctypes.c_int64), ("batch_size", ctypes.c_int32),
                ("worker", ctypes.c_int32), ("submit_ms", ctypes.c_double),
                ("start_ms", ctypes.c_double), ("done_ms", ctypes.c_double),
                ("batch_estimate", ctypes.c_int64), ("batch_device", ctypes.c_int64)]


EXPORTS = ["mj_ctx_create", "mj_ctx_destroy", "mj_ctx_set_streaming", "mj_ctx_set_pair_test_pass",
           "mj_ctx_set_member_filter", "mj_ctx_set_tile_emission",
           "mj_last_error", "mj_version", "mj_join",
           "mj_partition", "mj_candidates", "mj_verify", "mj_index_build", "mj_index_free",
           "mj_index_records", "mj_index_bytes", "mj_search", "mj_pairs_count", "mj_pairs_device",
           "mj_pairs_copy_to_host", "mj_pairs_free", "mj_records_count",
           "mj_records_copy_to_host", "mj_records_free", "mj_server_create", "mj_server_submit",
           "mj_server_poll", "mj_server_pending", "mj_server_destroy", "mj_verify_noalloc"]

_lib = None


class MinJoinError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s: %s" % (STATUS_NAMES.get(status, status), msg))
        self.status = status


def load_library(path: str = LIB_PATH):
    """Loads libminjoin.so and declares its C signatures.  Raises if it is not built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError("libminjoin.so is not built (%s); run "
                           "`python -m paper_1810_08833_amd.build`" % path)
    L = ctypes.CDLL(path)
    P, VP, I64 = ctypes.POINTER, ctypes.c_void_p, ctypes.c_int64
    L.mj_ctx_create.argtypes = [ctypes.c_int, P(MjAllocator), P(VP)]
    L.mj_ctx_destroy.argtypes = [VP]
    L.mj_ctx_destroy.restype = None
    L.mj_ctx_set_streaming.argtypes = [VP, ctypes.c_int]
    L.mj_ctx_set_streaming.restype = ctypes.c_int
    L.mj_ctx_set_pair_test_pass.argtypes = [VP, ctypes.c_int64]
    L.mj_ctx_set_pair_test_pass.restype = ctypes.c_int
    L.mj_ctx_set_member_filter.argtypes = [VP, ctypes.c_int64, ctypes.c_int32]
    L.mj_ctx_set_member_filter.restype = ctypes.c_int
    L.mj_ctx_set_tile_emission.argtypes = [VP, ctypes.c_int64]
    L.mj_ctx_set_tile_emission.restype = ctypes.c_int
    L.mj_last_error.restype = ctypes.c_char_p
    L.mj_version.restype = ctypes.c_char_p
    L.mj_join.argtypes = [VP, P(MjStrings), P(MjParams), VP, P(VP), P(MjStats)]
    L.mj_candidates.argtypes = [VP, P(MjStrings), P(MjParams), VP, P(VP), P(MjStats)]
    L.mj_partition.argtypes = [VP, P(MjStrings), P(MjParams), VP, P(VP)]
    L.mj_verify.argtypes = [VP, P(MjStrings), P(MjParams), VP, I64, VP, VP]
    L.mj_verify_noalloc.argtypes = [P(MjStrings), P(MjParams), VP, I64, VP, VP]
    L.mj_index_build.argtypes = [VP, P(MjStrings), P(MjParams), VP, P(VP)]
    L.mj_index_free.argtypes = [VP]
    L.mj_index_free.restype = None
    L.mj_index_records.argtypes = [VP]
    L.mj_index_records.restype = I64
    L.mj_index_bytes.argtypes = [VP]
    L.mj_index_bytes.restype = I64
    L.mj_search.argtypes = [VP, VP, P(MjStrings), P(MjParams), VP, P(VP), P(MjStats)]
    L.mj_pairs_count.argtypes = [VP]
    L.mj_pairs_count.restype = I64
    L.mj_pairs_device.argtypes = [VP]
    L.mj_pairs_device.restype = VP
    L.mj_pairs_copy_to_host.argtypes = [VP, VP, I64]
    L.mj_pairs_free.argtypes = [VP]
    L.mj_pairs_free.restype = None
    L.mj_records_count.argtypes = [VP]
    L.mj_records_count.restype = I64
    L.mj_records_copy_to_host.argtypes = [VP, VP, VP, VP, VP, I64]
    L.mj_records_free.argtypes = [VP]
    L.mj_records_free.restype = None
    L.mj_server_create.argtypes = [ctypes.c_int, VP, P(MjServerConfig), P(VP)]
    L.mj_server_submit.argtypes = [VP, VP, ctypes.c_int32, ctypes.c_int32, ctypes.c_uint64]
    L.mj_server_poll.argtypes = [VP, P(MjReply), ctypes.c_int32, VP, I64, ctypes.c_int32,
                                 P(ctypes.c_int32), P(I64)]
    L.mj_server_pending.argtypes = [VP]
    L.mj_server_pending.restype = I64
    L.mj_server_destroy.argtypes = [VP]
    L.mj_server_destroy.restype = None
    for fn in ("mj_server_create", "mj_server_submit", "mj_server_poll"):
        getattr(L, fn).restype = ctypes.c_int
    for fn in ("mj_ctx_create", "mj_join", "mj_candidates", "mj_partition", "mj_verify",
               "mj_verify_noalloc",
               "mj_index_build", "mj_search", "mj_pairs_copy_to_host", "mj_records_copy_to_host"):
        getattr(L, fn).restype = ctypes.c_int
    _lib = L
    return L


def _check(status):
    if status != MJ_OK:
        raise MinJoinError(status, load_library().mj_last_error().decode())


def _torch():
    import torch
    return torch


def _stream_ptr(stream=None):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


class TorchAllocator:
    """An mj_allocator backed by torch's caching allocator (torch.cuda.caching_allocator_alloc
    and _delete on the context's device), so that the library's device buffers come from the
    same pool as the framework's tensors.  Counts the blocks it hands out and takes back."""

    def __init__(self, device: int):
        self.device = device
        self.allocs = 0
        self.frees = 0
        self.live = {}

        def _alloc(nbytes, user):
            torch = _torch()
            try:
                p = torch.cuda.caching_allocator_alloc(int(nbytes), self.device)
            except Exception:
                return None
            self.allocs += 1
            self.live[p] = int(nbytes)
            return p

        def _free(ptr, user):
            torch = _torch()
            self.frees += 1
            self.live.pop(ptr, None)
            torch.cuda.caching_allocator_delete(ptr)

        self._alloc_cb = ALLOC_FN(_alloc)
        self._free_cb = FREE_FN(_free)
        self.struct = MjAllocator(self._alloc_cb, self._free_cb, None)


class Context:
    """Owns an mj_ctx (device workspace) on one GPU.  allocator: None (the library's own
    hipMalloc) or a TorchAllocator whose pool backs every device buffer of the context."""

    def __init__(self, device: Optional[int] = None, allocator: Optional[TorchAllocator] = None):
        torch = _torch()
        L = load_library()
        self.device = torch.cuda.current_device() if device is None else int(device)
        self.allocator = allocator  # kept alive as long as the context
        h = ctypes.c_void_p()
        _check(L.mj_ctx_create(self.device, ctypes.byref(allocator.struct) if allocator else None,
                               ctypes.byref(h)))
        self.handle = h

    def set_streaming(self, mode):
        """0 (or False): stage by stage; 1 (or True): streamed, two host reads per join;
        2: streamed and captured into HIP graphs, replayed while inputs repeat."""
        _check(load_library().mj_ctx_set_streaming(self.handle, int(mode)))

    def set_pair_test_pass(self, tests: int):
        """Record-pair tests per emission pass (joins with more run in passes)."""
        _check(load_library().mj_ctx_set_pair_test_pass(self.handle, int(tests)))

    def set_tile_emission(self, min_tile_pairs: int):
        """Joins whose groups of 64 records or more hold at least min_tile_pairs 64 x 64
        tile pairs (0: every such join, -1: none) test those groups by tile pairs."""
        _check(load_library().mj_ctx_set_tile_emission(self.handle, int(min_tile_pairs)))

    def set_member_filter(self, min_records: int, bucket_limit: int = 0):
        """Joins with at least min_records records sort only the records that may share
        their key (0: every join, -1: none); buckets above bucket_limit records (0: the
        default) are kept whole."""
        _check(load_library().mj_ctx_set_member_filter(self.handle, int(min_records),
                                                       int(bucket_limit)))

    def close(self):
        if self.handle:
            load_library().mj_ctx_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


_default_ctx = {}


def default_context(device: Optional[int] = None) -> Context:
    torch = _torch()
    dev = torch.cuda.current_device() if device is None else int(device)
    if dev not in _default_ctx:
        _default_ctx[dev] = Context(dev)
    return _default_ctx[dev]


def pack_2bit(codes) -> np.ndarray:
    """Symbol codes < 4 packed four to a byte, the first in the low bits, as whole
    little-endian 32-bit words (ceil(len / 16) of them): the layout of MJ_PACK_2BIT."""
    c = np.ascontiguousarray(codes, dtype=np.uint8)
    if c.size and int(c.max()) > 3:
        raise ValueError("2-bit packing needs codes < 4")
    n16 = -(-c.size // 16) * 16
    pad = np.zeros(n16, dtype=np.uint8)
    pad[:c.size] = c
    q = pad.reshape(-1, 4)
    b = (q[:, 0] | (q[:, 1] << 2) | (q[:, 2] << 4) | (q[:, 3] << 6)).astype(np.uint8)
    return b.view("<u4").copy() if b.size else np.zeros(0, dtype="<u4")


@dataclass
class DeviceStrings:
    """Strings resident on the GPU: symbol codes (uint8, one per byte, or 2-bit packed) +
    int64 offsets (torch tensors)."""
    chars: "object"
    offsets: "object"
    sigma: int
    packing: int = PACK_U8

    @property
    def n(self) -> int:
        return int(self.offsets.numel()) - 1

    @classmethod
    def from_host(cls, chars, offsets, sigma, device=None, packing=PACK_U8):
        torch = _torch()
        dev = torch.device("cuda", torch.cuda.current_device() if device is None else device)
        if packing == PACK_2BIT:
            words = pack_2bit(chars)
            c = torch.from_numpy(words.view(np.int32) if words.size else np.zeros(1, np.int32))
        else:
            c = torch.from_numpy(np.ascontiguousarray(chars, dtype=np.uint8))
            if c.numel() == 0:
                c = torch.zeros(1, dtype=torch.uint8)
        return cls(c.to(dev), torch.from_numpy(np.ascontiguousarray(offsets, dtype=np.int64)).to(dev),
                   int(sigma), int(packing))

    @classmethod
    def from_packed_host(cls, words, offsets, sigma, device=None):
        """Strings already packed 2 bits per symbol on the host (pack_2bit's layout)."""
        torch = _torch()
        dev = torch.device("cuda", torch.cuda.current_device() if device is None else device)
        w = np.ascontiguousarray(words, dtype="<u4")
        c = torch.from_numpy(w.view(np.int32) if w.size else np.zeros(1, np.int32))
        return cls(c.to(dev), torch.from_numpy(np.ascontiguousarray(offsets, dtype=np.int64)).to(dev),
                   int(sigma), PACK_2BIT)

    def struct(self) -> MjStrings:
        s = MjStrings()
        s.chars = self.chars.data_ptr()
        s.offsets = self.offsets.data_ptr()
        s.n = self.n
        s.sigma = self.sigma
        s.packing = self.packing
        s.reserved = 0
        return s


@dataclass
class Params:
    """Method parameters: q-gram length, K (uniform or per string), T rule, seed."""
    q: int
    k: int = -1
    k_per_string: Optional[object] = None   # torch int32 tensor on the GPU
    t_div: int = 1
    t_fixed: int = 0
    reps: int = 1
    seed: int = 0
    pi_table: Optional[object] = None       # torch uint64/int64 tensor on the GPU
    verifier: int = VERIFY_BATCHED          # or VERIFY_PLAIN
    verify_lanes: int = 0                   # batched: 0 timed; 1/2/4/8 word split; -2 column
                                            # split; -3 band classes (window per pair)

    def struct(self) -> MjParams:
        p = MjParams()
        p.verifier = self.verifier
        p.verify_lanes = self.verify_lanes
        p.q, p.t_div, p.t_fixed, p.reps = self.q, self.t_div, self.t_fixed, self.reps
        p.seed = self.seed
        p.k = self.k if self.k_per_string is None else -1
        p.k_per_string = None if self.k_per_string is None else self.k_per_string.data_ptr()
        p.pi_table = None if self.pi_table is None else self.pi_table.data_ptr()
        return p


def _take_pairs(h) -> np.ndarray:
    L = load_library()
    n = L.mj_pairs_count(h)
    out = np.zeros(max(n, 1), dtype=np.uint64)
    st = L.mj_pairs_copy_to_host(h, out.ctypes.data_as(ctypes.c_void_p), len(out))
    L.mj_pairs_free(h)
    _check(st)
    return out[:n]


def join(strings: DeviceStrings, params: Params, ctx: Optional[Context] = None, stream=None):
    """All pairs i < j with ED <= K sharing a filtered partition (Alg. 3).
    Returns (pairs uint64 array, stats dict)."""
    L = load_library()
    ctx = ctx or default_context()
    s, p, st, h = strings.struct(), params.struct(), MjStats(), ctypes.c_void_p()
    _check(L.mj_join(ctx.handle, ctypes.byref(s), ctypes.byref(p), _stream_ptr(stream),
                     ctypes.byref(h), ctypes.byref(st)))
    return _take_pairs(h), st.as_dict()


def candidates(strings: DeviceStrings, params: Params, ctx: Optional[Context] = None, stream=None):
    """Distinct candidate pairs before verification (Alg. 3 up to the dedup)."""
    L = load_library()
    ctx = ctx or default_context()
    s, p, st, h = strings.struct(), params.struct(), MjStats(), ctypes.c_void_p()
    _check(L.mj_candidates(ctx.handle, ctypes.byref(s), ctypes.byref(p), _stream_ptr(stream),
                           ctypes.byref(h), ctypes.byref(st)))
    return _take_pairs(h), st.as_dict()


RECORD_DTYPE = np.dtype([("key", "<u8"), ("sid", "<i4"), ("pos", "<i4"), ("len", "<i4")])


def partition(strings: DeviceStrings, params: Params, ctx: Optional[Context] = None, stream=None):
    """Partition records of every string and repetition (Alg. 1-2), host structured array
    ordered by (repetition, string, position)."""
    L = load_library()
    ctx = ctx or default_context()
    s, p, h = strings.struct(), params.struct(), ctypes.c_void_p()
    _check(L.mj_partition(ctx.handle, ctypes.byref(s), ctypes.byref(p), _stream_ptr(stream),
                          ctypes.byref(h)))
    n = L.mj_records_count(h)
    cap = max(n, 1)
    key = np.zeros(cap, np.uint64)
    sid = np.zeros(cap, np.int32)
    pos = np.zeros(cap, np.int32)
    ln = np.zeros(cap, np.int32)
    st = L.mj_records_copy_to_host(h, key.ctypes.data, sid.ctypes.data, pos.ctypes.data,
                                   ln.ctypes.data, cap)
    L.mj_records_free(h)
    _check(st)
    out = np.zeros(n, RECORD_DTYPE)
    out["key"], out["sid"], out["pos"], out["len"] = key[:n], sid[:n], pos[:n], ln[:n]
    return out


def verify(strings: DeviceStrings, params: Params, pairs, ctx: Optional[Context] = None,
           stream=None) -> np.ndarray:
    """Banded verification of the given pairs (a << 32 | b): bool array ED <= max(K_a, K_b)."""
    torch = _torch()
    L = load_library()
    ctx = ctx or default_context()
    dev = strings.chars.device
    pt = torch.from_numpy(np.ascontiguousarray(pairs, dtype=np.uint64).view(np.int64)).to(dev)
    n = int(pt.numel())
    flags = torch.zeros(max(n, 1), dtype=torch.uint8, device=dev)
    s, p = strings.struct(), params.struct()
    _check(L.mj_verify(ctx.handle, ctypes.byref(s), ctypes.byref(p),
                       ctypes.c_void_p(pt.data_ptr() if n else 0), n,
                       ctypes.c_void_p(flags.data_ptr()), _stream_ptr(stream)))
    return flags[:n].cpu().numpy().astype(bool)


class Index:
    """Device-resident partition index over a string collection (for search)."""

    def __init__(self, strings: DeviceStrings, params: Params, ctx: Optional[Context] = None,
                 stream=None):
        L = load_library()
        self.ctx = ctx or default_context()
        s, p, h = strings.struct(), params.struct(), ctypes.c_void_p()
        _check(L.mj_index_build(self.ctx.handle, ctypes.byref(s), ctypes.byref(p),
                                _stream_ptr(stream), ctypes.byref(h)))
        self.handle = h
        self.sigma = strings.sigma

    @property
    def records(self) -> int:
        return load_library().mj_index_records(self.handle)

    @property
    def device_bytes(self) -> int:
        return load_library().mj_index_bytes(self.handle)

    def search(self, queries: DeviceStrings, k: int = -1, k_per_query=None, stream=None,
               verifier: int = VERIFY_BATCHED, verify_lanes: int = 0):
        """(query id << 32 | string id) pairs with ED <= K_query; returns (pairs, stats)."""
        L = load_library()
        qp = Params(q=1, k=k, k_per_string=k_per_query, verifier=verifier,
                    verify_lanes=verify_lanes)
        s, p, st, h = queries.struct(), qp.struct(), MjStats(), ctypes.c_void_p()
        _check(L.mj_search(self.ctx.handle, self.handle, ctypes.byref(s), ctypes.byref(p),
                           _stream_ptr(stream), ctypes.byref(h), ctypes.byref(st)))
        return _take_pairs(h), st.as_dict()

    def close(self):
        if self.handle:
            load_library().mj_index_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Continuous-batching search over a resident Index (native worker threads, one HIP
    stream each; admission by a device-memory budget)."""

    def __init__(self, index: Index, workers: int = 4, max_batch: int = 4096,
                 memory_budget: int = 16 << 30):
        L = load_library()
        cfg = MjServerConfig(workers, max_batch, memory_budget)
        h = ctypes.c_void_p()
        _check(L.mj_server_create(index.ctx.device, index.handle, ctypes.byref(cfg), ctypes.byref(h)))
        self.handle = h
        self.index = index  # keep the index alive

    def submit(self, codes, k: int, tag: int):
        codes = np.ascontiguousarray(codes, dtype=np.uint8)
        _check(load_library().mj_server_submit(self.handle, codes.ctypes.data_as(ctypes.c_void_p),
                                               len(codes), int(k), int(tag)))

    def pending(self) -> int:
        return load_library().mj_server_pending(self.handle)

    def poll(self, timeout_ms: int = -1, max_replies: int = 4096, ids_cap: int = 1 << 20):
        """Returns a list of dicts: tag, ids (np.uint32), batch_size, worker, status,
        submit/start/done times in ms, and the batch's admission estimate and measured device
        bytes."""
        L = load_library()
        reps = (MjReply * max_replies)()
        ids = np.zeros(ids_cap, dtype=np.uint32)
        nr, ni = ctypes.c_int32(), ctypes.c_int64()
        _check(L.mj_server_poll(self.handle, reps, max_replies, ids.ctypes.data_as(ctypes.c_void_p),
                                ids_cap, int(timeout_ms), ctypes.byref(nr), ctypes.byref(ni)))
        out = []
        for r in reps[:nr.value]:
            out.append({"tag": r.tag, "status": r.status, "ids": ids[r.offset:r.offset + r.count].copy(),
                        "batch_size": r.batch_size, "worker": r.worker, "submit_ms": r.submit_ms,
                        "start_ms": r.start_ms, "done_ms": r.done_ms,
                        "batch_estimate": r.batch_estimate, "batch_device": r.batch_device})
        return out

    def close(self):
        if self.handle:
            load_library().mj_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def version() -> str:
    return load_library().mj_version().decode()
