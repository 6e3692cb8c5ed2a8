// Banded verification of caller-given pairs without any device allocation, for callers
// that cannot allocate (code under HIP graph capture, tight serving loops, harnesses
// that forbid hipMalloc).  Every scratch buffer of the call -- per-string parameters,
// bit planes, the verifier's queue counters, length bins and longest-first order, the
// scan state -- comes from one fixed array in device memory, `scratch`, which each GPU
// the library runs on holds until the process ends.
#include <string.h>

#include <mutex>

#include "capi_internal.h"

using namespace mj;

// 64 MiB per device: enough for, e.g., 10^6 strings of 50 M DNA symbols in all and 10^6
// pairs (planes 2 bits per symbol, 12 bytes per string, 8 bytes per pair, ~70 KB fixed).
constexpr size_t NOALLOC_SCRATCH_BYTES = (size_t)64 << 20;
static __device__ __align__(256) uint8_t scratch[NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int MAX_DEVICES = 64;

// Per device: the device address of its copy of `scratch` (taken once with
// hipGetSymbolAddress, with that device current; the array's name is not a device
// address in host code), the workspace bound to it, and host words for read-backs.
struct NoAllocDevice {
    std::mutex mu;  // serialises the calls on this device: they share the array
    bool ready = false;
    uint8_t *ptr = nullptr;
    Workspace ws;
    uint64_t host_words[HOST_SCRATCH_BYTES / 8];
};

NoAllocDevice g_dev[MAX_DEVICES];

}  // namespace

extern "C" mj_status mj_verify_noalloc(const mj_strings *strings, const mj_params *params,
                                       const uint64_t *pairs, int64_t n, uint8_t *flags,
                                       void *stream) {
    if (n < 0 || (n > 0 && (!pairs || !flags))) return mj_fail(MJ_EINVAL, "bad pair list");
    if (!strings || !params) return mj_fail(MJ_EINVAL, "strings/params is NULL");
    try {
        int device = 0;
        MJ_HIP(hipGetDevice(&device));
        if (device < 0 || device >= MAX_DEVICES) return mj_fail(MJ_EINVAL, "device index too large");
        NoAllocDevice &nd = g_dev[device];
        std::lock_guard<std::mutex> lk(nd.mu);
        hipStream_t s = (hipStream_t)stream;
        if (!nd.ready) {
            void *p = nullptr;
            const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
            if (e != hipSuccess || !p)
                return mj_fail(MJ_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") +
                                               hipGetErrorString(e));
            nd.ptr = static_cast<uint8_t *>(p);
            nd.ws.bind_arena(nd.ptr, NOALLOC_SCRATCH_BYTES);
            // the single-pass scans' state starts at zero (a fill kernel: no memset node)
            fill_u64(reinterpret_cast<uint64_t *>(nd.ptr), 0, Workspace::ARENA_SCAN_BYTES / 8, s);
            nd.ready = true;
        }
        if (strings->n < 0 || (strings->n > 0 && !strings->offsets))
            throw Error(MJ_EINVAL, "bad strings");
        if (strings->sigma < 2 || strings->sigma > 256) throw Error(MJ_EINVAL, "sigma must be in 2..256");
        if (strings->packing != MJ_PACK_U8 && strings->packing != MJ_PACK_2BIT)
            throw Error(MJ_EINVAL, "packing must be MJ_PACK_U8 or MJ_PACK_2BIT");
        if (strings->packing == MJ_PACK_2BIT && (strings->sigma > 4 || ((uintptr_t)strings->chars & 3)))
            throw Error(MJ_EINVAL, "2-bit packing needs sigma <= 4 and 4-byte aligned words");
        if (params->k > 2047) throw Error(MJ_ECAPACITY, "threshold K exceeds the verifier's band limit (K <= 2047)");
        if (params->k < -1 || (params->k == -1 && !params->k_per_string))
            throw Error(MJ_EINVAL, "bad threshold");
        if (params->verifier != MJ_VERIFY_BATCHED)
            throw Error(MJ_EINVAL, "the allocation-free verification uses the batched verifier");
        if (params->verify_lanes != 0 && params->verify_lanes != 1 && params->verify_lanes != 2 &&
            params->verify_lanes != 4 && params->verify_lanes != 8 && params->verify_lanes != -2)
            throw Error(MJ_EINVAL, "verify_lanes must be 0, 1, 2, 4, 8 or -2");
        Workspace &ws = nd.ws;
        struct Release { Workspace &w; ~Release() { w.release_all(); } } rel{ws};
        DevStrings d;
        d.chars = static_cast<const uint8_t *>(strings->chars);
        d.packing = strings->packing;
        d.offsets = strings->offsets;
        d.n = strings->n;
        d.sigma = strings->sigma;
        d.bits = symbol_bits(strings->sigma);
        d.total = d.n > 0 ? -1 : 0;  // read back with the per-string set-up
        PartitionParams pp{};
        pp.q = 1;
        pp.bits = d.bits;
        pp.t_div = 1;
        pp.reps = 1;
        pp.k = params->k;
        pp.k_per_string = params->k_per_string;
        (void)prepare_strings(d, pp, ws, s, nd.host_words);
        pack_planes(d, verify_planes(d.bits), ws, s);
        check_symbols(d, s, nd.host_words);
        // no tuning table: the fixed configuration, no timing runs (no events created)
        verify_pairs_batched(pairs, n, d, d, 0, flags, ws, s, nd.host_words, nullptr, nullptr, -1,
                             nullptr, params->verify_lanes);
        MJ_HIP(hipStreamSynchronize(s));
        return MJ_OK;
    } catch (const Error &e) {
        return mj_fail(e.status, e.what());
    } catch (const std::exception &e) {
        return mj_fail(MJ_EDEVICE, e.what());
    } catch (...) {
        return mj_fail(MJ_EDEVICE, "unknown error");
    }
}
