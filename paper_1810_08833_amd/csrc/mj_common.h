// Internal declarations shared by the HIP sources of libminjoin (gfx950).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/minjoin.h"

namespace mj {

// ---------------------------------------------------------------- errors
struct Error : std::runtime_error {
    mj_status status;
    Error(mj_status s, const std::string &m) : std::runtime_error(m), status(s) {}
};

#define MJ_HIP(expr)                                                                   \
    do {                                                                               \
        hipError_t e_ = (expr);                                                        \
        if (e_ != hipSuccess)                                                          \
            throw ::mj::Error(MJ_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

#define MJ_LAUNCH_CHECK() MJ_HIP(hipGetLastError())

// ---------------------------------------------------------------- constants
constexpr uint64_t GAMMA = 0x9E3779B97F4A7C15ull;    // salt increment for the q-gram hash
constexpr uint64_t GAMMA_B = 0x632BE59BD9B4E019ull;  // separates the partition-key base
constexpr uint64_t P61 = (1ull << 61) - 1;           // Mersenne prime of the Karp-Rabin key

// SplitMix64 output function: a bijection on 64-bit words (Steele, Lea & Flood 2014).
__host__ __device__ __forceinline__ uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// a * b mod 2^61-1 for a, b < 2^61.
__device__ __forceinline__ uint64_t mulmod61(uint64_t a, uint64_t b) {
    uint64_t lo = a * b;
    uint64_t hi = __umul64hi(a, b);
    uint64_t r = (lo & P61) + ((hi << 3) | (lo >> 61));
    return r >= P61 ? r - P61 : r;
}

inline int symbol_bits(int sigma) {
    int b = 1;
    while ((1 << b) < sigma) b++;
    return b;
}

// ---------------------------------------------------------------- device memory
// Device allocations come from the caller's mj_allocator when the context has one, else
// from hipMalloc (alloc == nullptr).  Entry points install their context's allocator for
// their thread with AllocScope; objects that outlive the call (results, indexes) keep a
// copy of the allocator that made their memory and free with it.
extern thread_local mj_allocator t_dev_alloc;
struct AllocScope {
    mj_allocator prev;
    explicit AllocScope(const mj_allocator &a) : prev(t_dev_alloc) { t_dev_alloc = a; }
    ~AllocScope() { t_dev_alloc = prev; }
};
void *dev_alloc(size_t bytes, const mj_allocator &a);
void dev_free(void *p, const mj_allocator &a);
// From / to the current thread's allocator.
void *dev_alloc(size_t bytes);
void dev_free(void *p);
// Buffers handed to the caller (result pairs): from the caller's allocator when there is
// one, else stream-ordered (hipMallocFromPoolAsync on `s` from a per-device pool that keeps
// up to RESULT_POOL_KEEP bytes of freed blocks), so neither taking nor freeing one waits
// for the device.  result_free orders the free after the work queued on `s`.
constexpr uint64_t RESULT_POOL_KEEP = 1ull << 30;
void *result_alloc(size_t bytes, const mj_allocator &a, hipStream_t s);
void result_free(void *p, const mj_allocator &a, hipStream_t s);

// ---------------------------------------------------------------- workspace
// Grow-only cache of device blocks; blocks handed out during one call are released
// together at its end and reused by the next call.  Blocks come from `alloc` (the
// context's allocator; hipMalloc when its alloc is null).
class Workspace {
  public:
    mj_allocator alloc{};
    ~Workspace();
    void *get(size_t bytes);
    template <class T> T *get_n(size_t n) { return static_cast<T *>(get(n * sizeof(T) + 16)); }
    void release_all();
    size_t bytes_held() const { return held_; }
    // bytes of the blocks the last call used (measured by release_all)
    size_t last_call_bytes() const { return last_used_; }
    // Arena mode: every block comes from the fixed device region [base, base + bytes)
    // (bump allocation, reset by release_all; MJ_ECAPACITY when it is exhausted) and the
    // workspace never allocates or frees device memory.  The region's first
    // ARENA_SCAN_BYTES hold the single-pass scans' state, which must be zero before the
    // first scan (the caller clears it once).
    static constexpr size_t ARENA_SCAN_BYTES = 4096;
    void bind_arena(void *base, size_t bytes);
    bool arena() const { return arena_base_ != nullptr; }
    // Holding: blocks handed out while holding stay reserved across release_all (their
    // addresses are baked into a captured graph) until drop_holds.
    void hold(bool on) { holding_ = on; }
    void drop_holds();
    // Scans launch their multi-pass form (no state kept across calls: a captured graph
    // replays its launch arguments unchanged).
    bool no_lookback = false;
    // State of the single-pass scans (prims.hip), kept across calls: one word per tile
    // tagged with the call's epoch (so it never needs clearing) and a tile ticket counter
    // that only grows (`base` = its value before the next scan).
    struct ScanState {
        uint64_t *state = nullptr;
        unsigned long long *ticket = nullptr;
        uint64_t base = 0;
        uint32_t epoch = 0;
    } scan;

  private:
    struct Block { void *p; size_t n; bool used; bool held; };
    bool holding_ = false;
    std::vector<Block> blocks_;
    size_t held_ = 0, last_used_ = 0;
    uint8_t *arena_base_ = nullptr;
    size_t arena_bytes_ = 0, arena_used_ = 0;
};


// ---------------------------------------------------------------- kernel timers
// HIP events recorded on the launching stream around each launch of a hot kernel;
// summed per slot after the call has synchronised.
struct KTimer {
    enum { ANCHORS = 0, RECORDS = 1, EMIT = 2, VERIFY = 3, SLOTS = 4, POOL = 96 };
    hipEvent_t ev[POOL] = {};
    int used = 0;
    int slot_of[POOL / 2] = {};
    int count_of[POOL / 2] = {};  // launches of the hot kernel inside each bracket
    void create();
    void destroy();
    void reset() { used = 0; }
    // returns a handle for end(); -1 when the pool is exhausted (launch not timed)
    int begin(int slot, hipStream_t s);
    // closes the bracket opened by begin(); `launches` is how many launches of the slot's
    // kernel it holds (the anchor kernel runs once per repetition inside one bracket)
    void end(int h, hipStream_t s, int launches = 1);
    void collect(float *ms, int32_t *launches);  // stream must be synchronised
};

// ---------------------------------------------------------------- primitives (prims.hip)
void fill_u32(uint32_t *p, uint32_t v, int64_t n, hipStream_t s);
void fill_u64(uint64_t *p, uint64_t v, int64_t n, hipStream_t s);
// out[0..n] = exclusive prefix sums of in[0..n), out[n] = total.
void exclusive_scan_u32(const uint32_t *in, uint32_t *out, int64_t n, Workspace &ws, hipStream_t s);
void exclusive_scan_u64(const uint64_t *in, uint64_t *out, int64_t n, Workspace &ws, hipStream_t s);
// The same over the first min(n, *count) elements, count a device value (launch sizes
// from the bound n); the grand total also goes to *total_out.
void exclusive_scan_u64_dev(const uint64_t *in, uint64_t *out, int64_t n, const uint32_t *count,
                            uint64_t *total_out, Workspace &ws, hipStream_t s);
// Indices i (ascending) with flags[i] != 0; returns count (reads it back).
int64_t compact_flags(const uint8_t *flags, int64_t n, int64_t *idx_out, Workspace &ws,
                      hipStream_t s, uint64_t *host_scratch);
// The same without the read-back: returns the device address of the count (n >= 1).
const uint32_t *compact_flags_async(const uint8_t *flags, int64_t n, int64_t *idx_out,
                                    Workspace &ws, hipStream_t s);
// Size of the pinned host buffer each context keeps for small device-to-host reads.
constexpr size_t HOST_SCRATCH_BYTES = 16384;

// Stable sort of keys (and an optional payload) ascending, in place.  key_mask has a 1
// at every bit that may be set in some key (the others must be zero in all keys).
// n_dev (nullable): the element count on the device, n then being its capacity.
// k2 / v2 (nullable): second buffers of n elements (else taken from the workspace).
// sorted_keys (nullable, keys only): receives the buffer that holds the sorted keys (key
// or the second buffer) instead of a copy back into key after an odd number of passes.
void radix_sort(uint64_t *key, uint64_t *val, int64_t n, uint64_t key_mask, Workspace &ws,
                hipStream_t s, const int64_t *n_dev = nullptr, uint64_t *k2 = nullptr,
                uint64_t *v2 = nullptr, uint64_t **sorted_keys = nullptr);
// Records (key, payload) sorted by the full 64-bit key, in place; equal keys keep their
// order only up to the runs that the repair step reorders.
void sort_records(uint64_t *key, uint64_t *val, int64_t n, Workspace &ws, hipStream_t s,
                  uint64_t *host_scratch, const int64_t *n_dev = nullptr);
// Records that may share their key with another record (a superset of every group of
// two or more; see prims.hip): their (key, payload) into mkey / mval, in index order, at
// most mcap of them; *m_dev = their count (on the device; a count above mcap means the
// arrays were too small).  n_dev (nullable): the record count on the device, n then
// being its capacity.  Buckets (records of equal top 16 key bits) of more than `big`
// records are kept whole.
void group_members(const uint64_t *key, const uint64_t *val, int64_t n, const int64_t *n_dev,
                   uint64_t *mkey, uint64_t *mval, int64_t mcap, int64_t *m_dev, uint32_t big,
                   Workspace &ws, hipStream_t s);
// Gather: dst[i] = src[idx[i]] for i < n (or < *n_dev when given).
void gather_u64(const uint64_t *src, const int64_t *idx, uint64_t *dst, int64_t n, hipStream_t s,
                const uint32_t *n_dev = nullptr);

// Read one device value back (synchronises the stream).
template <class T>
T read_back(const T *dev, hipStream_t s, void *pinned) {
    MJ_HIP(hipMemcpyAsync(pinned, dev, sizeof(T), hipMemcpyDeviceToHost, s));
    MJ_HIP(hipStreamSynchronize(s));
    T v;
    memcpy(&v, pinned, sizeof(T));
    return v;
}

// ---------------------------------------------------------------- device views
// A string collection prepared on the device.
struct DevStrings {
    const uint8_t *chars = nullptr;
    int packing = MJ_PACK_U8;  // MJ_PACK_2BIT: four 2-bit symbols per byte, first in the low bits
    const int64_t *offsets = nullptr;
    int32_t n = 0;
    int32_t sigma = 0;
    int32_t bits = 0;        // b = ceil(log2 sigma)
    int64_t total = 0;       // offsets[n]
    int32_t *len = nullptr;  // m_i
    int32_t *kk = nullptr;   // K_i
    int32_t *rr = nullptr;   // r_i (repetition-independent)
    uint32_t *planes = nullptr;  // bit planes, interleaved: planes[w * np + p]
    int64_t plane_words = 0;
    // device word set by the plane packing when a symbol code is >= sigma (nullptr: the
    // symbols were not checked)
    uint32_t *symbol_err = nullptr;
    // strings whose radius exceeds the tile kernel's halo: their ids and radii (device),
    // their number and their q-gram starts in all (host, from the set-up read-back)
    int32_t *wide_ids = nullptr, *wide_r = nullptr;
    int32_t wide_count = 0;
    int64_t wide_pos = 0;
};

inline void check_total(const DevStrings &d) {
    if (d.total < 0) throw Error(MJ_EINVAL, "offsets[n] < 0");
    if (d.total > 0 && !d.chars) throw Error(MJ_EINVAL, "chars is NULL");
}

struct PartitionParams {
    int q, bits, t_div, t_fixed, reps;
    uint64_t seed;
    int64_t k;
    const int32_t *k_per_string;
    const uint64_t *pi_table;
};

// Growable, owned arrays of partition records: key f, payload (sid << 32 | pos), and
// optionally the length.
// Partition records.  With `ws` set the arrays come from that workspace (valid until
// its release); otherwise they are owned allocations freed by release().
struct RecBuf {
    uint64_t *key = nullptr;
    uint64_t *val = nullptr;
    uint32_t *len = nullptr;
    int64_t cap = 0, count = 0;
    bool with_len = false;
    Workspace *ws = nullptr;
    mj_allocator alloc{};  // owned arrays (ws == nullptr): the allocator that made them
    void reserve(int64_t need, hipStream_t s);
    void release();
};

// partition.hip
// What the per-string set-up reads back: the halo radius the anchor kernel needs, a bound
// on the partitions of one repetition (summed over strings), and the largest K.
struct SetupInfo {
    int32_t halo = 0;
    int64_t rec_bound = 0;
    int32_t kmax = 0;
};
int32_t prepare_strings(DevStrings &d, const PartitionParams &p, Workspace &ws, hipStream_t s,
                        uint64_t *host_scratch, SetupInfo *info = nullptr);  // returns the halo
// The same in two halves: the launches and the copies to host_dst (pinned, 5 words), and,
// once the stream has synchronised, the checks and results.
void prepare_launch(DevStrings &d, const PartitionParams &p, Workspace &ws, hipStream_t s,
                    uint64_t *host_dst);
int32_t prepare_finish(DevStrings &d, const uint64_t *host_src, SetupInfo *info);
// Builds the verifier's bit planes and checks every symbol against sigma (the result in
// d.symbol_err, read with the partition stage's counts or by check_symbols).
void pack_planes(DevStrings &d, int planes, Workspace &ws, hipStream_t s,
                 uint32_t *dest = nullptr);  // dest: plane_words_for(total) * planes words
// Plane words per plane for `total` symbols (with padding: verifier windows read past the
// end).
inline int64_t plane_words_for(int64_t total) { return (total + 31) / 32 + 96; }
// Reads d.symbol_err back (synchronises); MJ_EINVAL when a symbol code is >= sigma.
void check_symbols(const DevStrings &d, hipStream_t s, uint64_t *host_scratch);
// Appends the records of every partition of every repetition (repetition rho seeds Pi
// with seed + rho) to `out`; returns how many.
int64_t partition_records(const DevStrings &d, const PartitionParams &p, int32_t halo, RecBuf &out,
                          Workspace &ws, hipStream_t s, uint64_t *host_scratch,
                          KTimer *kt = nullptr);

// The same with every size after the set-up on the device: the records of all
// repetitions go to key/val (room for reps * si.rec_bound), their count to *R_dev; no
// host read.  Returns the record capacity used (reps * si.rec_bound).
int64_t partition_records_streamed(const DevStrings &d, const PartitionParams &p, const SetupInfo &si,
                                   uint64_t *key, uint64_t *val, int64_t *R_dev, Workspace &ws,
                                   hipStream_t s, KTimer *kt = nullptr);

// join.hip
// Groups of at least EMIT_TILE records have their pair tests taken by tile pairs (64 x 64
// records, one wave each) in a join with at least EMIT_SPLIT_UNITS such tile pairs (a
// context setting); the smaller groups test by test.  With fewer tile pairs the two tile
// passes sit at their latency floor (about 75 us each) and the smaller groups gain little
// (measured: text, 9.5e3 tile pairs, loses 0.05 ms; protein, about 1e5, gains 0.4 ms).
constexpr int EMIT_TILE = 64;
constexpr int64_t EMIT_SPLIT_UNITS = (int64_t)1 << 15;
struct GroupInfo {
    int64_t groups = 0;          // -1: on the device (slot)
    uint64_t tests = 0;          // pair tests of all groups
    uint64_t small_tests = 0;    // of the groups below EMIT_TILE records
    uint64_t units = 0;          // tile pairs of the groups of EMIT_TILE or more
    int64_t *gstart = nullptr;   // group start index in the sorted records
    int64_t *gend = nullptr;     // group end index (inclusive)
    uint64_t *tstart = nullptr;  // exclusive prefix of pair tests, all groups
    uint64_t *tsmall = nullptr;  // exclusive prefix of pair tests, 0 for the large groups
    uint64_t *ustart = nullptr;  // exclusive prefix of tile pairs, 0 for the small groups
    // streamed: [0] c1 | c2 << 32, [1] groups, [2] tests, [3] small tests, [4] tile pairs
    uint64_t *slot = nullptr;
    int64_t gmax = 0;            // streamed: capacity of the group arrays
};
// Speed-only choices of the emission kernels (see emit_candidates): gather (m, K) by string
// id at each use (lazy), one packed (m, K) word per string, the large groups by tile pairs
// (split), tests per thread, workgroups of the test-by-test kernel and of the tile-pair
// kernel.
struct EmitHints {
    bool lazy = true;
    bool string_words = false;
    bool split = false;
    int chunk = 16;
    int64_t blocks = 4096;
    int64_t tile_blocks = 1024;
};
// tile_min: the context's threshold (tile pairs; -1: never by tile pairs)
EmitHints emit_hints(uint64_t tests, uint64_t small_tests, uint64_t units, int64_t R, int32_t n,
                     int64_t tile_min);
GroupInfo find_groups(const uint64_t *key, int64_t R, Workspace &ws, hipStream_t s,
                      uint64_t *host_scratch);
// The same with the record count on the device (*R_dev <= R_cap); no host read.
GroupInfo find_groups_streamed(const uint64_t *key, int64_t R_cap, const int64_t *R_dev,
                               Workspace &ws, hipStream_t s);
void emit_candidates_streamed(const uint64_t *val, int64_t R_cap, const int64_t *R_dev,
                              const GroupInfo &g, const DevStrings &d, uint64_t *out, int64_t cap,
                              unsigned long long *count, const EmitHints &h, Workspace &ws,
                              hipStream_t s, KTimer *kt = nullptr);
const uint32_t *dedup_pairs_streamed(uint64_t *pairs, int64_t cap, const unsigned long long *count,
                                     int32_t n_first, int32_t n_second, Workspace &ws, hipStream_t s,
                                     uint64_t **result);
// Emit candidate pair keys for all pair tests; returns count emitted (<= cap).
// Tests [t_begin, t_end) only when t_end > 0 (a join emitted in passes).
// tile_min as for emit_hints.
int64_t emit_candidates(const uint64_t *val, int64_t R, const GroupInfo &g, const DevStrings &d,
                        uint64_t *out, int64_t cap, Workspace &ws, hipStream_t s,
                        uint64_t *host_scratch, int64_t tile_min, KTimer *kt = nullptr,
                        uint64_t t_begin = 0, uint64_t t_end = 0);
// Sorted unique copy of pairs (first << 32 | second, first < n_first, second <
// n_second) in *result (owned allocation); sorts `pairs` in place; returns the count.
// The distinct pairs in *result: a workspace block when to_ws, else a result buffer
// (result_alloc with the thread's allocator on s) that the caller owns.
int64_t dedup_pairs(uint64_t *pairs, int64_t n, int32_t n_first, int32_t n_second, Workspace &ws,
                    hipStream_t s, uint64_t *host_scratch, uint64_t **result, bool to_ws);
// Search: probe sorted index keys with sorted query records.
int64_t probe_candidates(const uint64_t *qkey, const uint64_t *qval, int64_t RQ,
                         const uint64_t *ikey, const uint64_t *ival, int64_t RI,
                         const DevStrings &qd, const DevStrings &id, uint64_t *out,
                         int64_t cap, uint64_t *tests_out, Workspace &ws, hipStream_t s,
                         uint64_t *host_scratch);

// verify.hip
// flags[i] = ED(A[a], B[b]) <= K for pairs[i] = a << 32 | b; K = max(K_a, K_b) when
// kmode == 0, else K_a.  uniform_k >= 0 promises that every pair's K equals it and that
// all ids are valid (pairs produced by the library): then no binning pass is needed.
// Returns band cells processed (device counter read back).
int64_t verify_pairs(const uint64_t *pairs, int64_t n, const DevStrings &A, const DevStrings &B,
                     int kmode, uint8_t *flags, Workspace &ws, hipStream_t s,
                     uint64_t *host_scratch, KTimer *kt = nullptr, int64_t uniform_k = -1);
int verify_planes(int bits);   // planes the verifier needs for b bits per symbol

// verify_lg.hip: one persistent launch for all pairs (lane groups, longest first).
// The lane-group width is timed once per (ceil(Kmax/32), planes) and kept in `tune`.
// VerifyTuning::last_g value of the kernel that splits each pair's text columns over two
// lanes (forward and reversed halves), and of the launch that sizes each pair's window by
// its band class
constexpr int VERIFY_BIDIR = 3;
constexpr int VERIFY_CLASSES = 5;
struct VerifyTuning {
    int best_g[64][4] = {};
    int best_blocks[64][4] = {};
    int last_g = 0, last_nwl = 0, last_blocks = 0;
};
// uniform_k >= 0 promises that every pair's K equals it and that all ids are valid (pairs
// produced by the library): the pass that finds the largest K is skipped.  With
// cells_defer set (two words of pinned host memory) the band-cell count and an error word
// (nonzero when some pair's band did not fit the launched window) are copied there
// asynchronously and the call returns 0 without synchronising; otherwise the call reads
// both and fails with MJ_ECAPACITY on the error word.  force_lanes != 0 fixes
// the configuration (mj_params.verify_lanes) instead of the timed choice; tune == nullptr
// takes the fixed small-call configuration (no timing runs on the call).
int64_t verify_pairs_batched(const uint64_t *pairs, int64_t n, const DevStrings &A,
                             const DevStrings &B, int kmode, uint8_t *flags, Workspace &ws,
                             hipStream_t s, uint64_t *host_scratch, KTimer *kt,
                             VerifyTuning *tune, int64_t uniform_k = -1,
                             uint64_t *cells_defer = nullptr, int force_lanes = 0);
int persist_max_c();
int verify_small_call_lanes(int cmax);
void verify_pairs_batched_streamed(const uint64_t *pairs, int64_t cap, const uint32_t *n_dev,
                                   const DevStrings &A, const DevStrings &B, int kmode, int cmax,
                                   uint8_t *flags, Workspace &ws, hipStream_t s, KTimer *kt,
                                   const VerifyTuning &tune, int force_lanes,
                                   unsigned long long **cells_out);

}  // namespace mj
