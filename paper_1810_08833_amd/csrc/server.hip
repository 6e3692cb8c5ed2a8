// Continuous-batching search server over a device-resident index.
//
// Worker threads each own a HIP stream and a context (workspace).  A free worker admits
// every queued request that fits: at most max_batch queries, and only while the
// estimated device memory of all batches in flight stays within the budget (a request
// waits for memory to free up; a worker with nothing in flight always takes at least one
// request).  The batch is uploaded, searched (mj_search) and split back into per-request
// replies.  Batches of different workers run concurrently on their own streams.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <thread>
#include <vector>

#include "capi_internal.h"

namespace {

struct Request {
    uint64_t tag;
    std::vector<uint8_t> codes;
    int32_t k;
    double submit_ms;
    int64_t est;
};

struct Done {
    mj_reply reply;
    std::vector<uint32_t> ids;
};

// Admission estimate: BATCH_BYTES for a batch plus request_bytes for each of its queries.
// Measured (one worker's search workspace and query buffers, 1M-string DNA index): 1.6-2.9
// MB per batch plus 18-39 bytes per query symbol, within 4.8 MB of that line.
constexpr int64_t BATCH_BYTES = 8 << 20;
int64_t request_bytes(int64_t len) { return 96 * len + 4096; }

}  // namespace

struct mj_server {
    int device = 0;
    const mj_index *ix = nullptr;
    mj_server_config cfg{};
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Request> queue;
    std::deque<Done> done;
    int64_t inflight_bytes = 0;
    int64_t pending = 0;
    bool stop = false;
    std::vector<std::thread> threads;
    std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();

    double now_ms() const {
        return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    }
    bool can_admit() const {
        return !queue.empty() &&
               (inflight_bytes == 0 || inflight_bytes + BATCH_BYTES + queue.front().est <= cfg.memory_budget);
    }
    void worker(int w);
};

void mj_server::worker(int w) {
    if (hipSetDevice(device) != hipSuccess) return;
    hipStream_t st = nullptr;
    mj_ctx *ctx = nullptr;
    if (hipStreamCreate(&st) != hipSuccess) return;
    if (mj_ctx_create(device, nullptr, &ctx) != MJ_OK) {
        (void)hipStreamDestroy(st);
        return;
    }
    ctx->no_tuning = true;  // a timing pass inside a request would set the tail latency
    uint8_t *hchars = nullptr, *dchars = nullptr;
    int64_t *hoff = nullptr, *doff = nullptr;
    int32_t *hk = nullptr, *dk = nullptr;
    int64_t cap_chars = 0, cap_n = 0;
    for (;;) {
        std::vector<Request> batch;
        int64_t bytes = BATCH_BYTES;
        {
            std::unique_lock<std::mutex> lk(mu);
            cv_work.wait(lk, [&] { return stop || can_admit(); });
            if (stop) break;
            while (!queue.empty() && (int32_t)batch.size() < cfg.max_batch) {
                int64_t est = queue.front().est;
                bool alone = batch.empty() && inflight_bytes == 0;
                if (!alone && inflight_bytes + bytes + est > cfg.memory_budget) break;
                batch.push_back(std::move(queue.front()));
                queue.pop_front();
                bytes += est;
            }
            inflight_bytes += bytes;
        }
        if (batch.empty()) {
            std::lock_guard<std::mutex> lk(mu);
            inflight_bytes -= bytes;
            continue;
        }
        const double start = now_ms();
        const int32_t n = (int32_t)batch.size();
        int64_t total = 0;
        for (auto &r : batch) total += (int64_t)r.codes.size();
        mj_status status = MJ_OK;
        std::vector<uint64_t> pairs;
        int64_t used = 0;
        // host staging and device buffers grow to the largest batch seen
        if (total + 16 > cap_chars || n + 1 > cap_n) {
            int64_t nc = std::max<int64_t>(total + 16, cap_chars), nn = std::max<int64_t>(n + 1, cap_n);
            if (hchars) (void)hipHostFree(hchars);
            if (hoff) (void)hipHostFree(hoff);
            if (hk) (void)hipHostFree(hk);
            if (dchars) (void)hipFree(dchars);
            if (doff) (void)hipFree(doff);
            if (dk) (void)hipFree(dk);
            hchars = nullptr; hoff = nullptr; hk = nullptr; dchars = nullptr; doff = nullptr; dk = nullptr;
            cap_chars = cap_n = 0;
            if (hipHostMalloc((void **)&hchars, nc, hipHostMallocDefault) == hipSuccess &&
                hipHostMalloc((void **)&hoff, nn * 8, hipHostMallocDefault) == hipSuccess &&
                hipHostMalloc((void **)&hk, nn * 4, hipHostMallocDefault) == hipSuccess &&
                hipMalloc((void **)&dchars, nc) == hipSuccess && hipMalloc((void **)&doff, nn * 8) == hipSuccess &&
                hipMalloc((void **)&dk, nn * 4) == hipSuccess) {
                cap_chars = nc;
                cap_n = nn;
            } else {
                (void)hipGetLastError();
                status = MJ_ENOMEM;
            }
        }
        if (status == MJ_OK) {
            int64_t o = 0;
            for (int32_t i = 0; i < n; i++) {
                hoff[i] = o;
                if (!batch[i].codes.empty()) memcpy(hchars + o, batch[i].codes.data(), batch[i].codes.size());
                o += (int64_t)batch[i].codes.size();
                hk[i] = batch[i].k;
            }
            hoff[n] = o;
            if (hipMemcpyAsync(dchars, hchars, (size_t)std::max<int64_t>(total, 1), hipMemcpyHostToDevice, st) != hipSuccess ||
                hipMemcpyAsync(doff, hoff, (size_t)(n + 1) * 8, hipMemcpyHostToDevice, st) != hipSuccess ||
                hipMemcpyAsync(dk, hk, (size_t)n * 4, hipMemcpyHostToDevice, st) != hipSuccess) {
                (void)hipGetLastError();
                status = MJ_EDEVICE;
            }
        }
        if (status == MJ_OK) {
            mj_strings qs{dchars, doff, n, ix->sigma, MJ_PACK_U8, 0};
            mj_params qp{};
            qp.q = ix->pp.q;
            qp.k = -1;
            qp.k_per_string = dk;
            qp.verifier = MJ_VERIFY_BATCHED;
            mj_pairs *res = nullptr;
            status = mj_search(ctx, ix, &qs, &qp, (void *)st, &res, nullptr);
            used = (int64_t)ctx->ws.last_call_bytes() + total + (int64_t)(n + 1) * 12 +
                   (res ? (int64_t)res->n * 8 : 0);
            if (status == MJ_OK) {
                pairs.resize((size_t)mj_pairs_count(res));
                status = mj_pairs_copy_to_host(res, pairs.data(), (int64_t)pairs.size());
                mj_pairs_free(res);
            }
        }
        const double end = now_ms();
        std::vector<Done> out((size_t)n);
        for (int32_t i = 0; i < n; i++) {
            mj_reply &r = out[i].reply;
            r.tag = batch[i].tag;
            r.status = status;
            r.count = 0;
            r.offset = 0;
            r.batch_size = n;
            r.worker = w;
            r.submit_ms = batch[i].submit_ms;
            r.start_ms = start;
            r.done_ms = end;
            r.batch_estimate = bytes;
            r.batch_device = used;
        }
        if (status == MJ_OK)
            for (uint64_t p : pairs) out[(size_t)(p >> 32)].ids.push_back((uint32_t)p);  // pairs are sorted
        {
            std::lock_guard<std::mutex> lk(mu);
            for (auto &d : out) done.push_back(std::move(d));
            inflight_bytes -= bytes;
        }
        cv_done.notify_all();
        cv_work.notify_all();
    }
    if (hchars) (void)hipHostFree(hchars);
    if (hoff) (void)hipHostFree(hoff);
    if (hk) (void)hipHostFree(hk);
    if (dchars) (void)hipFree(dchars);
    if (doff) (void)hipFree(doff);
    if (dk) (void)hipFree(dk);
    (void)hipStreamSynchronize(st);
    mj_ctx_destroy(ctx);
    (void)hipStreamDestroy(st);
}

extern "C" mj_status mj_server_create(int device, const mj_index *index, const mj_server_config *cfg,
                                      mj_server **out) {
    if (!index || !cfg || !out) return mj_fail(MJ_EINVAL, "index/cfg/out is NULL");
    if (cfg->workers < 1 || cfg->workers > 16) return mj_fail(MJ_EINVAL, "workers must be 1..16");
    if (cfg->max_batch < 1 || cfg->max_batch > 65536) return mj_fail(MJ_EINVAL, "max_batch must be 1..65536");
    if (cfg->memory_budget <= 0) return mj_fail(MJ_EINVAL, "memory_budget must be > 0");
    if (device != index->device) return mj_fail(MJ_EINVAL, "server device differs from the index device");
    try {
        mj_server *s = new mj_server();
        s->device = device;
        s->ix = index;
        s->cfg = *cfg;
        for (int w = 0; w < cfg->workers; w++) s->threads.emplace_back([s, w] { s->worker(w); });
        *out = s;
        return MJ_OK;
    } catch (const std::exception &e) {
        return mj_fail(MJ_EDEVICE, e.what());
    }
}

extern "C" mj_status mj_server_submit(mj_server *srv, const uint8_t *codes, int32_t len, int32_t k,
                                      uint64_t tag) {
    if (!srv) return mj_fail(MJ_EINVAL, "server is NULL");
    if (len < 0 || (len > 0 && !codes)) return mj_fail(MJ_EINVAL, "bad query");
    if (k < 0 || k > 2047) return mj_fail(MJ_EINVAL, "k must be in 0..2047");
    for (int32_t i = 0; i < len; i++)
        if ((int32_t)codes[i] >= srv->ix->sigma)
            return mj_fail(MJ_EINVAL, "query symbol code is not below the index alphabet");
    int64_t est = request_bytes(len);
    if (BATCH_BYTES + est > srv->cfg.memory_budget)
        return mj_fail(MJ_EINVAL, "query exceeds the memory budget");
    Request r;
    r.tag = tag;
    r.codes.assign(codes, codes + len);
    r.k = k;
    r.est = est;
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        r.submit_ms = srv->now_ms();
        srv->queue.push_back(std::move(r));
        srv->pending++;
    }
    srv->cv_work.notify_one();
    return MJ_OK;
}

extern "C" mj_status mj_server_poll(mj_server *srv, mj_reply *replies, int32_t max_replies,
                                    uint32_t *ids, int64_t ids_cap, int32_t timeout_ms,
                                    int32_t *n_replies, int64_t *n_ids) {
    if (!srv || !n_replies || !n_ids || max_replies < 0 || (max_replies > 0 && !replies) || ids_cap < 0)
        return mj_fail(MJ_EINVAL, "bad poll arguments");
    *n_replies = 0;
    *n_ids = 0;
    std::unique_lock<std::mutex> lk(srv->mu);
    auto ready = [&] { return !srv->done.empty() || srv->pending == 0; };
    if (timeout_ms < 0)
        srv->cv_done.wait(lk, ready);
    else if (timeout_ms > 0)
        srv->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), ready);
    int32_t nr = 0;
    int64_t ni = 0;
    while (nr < max_replies && !srv->done.empty()) {
        Done &d = srv->done.front();
        int64_t c = (int64_t)d.ids.size();
        if (ni + c > ids_cap) {
            if (nr == 0) return mj_fail(MJ_EINVAL, "ids_cap too small for the next reply");
            break;
        }
        if (c) memcpy(ids + ni, d.ids.data(), (size_t)c * 4);
        replies[nr] = d.reply;
        replies[nr].offset = ni;
        replies[nr].count = (int32_t)c;
        ni += c;
        nr++;
        srv->done.pop_front();
        srv->pending--;
    }
    *n_replies = nr;
    *n_ids = ni;
    return MJ_OK;
}

extern "C" int64_t mj_server_pending(const mj_server *srv) {
    if (!srv) return 0;
    std::lock_guard<std::mutex> lk(const_cast<mj_server *>(srv)->mu);
    return srv->pending;
}

extern "C" void mj_server_destroy(mj_server *srv) {
    if (!srv) return;
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        srv->stop = true;
        srv->pending -= (int64_t)srv->queue.size();
        srv->queue.clear();
    }
    srv->cv_work.notify_all();
    for (auto &t : srv->threads) t.join();
    delete srv;
}
