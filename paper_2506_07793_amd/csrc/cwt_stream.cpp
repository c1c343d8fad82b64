// Streaming server of libcwt: sessions, HBM-budget admission, hop batching,
// latency stamps.
//
// Sessions push host samples; every completed hop becomes a pending job.  A
// worker thread forms batches of hops that share a (plan, C, hop) class (at
// most one hop per session per batch, so that each window sees exactly the
// samples up to its own hop), launches them on the server's stream and
// delivers the band-power results with their completion time stamps.
#include <hip/hip_runtime.h>
#include <time.h>

#include <algorithm>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_set>
#include <vector>

#include "../../include/cwt.h"
#include "cwt_internal.hpp"
#include "cwt_kernels.hpp"

using namespace cwtk;
using namespace cwtrt;

extern "C" uint64_t cwt_now_ns(void)
{
    struct timespec ts;
    clock_gettime(CLOCK_MONOTONIC, &ts);
    return (uint64_t)ts.tv_sec * 1000000000ull + (uint64_t)ts.tv_nsec;
}

namespace {

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

// Batch workspace of one (plan, C, hop) class.
struct StreamClass {
    const cwt_plan *plan = nullptr;
    int C = 0, hop = 0, W = 0, Lh = 0, nb = 0, ng = 0, max_batch = 0;  // ng: frequencies in bands
    float *d_slab = nullptr;
    StreamJob *d_jobs = nullptr;
    float *d_xb = nullptr;
    float2 *d_Xh = nullptr;
    float *d_out = nullptr;
    float *d_part = nullptr;  // [rows][ng] per-frequency sums over the hop
    float *h_slab = nullptr;
    StreamJob *h_jobs = nullptr;
    float *h_out = nullptr;
    size_t dev_bytes = 0;
    int n_sessions = 0;
};

size_t class_dev_bytes(int max_batch, int C, int hop, int W, int Lh, int nb, int ng)
{
    const size_t mb = (size_t)max_batch, c = (size_t)C;
    return align256(mb * c * hop * 4) + align256(mb * sizeof(StreamJob)) +
           align256(mb * c * W * 4) + align256(mb * c * Lh * 8) + align256(mb * c * nb * 4) +
           align256(mb * c * ng * 4);
}

struct PendingHop {
    cwt_session *s;
    uint64_t t_push;
    uint64_t t_enq;
    uint64_t hop_idx;
    bool emit;
    std::vector<float> data;  // [C][hop]
};

struct Result {
    std::vector<float> bp;
    uint64_t hop_idx, t_push, t_done;
};

}  // namespace

struct cwt_session {
    cwt_server *srv = nullptr;
    const cwt_plan *plan = nullptr;
    StreamClass *cls = nullptr;
    int C = 0, W = 0, hop = 0, nb = 0;
    float *d_ring = nullptr;
    size_t ring_bytes = 0;
    int ring_pos = 0;          // worker-side: ring slot of the next hop's first sample
    uint64_t samples_in = 0;   // push-side: samples accepted
    std::vector<float> acc;    // push-side: partial hop [C][hop]
    int acc_fill = 0;
    uint64_t next_hop_idx = 0;
    int queued = 0;            // hops not yet completed (pending or in flight)
    std::deque<Result> results;
};

struct cwt_server {
    size_t budget = 0, used = 0;
    cwt_server_opts opts{};
    int device = 0;
    hipStream_t stream = nullptr;
    hipEvent_t ev = nullptr;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<PendingHop> pending;
    std::vector<cwt_session *> sessions;
    std::vector<std::unique_ptr<StreamClass>> classes;
    std::thread worker;
    bool stop = false;
    int in_flight = 0;
    int error = CWT_OK;
    std::string error_msg;
    cwt_server_stats stats{};
};

namespace {

void free_class(StreamClass &k)
{
    void *dptr[] = {k.d_slab, k.d_jobs, k.d_xb, k.d_Xh, k.d_out, k.d_part};
    for (void *p : dptr)
        if (p) (void)hipFree(p);
    void *hptr[] = {k.h_slab, k.h_jobs, k.h_out};
    for (void *p : hptr)
        if (p) (void)hipHostFree(p);
    k = StreamClass{};
}

int alloc_class(StreamClass &k)
{
    const size_t mb = (size_t)k.max_batch, c = (size_t)k.C;
    struct {
        void **p;
        size_t n;
    } dev[] = {{(void **)&k.d_slab, mb * c * k.hop * 4},
               {(void **)&k.d_jobs, mb * sizeof(StreamJob)},
               {(void **)&k.d_xb, mb * c * k.W * 4},
               {(void **)&k.d_Xh, mb * c * k.Lh * 8},
               {(void **)&k.d_out, mb * c * k.nb * 4},
               {(void **)&k.d_part, mb * c * k.ng * 4}};
    for (auto &d : dev) {
        if (hipMalloc(d.p, std::max<size_t>(d.n, 256)) != hipSuccess) {
            *d.p = nullptr;
            return fail(CWT_E_NOMEM, "stream workspace allocation of %zu bytes failed", d.n);
        }
    }
    struct {
        void **p;
        size_t n;
    } host[] = {{(void **)&k.h_slab, mb * c * k.hop * 4},
                {(void **)&k.h_jobs, mb * sizeof(StreamJob)},
                {(void **)&k.h_out, mb * c * k.nb * 4}};
    for (auto &h : host) {
        if (hipHostMalloc(h.p, std::max<size_t>(h.n, 256), hipHostMallocDefault) != hipSuccess) {
            *h.p = nullptr;
            return fail(CWT_E_NOMEM, "pinned staging allocation of %zu bytes failed", h.n);
        }
    }
    return CWT_OK;
}

// Enqueue one batch and wait for it.  Runs on the worker thread without the
// server lock; touches only batch-local data, the class buffers and the
// sessions' ring positions (which only the worker uses).
int run_batch(cwt_server *srv, StreamClass &k, std::vector<PendingHop> &batch,
              std::vector<std::pair<cwt_session *, Result>> &done)
{
    const int n = (int)batch.size();
    const int C = k.C, hop = k.hop, W = k.W, nb = k.nb;
    int n_emit = 0;
    for (int j = 0; j < n; ++j) {
        PendingHop &h = batch[j];
        std::memcpy(k.h_slab + (size_t)j * C * hop, h.data.data(), (size_t)C * hop * 4);
        StreamJob &jb = k.h_jobs[j];
        jb.ring = h.s->d_ring;
        jb.pos = h.s->ring_pos;
        jb.slab_off = j * C * hop;
        jb.emit_row = h.emit ? n_emit++ : -1;
        jb.pad_ = 0;
        h.s->ring_pos = (h.s->ring_pos + hop) % W;
    }
    hipStream_t s = srv->stream;
    hipError_t e;
    if ((e = hipMemcpyAsync(k.d_jobs, k.h_jobs, (size_t)n * sizeof(StreamJob),
                            hipMemcpyHostToDevice, s)) != hipSuccess)
        return hip_fail(e, "stream jobs copy");
    if ((e = hipMemcpyAsync(k.d_slab, k.h_slab, (size_t)n * C * hop * 4, hipMemcpyHostToDevice,
                            s)) != hipSuccess)
        return hip_fail(e, "stream samples copy");
    StreamParams sp{};
    sp.jobs = k.d_jobs;
    sp.n_jobs = n;
    sp.slab = k.d_slab;
    sp.xb = k.d_xb;
    sp.C = C;
    sp.W = W;
    sp.hop = hop;
    if ((e = launch_stream_append(sp, s)) != hipSuccess) return hip_fail(e, "ring append");
    if (n_emit > 0) {
        if ((e = launch_stream_gather(sp, s)) != hipSuccess) return hip_fail(e, "window gather");
        const cwt_plan &P = *k.plan;
        int rc = enqueue_forward(P, k.d_xb, (int64_t)n_emit * C, W, k.d_Xh, s);
        if (rc != CWT_OK) return rc;
        StreamBPParams bp{};
        bp.Xh = k.d_Xh;
        bp.Lh = k.Lh;
        bp.L = P.L;
        bp.W = W;
        bp.hop = hop;
        bp.rows = n_emit * C;
        bp.H = P.d_H;
        bp.band = P.d_band;
        bp.tw = P.d_tw;
        bp.grp_freq = P.d_grp_freq;
        bp.grp_off = P.d_grp_off;
        bp.n_bands = nb;
        bp.n_grouped = k.ng;
        bp.part = k.d_part;
        bp.out = k.d_out;
        if ((e = launch_stream_bandpower(bp, P.max_bins, s)) != hipSuccess)
            return hip_fail(e, "band power launch");
        if ((e = hipMemcpyAsync(k.h_out, k.d_out, (size_t)n_emit * C * nb * 4,
                                hipMemcpyDeviceToHost, s)) != hipSuccess)
            return hip_fail(e, "result copy");
    }
    if ((e = hipEventRecord(srv->ev, s)) != hipSuccess) return hip_fail(e, "hipEventRecord");
    if ((e = hipEventSynchronize(srv->ev)) != hipSuccess)
        return hip_fail(e, "hipEventSynchronize");
    const uint64_t t_done = cwt_now_ns();
    for (int j = 0; j < n; ++j) {
        PendingHop &h = batch[j];
        Result r;
        r.hop_idx = h.hop_idx;
        r.t_push = h.t_push;
        r.t_done = t_done;
        const int row = k.h_jobs[j].emit_row;
        if (row >= 0) r.bp.assign(k.h_out + (size_t)row * C * nb, k.h_out + (size_t)(row + 1) * C * nb);
        done.emplace_back(h.s, std::move(r));
    }
    return CWT_OK;
}

void worker_main(cwt_server *srv)
{
    (void)hipSetDevice(srv->device);
    std::unique_lock<std::mutex> lk(srv->mu);
    for (;;) {
        srv->cv_work.wait(lk, [&] { return srv->stop || !srv->pending.empty(); });
        if (srv->pending.empty()) {
            if (srv->stop) break;
            continue;
        }
        // Wait for a full batch or the oldest hop's deadline.
        const uint64_t deadline = srv->pending.front().t_enq + (uint64_t)srv->opts.deadline_us * 1000;
        while (!srv->stop && (int)srv->pending.size() < srv->opts.max_batch) {
            const uint64_t now = cwt_now_ns();
            if (now >= deadline) break;
            srv->cv_work.wait_for(lk, std::chrono::nanoseconds(deadline - now));
        }
        StreamClass *cls = srv->pending.front().s->cls;
        std::vector<PendingHop> batch;
        std::unordered_set<cwt_session *> seen;
        std::deque<PendingHop> rest;
        while (!srv->pending.empty()) {
            PendingHop h = std::move(srv->pending.front());
            srv->pending.pop_front();
            if (h.s->cls == cls && (int)batch.size() < srv->opts.max_batch && !seen.count(h.s)) {
                seen.insert(h.s);
                batch.push_back(std::move(h));
            } else {
                rest.push_back(std::move(h));
            }
        }
        srv->pending.swap(rest);
        srv->in_flight = 1;
        lk.unlock();
        std::vector<std::pair<cwt_session *, Result>> done;
        int rc = CWT_OK;
        if (srv->error == CWT_OK) rc = run_batch(srv, *cls, batch, done);
        lk.lock();
        if (rc != CWT_OK && srv->error == CWT_OK) {
            srv->error = rc;
            srv->error_msg = cwt_last_error();
        }
        for (auto &d : done) {
            cwt_session *s = d.first;
            if (!d.second.bp.empty()) {
                s->results.push_back(std::move(d.second));
                srv->stats.results++;
            }
        }
        for (auto &h : batch) h.s->queued--;
        srv->stats.batches++;
        srv->stats.hops += batch.size();
        srv->in_flight = 0;
        srv->cv_done.notify_all();
    }
}

}  // namespace

extern "C" int cwt_server_opts_init(cwt_server_opts *o)
{
    if (!o) return fail(CWT_E_INVALID, "cwt_server_opts_init: NULL");
    std::memset(o, 0, sizeof *o);
    o->max_batch = 256;
    o->deadline_us = 500;
    o->max_pending = 64;
    return CWT_OK;
}

extern "C" int cwt_server_create(cwt_server **out, size_t budget, const cwt_server_opts *opts)
{
    clear_error();
    if (!out) return fail(CWT_E_INVALID, "cwt_server_create: out is NULL");
    *out = nullptr;
    cwt_server_opts o;
    cwt_server_opts_init(&o);
    if (opts) o = *opts;
    if (o.max_batch < 1 || o.max_batch > 65536)
        return fail(CWT_E_INVALID, "max_batch must be in [1, 65536]");
    if (o.deadline_us < 0) return fail(CWT_E_INVALID, "deadline_us must be >= 0");
    if (o.max_pending < 1) return fail(CWT_E_INVALID, "max_pending must be >= 1");
    if (budget == 0) return fail(CWT_E_INVALID, "hbm_budget_bytes must be > 0");
    int dev = 0;
    int rc = check_device(&dev);
    if (rc != CWT_OK) return rc;
    cwt_server *srv = new (std::nothrow) cwt_server();
    if (!srv) return fail(CWT_E_NOMEM, "host allocation of the server failed");
    srv->budget = budget;
    srv->opts = o;
    srv->device = dev;
    hipError_t e = hipStreamCreateWithFlags(&srv->stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&srv->ev, hipEventDisableTiming);
    if (e != hipSuccess) {
        if (srv->stream) (void)hipStreamDestroy(srv->stream);
        delete srv;
        return hip_fail(e, "server stream/event creation");
    }
    srv->stats.hbm_budget_bytes = budget;
    srv->worker = std::thread(worker_main, srv);
    *out = srv;
    return CWT_OK;
}

static void release_session_locked(cwt_server *srv, cwt_session *s)
{
    if (s->d_ring) (void)hipFree(s->d_ring);
    srv->used -= s->ring_bytes;
    StreamClass *k = s->cls;
    if (k && --k->n_sessions == 0) {
        srv->used -= k->dev_bytes;
        for (size_t i = 0; i < srv->classes.size(); ++i)
            if (srv->classes[i].get() == k) {
                free_class(*k);
                srv->classes.erase(srv->classes.begin() + i);
                break;
            }
    }
    srv->sessions.erase(std::remove(srv->sessions.begin(), srv->sessions.end(), s),
                        srv->sessions.end());
    srv->stats.sessions_open = srv->sessions.size();
    srv->stats.hbm_bytes_used = srv->used;
    delete s;
}

extern "C" int cwt_server_destroy(cwt_server *srv)
{
    if (!srv) return CWT_OK;
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        srv->stop = true;
    }
    srv->cv_work.notify_all();
    if (srv->worker.joinable()) srv->worker.join();
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        while (!srv->sessions.empty()) release_session_locked(srv, srv->sessions.back());
        for (auto &k : srv->classes) free_class(*k);
        srv->classes.clear();
    }
    (void)hipEventDestroy(srv->ev);
    (void)hipStreamDestroy(srv->stream);
    delete srv;
    return CWT_OK;
}

extern "C" int cwt_stream_open(cwt_server *srv, const cwt_plan *plan, int64_t C, int64_t hop,
                               cwt_session **out)
{
    clear_error();
    if (!srv || !plan || !out) return fail(CWT_E_INVALID, "cwt_stream_open: NULL argument");
    *out = nullptr;
    if (plan->opts.out != CWT_OUT_BANDPOWER_F32)
        return fail(CWT_E_INVALID, "stream sessions need a plan with CWT_OUT_BANDPOWER_F32");
    if (plan->opts.precision != CWT_PREC_FP32)
        return fail(CWT_E_UNSUPPORTED, "stream sessions run the FP32 path");
    if (plan->user)
        return fail(CWT_E_UNSUPPORTED,
                    "stream sessions need a closed-form wavelet (plans from sampled wavelets "
                    "have complex spectra)");
    const int64_t W = plan->n;
    if (C < 1 || C > 4096) return fail(CWT_E_INVALID, "C must be in [1, 4096]");
    if (hop < 1 || hop > W) return fail(CWT_E_INVALID, "hop must be in [1, n = %lld]", (long long)W);
    if ((size_t)plan->max_bins * 8 + 1024 > 160 * 1024)
        return fail(CWT_E_UNSUPPORTED, "spectrum band too wide for the stream kernel's LDS");
    std::lock_guard<std::mutex> lk(srv->mu);
    if (srv->error != CWT_OK) return fail(srv->error, "server failed: %s", srv->error_msg.c_str());
    const int mb = srv->opts.max_batch;
    if ((int64_t)mb * C * W > (int64_t)INT32_MAX || (int64_t)mb * C * hop > (int64_t)INT32_MAX)
        return fail(CWT_E_UNSUPPORTED, "max_batch x C x n exceeds the index range");
    StreamClass *cls = nullptr;
    for (auto &k : srv->classes)
        if (k->plan == plan && k->C == C && k->hop == hop) cls = k.get();
    const int Lh = plan->L / 2 + 1;
    const size_t ring_bytes = align256((size_t)C * W * 4);
    const int ng = plan->grp_off.empty() ? 0 : plan->grp_off.back();
    const size_t cls_bytes =
        cls ? 0 : class_dev_bytes(mb, (int)C, (int)hop, (int)W, Lh, plan->n_bands, ng);
    if (srv->used + ring_bytes + cls_bytes > srv->budget)
        return fail(CWT_E_BUDGET, "session needs %zu bytes, %zu of %zu in use",
                    ring_bytes + cls_bytes, srv->used, srv->budget);
    cwt_session *s = new (std::nothrow) cwt_session();
    if (!s) return fail(CWT_E_NOMEM, "host allocation of the session failed");
    std::unique_ptr<StreamClass> fresh;
    if (!cls) {
        fresh.reset(new (std::nothrow) StreamClass());
        if (!fresh) {
            delete s;
            return fail(CWT_E_NOMEM, "host allocation of the stream class failed");
        }
        fresh->plan = plan;
        fresh->C = (int)C;
        fresh->hop = (int)hop;
        fresh->W = (int)W;
        fresh->Lh = Lh;
        fresh->nb = plan->n_bands;
        fresh->ng = ng;
        fresh->max_batch = mb;
        fresh->dev_bytes = cls_bytes;
        int rc = alloc_class(*fresh);
        if (rc != CWT_OK) {
            free_class(*fresh);
            delete s;
            return rc;
        }
        cls = fresh.get();
    }
    hipError_t e = hipMalloc((void **)&s->d_ring, ring_bytes);
    if (e == hipSuccess) e = hipMemsetAsync(s->d_ring, 0, ring_bytes, srv->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(srv->stream);
    if (e != hipSuccess) {
        if (s->d_ring) (void)hipFree(s->d_ring);
        if (fresh) free_class(*fresh);
        delete s;
        return fail(CWT_E_NOMEM, "ring allocation failed: %s", hipGetErrorName(e));
    }
    if (fresh) srv->classes.push_back(std::move(fresh));
    cls->n_sessions++;
    s->srv = srv;
    s->plan = plan;
    s->cls = cls;
    s->C = (int)C;
    s->W = (int)W;
    s->hop = (int)hop;
    s->nb = plan->n_bands;
    s->ring_bytes = ring_bytes;
    s->acc.assign((size_t)C * hop, 0.f);
    srv->used += ring_bytes + cls_bytes;
    srv->sessions.push_back(s);
    srv->stats.sessions_open = srv->sessions.size();
    srv->stats.hbm_bytes_used = srv->used;
    *out = s;
    return CWT_OK;
}

extern "C" int cwt_stream_push(cwt_session *s, const float *samples, int64_t m,
                               uint64_t t_arrival_ns)
{
    clear_error();
    if (!s) return fail(CWT_E_INVALID, "cwt_stream_push: session is NULL");
    if (m < 0) return fail(CWT_E_INVALID, "m must be >= 0");
    if (m == 0) return CWT_OK;
    if (!samples) return fail(CWT_E_INVALID, "samples is NULL");
    cwt_server *srv = s->srv;
    const uint64_t t = t_arrival_ns ? t_arrival_ns : cwt_now_ns();
    int new_hops;
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        if (srv->error != CWT_OK)
            return fail(srv->error, "server failed: %s", srv->error_msg.c_str());
        new_hops = (int)((s->acc_fill + m) / s->hop);
        if (s->queued + new_hops > srv->opts.max_pending) {
            srv->stats.rejected++;
            return fail(CWT_E_AGAIN, "session has %d hops queued (max_pending %d)", s->queued,
                        srv->opts.max_pending);
        }
        const uint64_t now = cwt_now_ns();
        int64_t used = 0;
        while (used < m) {
            const int64_t take = std::min<int64_t>(s->hop - s->acc_fill, m - used);
            for (int c = 0; c < s->C; ++c)
                std::memcpy(&s->acc[(size_t)c * s->hop + s->acc_fill],
                            samples + (size_t)c * m + used, (size_t)take * 4);
            s->acc_fill += (int)take;
            used += take;
            s->samples_in += (uint64_t)take;
            if (s->acc_fill == s->hop) {
                PendingHop h;
                h.s = s;
                h.t_push = t;
                h.t_enq = now;
                h.hop_idx = s->next_hop_idx++;
                h.emit = s->samples_in >= (uint64_t)s->W;
                h.data = s->acc;
                srv->pending.push_back(std::move(h));
                s->queued++;
                s->acc_fill = 0;
            }
        }
    }
    if (new_hops > 0) srv->cv_work.notify_one();
    return CWT_OK;
}

extern "C" int cwt_stream_poll(cwt_session *s, float *bp, uint64_t *hop_idx, uint64_t *t_push_ns,
                               uint64_t *t_done_ns)
{
    if (!s) return fail(CWT_E_INVALID, "cwt_stream_poll: session is NULL");
    std::lock_guard<std::mutex> lk(s->srv->mu);
    if (s->results.empty()) {
        if (s->srv->error != CWT_OK)
            return fail(s->srv->error, "server failed: %s", s->srv->error_msg.c_str());
        return CWT_E_AGAIN;
    }
    Result &r = s->results.front();
    if (bp) std::memcpy(bp, r.bp.data(), r.bp.size() * 4);
    if (hop_idx) *hop_idx = r.hop_idx;
    if (t_push_ns) *t_push_ns = r.t_push;
    if (t_done_ns) *t_done_ns = r.t_done;
    s->results.pop_front();
    return CWT_OK;
}

extern "C" int cwt_server_flush(cwt_server *srv)
{
    if (!srv) return fail(CWT_E_INVALID, "cwt_server_flush: NULL");
    std::unique_lock<std::mutex> lk(srv->mu);
    srv->cv_work.notify_all();
    srv->cv_done.wait(lk, [&] { return srv->pending.empty() && srv->in_flight == 0; });
    if (srv->error != CWT_OK) return fail(srv->error, "server failed: %s", srv->error_msg.c_str());
    return CWT_OK;
}

extern "C" int cwt_stream_close(cwt_session *s)
{
    if (!s) return CWT_OK;
    cwt_server *srv = s->srv;
    std::unique_lock<std::mutex> lk(srv->mu);
    // drop this session's pending hops, then wait for one in flight
    std::deque<PendingHop> keep;
    for (auto &h : srv->pending) {
        if (h.s == s)
            s->queued--;
        else
            keep.push_back(std::move(h));
    }
    srv->pending.swap(keep);
    srv->cv_done.wait(lk, [&] { return s->queued == 0; });
    release_session_locked(srv, s);
    return CWT_OK;
}

extern "C" int cwt_server_get_stats(const cwt_server *srv, cwt_server_stats *st)
{
    if (!srv || !st) return fail(CWT_E_INVALID, "cwt_server_get_stats: NULL");
    std::lock_guard<std::mutex> lk(const_cast<cwt_server *>(srv)->mu);
    *st = srv->stats;
    return CWT_OK;
}
