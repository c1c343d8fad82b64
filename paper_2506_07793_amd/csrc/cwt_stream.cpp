// Streaming server of libcwt: sessions, HBM-budget admission, hop batching,
// pipelined launches, latency stamps.
//
// Sessions push host samples; every completed hop becomes a pending job.  A
// launcher thread forms batches of hops that share a (plan, C, hop) class
// and enqueues them on the server's stream; a completion thread waits for
// each batch in launch order and delivers its band-power results with their
// completion time stamps, so the next batch is already queued on the GPU
// while the previous one finishes and its results are read back.
//
// A batch may hold several hops of one session, in order: all of them are
// appended to the session's ring before any window is gathered, so the ring
// keeps R = W + (K - 1) hop samples per channel, enough for K windows of the
// session in one launch (hops before the first full window produce no window
// and do not count against K).
//
// Every device operation (allocation, ring clearing, copies, launches, frees)
// is enqueued on the server's stream, so no call waits for the device: a
// ring freed at close is reused only after the launches that read it.
#include <hip/hip_runtime.h>
#include <time.h>

#include <algorithm>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <unordered_map>
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

constexpr int kSlots = 2;  // batches of one class in flight at once

// Host staging of one in-flight batch (pinned): the hops' samples and job
// table going up, the band powers coming back.
struct Staging {
    float *h_slab = nullptr;
    StreamJob *h_jobs = nullptr;
    float *h_out = nullptr;
    hipEvent_t done = nullptr;
    bool busy = false;
};

// Buffers of one (plan, C, hop) class.  The device buffers are shared by the
// class's batches (they run in stream order); the host staging is per slot.
struct StreamClass {
    const cwt_plan *plan = nullptr;
    int C = 0, hop = 0, W = 0, R = 0, Lh = 0, nb = 0, ng = 0, max_batch = 0;
    float *d_slab = nullptr;
    StreamJob *d_jobs = nullptr;
    float *d_xb = nullptr;
    float2 *d_Xh = nullptr;
    float *d_out = nullptr;
    float *d_part = nullptr;  // [rows][ng] per-frequency sums over the hop
    Staging st[kSlots];
    size_t dev_bytes = 0;
    int n_sessions = 0;
};

// Device buffers of a class: {pointer, bytes} in allocation order.
struct DevBuf {
    void **p;
    size_t n;
};

std::vector<DevBuf> class_dev_bufs(StreamClass &k)
{
    const size_t mb = (size_t)k.max_batch, c = (size_t)k.C;
    return {{(void **)&k.d_slab, align256(mb * c * k.hop * 4)},
            {(void **)&k.d_jobs, align256(mb * sizeof(StreamJob))},
            {(void **)&k.d_xb, align256(mb * c * k.W * 4)},
            {(void **)&k.d_Xh, align256(mb * c * k.Lh * 8)},
            {(void **)&k.d_out, align256(mb * c * k.nb * 4)},
            {(void **)&k.d_part, align256(mb * c * std::max(k.ng, 1) * 4)}};
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

// One launched batch, waiting for completion.
struct InFlight {
    StreamClass *cls;
    int slot;
    uint64_t t_formed;  // host clock when the batch was taken from the queue
    struct Hop {
        cwt_session *s;
        uint64_t hop_idx, t_push;
        int emit_row;
    };
    std::vector<Hop> hops;
};

}  // namespace

struct cwt_session {
    cwt_server *srv = nullptr;
    const cwt_plan *plan = nullptr;
    StreamClass *cls = nullptr;
    int C = 0, W = 0, R = 0, hop = 0, nb = 0;
    float *d_ring = nullptr;
    size_t ring_bytes = 0;
    int ring_pos = 0;          // launcher-side: ring slot of the next hop's first sample
    uint64_t samples_in = 0;   // push-side: samples accepted
    std::vector<float> acc;    // push-side: partial hop [C][hop]
    int acc_fill = 0;
    uint64_t next_hop_idx = 0;
    int queued = 0;            // hops not yet delivered (pending or in flight)
    int queued_windows = 0;    // of those, hops that produce a window
    std::deque<Result> results;
};

struct cwt_server {
    size_t budget = 0, used = 0;
    cwt_server_opts opts{};
    DevMem mem{};
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    std::mutex mu;
    std::condition_variable cv_work, cv_done, cv_flight;
    std::deque<PendingHop> pending;
    std::deque<InFlight> flight;  // launched, in launch order
    std::vector<cwt_session *> sessions;
    std::vector<std::unique_ptr<StreamClass>> classes;
    std::thread launcher, completer;
    bool stop = false;
    bool launcher_done = false;
    int launching = 0;  // batches formed but not yet in `flight`
    int error = CWT_OK;
    std::string error_msg;
    cwt_server_stats stats{};
};

namespace {

void free_class(cwt_server *srv, StreamClass &k)
{
    for (const DevBuf &b : class_dev_bufs(k)) {
        dev_free(srv->mem, *b.p, b.n, srv->stream);
        *b.p = nullptr;
    }
    for (Staging &st : k.st) {
        void *hptr[] = {st.h_slab, st.h_jobs, st.h_out};
        for (void *p : hptr)
            if (p) (void)hipHostFree(p);
        if (st.done) (void)hipEventDestroy(st.done);
        st = Staging{};
    }
}

int alloc_class(cwt_server *srv, StreamClass &k)
{
    for (const DevBuf &b : class_dev_bufs(k)) {
        int rc = dev_alloc(srv->mem, b.p, b.n, srv->stream, "stream batch buffer");
        if (rc != CWT_OK) return rc;
    }
    const size_t mb = (size_t)k.max_batch, c = (size_t)k.C;
    for (Staging &st : k.st) {
        struct {
            void **p;
            size_t n;
        } host[] = {{(void **)&st.h_slab, mb * c * k.hop * 4},
                    {(void **)&st.h_jobs, mb * sizeof(StreamJob)},
                    {(void **)&st.h_out, mb * c * k.nb * 4}};
        for (auto &h : host) {
            if (hipHostMalloc(h.p, std::max<size_t>(h.n, 256), hipHostMallocDefault) !=
                hipSuccess) {
                *h.p = nullptr;
                return fail(CWT_E_NOMEM, "pinned staging allocation of %zu bytes failed", h.n);
            }
        }
        hipError_t e = hipEventCreateWithFlags(&st.done, hipEventDisableTiming);
        if (e != hipSuccess) return hip_fail(e, "stream batch event");
    }
    return CWT_OK;
}

// Enqueue one batch from staging slot `st` (no wait).  Runs on the launcher
// thread without the server lock; touches only the batch, the class buffers
// and the sessions' ring positions (which only the launcher uses).
int launch_batch(cwt_server *srv, StreamClass &k, Staging &st, std::vector<PendingHop> &batch,
                 InFlight &fl)
{
    const int n = (int)batch.size();
    const int C = k.C, hop = k.hop, W = k.W, nb = k.nb;
    int n_emit = 0;
    fl.hops.clear();
    for (int j = 0; j < n; ++j) {
        PendingHop &h = batch[j];
        std::memcpy(st.h_slab + (size_t)j * C * hop, h.data.data(), (size_t)C * hop * 4);
        StreamJob &jb = st.h_jobs[j];
        jb.ring = h.s->d_ring;
        jb.pos = h.s->ring_pos;
        jb.slab_off = j * C * hop;
        jb.emit_row = h.emit ? n_emit++ : -1;
        jb.pad_ = 0;
        h.s->ring_pos = (h.s->ring_pos + hop) % h.s->R;
        fl.hops.push_back({h.s, h.hop_idx, h.t_push, jb.emit_row});
    }
    hipStream_t s = srv->stream;
    hipError_t e;
    if ((e = hipMemcpyAsync(k.d_jobs, st.h_jobs, (size_t)n * sizeof(StreamJob),
                            hipMemcpyHostToDevice, s)) != hipSuccess)
        return hip_fail(e, "stream jobs copy");
    if ((e = hipMemcpyAsync(k.d_slab, st.h_slab, (size_t)n * C * hop * 4, hipMemcpyHostToDevice,
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
    sp.R = k.R;
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
        if ((e = hipMemcpyAsync(st.h_out, k.d_out, (size_t)n_emit * C * nb * 4,
                                hipMemcpyDeviceToHost, s)) != hipSuccess)
            return hip_fail(e, "result copy");
    }
    if ((e = hipEventRecord(st.done, s)) != hipSuccess) return hip_fail(e, "hipEventRecord");
    return CWT_OK;
}

void set_error(cwt_server *srv, int rc)
{
    if (rc != CWT_OK && srv->error == CWT_OK) {
        srv->error = rc;
        srv->error_msg = cwt_last_error();
    }
}

// Take from `pending` the next batch of the front hop's class: hops in queue
// order, at most max_batch of them, each session's hops in order and at most
// K of a session's window-producing hops (a session's hops after one it
// could not take stay queued, behind it).
void form_batch(cwt_server *srv, std::vector<PendingHop> &batch, StreamClass *&cls)
{
    cls = srv->pending.front().s->cls;
    const int K = srv->opts.max_session_windows;  // windows per session per launch
    std::unordered_map<cwt_session *, int> emits;
    std::unordered_map<cwt_session *, bool> blocked;
    std::deque<PendingHop> rest;
    while (!srv->pending.empty()) {
        PendingHop h = std::move(srv->pending.front());
        srv->pending.pop_front();
        bool take = h.s->cls == cls && (int)batch.size() < srv->opts.max_batch &&
                    !blocked[h.s];
        if (take && h.emit) {
            int &ne = emits[h.s];
            if (ne >= K)
                take = false;
            else
                ++ne;
        }
        if (take) {
            batch.push_back(std::move(h));
        } else {
            blocked[h.s] = true;
            rest.push_back(std::move(h));
        }
    }
    srv->pending.swap(rest);
}

void launcher_main(cwt_server *srv)
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
        const uint64_t deadline =
            srv->pending.front().t_enq + (uint64_t)srv->opts.deadline_us * 1000;
        while (!srv->stop && (int)srv->pending.size() < srv->opts.max_batch) {
            const uint64_t now = cwt_now_ns();
            if (now >= deadline) break;
            srv->cv_work.wait_for(lk, std::chrono::nanoseconds(deadline - now));
        }
        if (srv->pending.empty()) continue;  // a close dropped them
        // A free staging slot of the front hop's class (the completion
        // thread frees one when a batch of that class completes).
        StreamClass *cls = srv->pending.front().s->cls;
        int slot = -1;
        for (;;) {
            for (int i = 0; i < kSlots; ++i)
                if (!cls->st[i].busy) slot = i;
            if (slot >= 0 || srv->error != CWT_OK) break;
            srv->stats.slot_waits++;
            srv->cv_done.wait(lk);
            if (srv->pending.empty() || srv->pending.front().s->cls != cls) break;
        }
        if (slot < 0 && srv->error == CWT_OK) continue;  // the queue changed while waiting
        std::vector<PendingHop> batch;
        form_batch(srv, batch, cls);
        InFlight fl;
        fl.cls = cls;
        fl.slot = slot;
        fl.t_formed = cwt_now_ns();
        int rc = srv->error;
        if (rc == CWT_OK) {
            cls->st[slot].busy = true;
            srv->launching++;
            lk.unlock();
            rc = launch_batch(srv, *cls, cls->st[slot], batch, fl);
            lk.lock();
            srv->launching--;
        }
        if (rc != CWT_OK) {
            set_error(srv, rc);
            if (slot >= 0) cls->st[slot].busy = false;
            for (auto &h : batch) {  // dropped
                h.s->queued--;
                if (h.emit) h.s->queued_windows--;
            }
            srv->cv_done.notify_all();
            continue;
        }
        srv->flight.push_back(std::move(fl));
        srv->cv_flight.notify_one();
    }
    srv->launcher_done = true;
    srv->cv_flight.notify_all();
}

void completer_main(cwt_server *srv)
{
    (void)hipSetDevice(srv->device);
    std::unique_lock<std::mutex> lk(srv->mu);
    for (;;) {
        srv->cv_flight.wait(lk, [&] { return srv->launcher_done || !srv->flight.empty(); });
        if (srv->flight.empty()) {
            if (srv->launcher_done) break;
            continue;
        }
        InFlight &fl = srv->flight.front();
        Staging &st = fl.cls->st[fl.slot];
        lk.unlock();
        hipError_t e = hipEventSynchronize(st.done);
        const uint64_t t_done = cwt_now_ns();
        lk.lock();
        if (e != hipSuccess) set_error(srv, hip_fail(e, "stream batch completion"));
        const int C = fl.cls->C, nb = fl.cls->nb;
        for (const InFlight::Hop &h : fl.hops) {
            if (h.emit_row >= 0 && e == hipSuccess) {
                Result r;
                r.hop_idx = h.hop_idx;
                r.t_push = h.t_push;
                r.t_done = t_done;
                r.bp.assign(st.h_out + (size_t)h.emit_row * C * nb,
                            st.h_out + (size_t)(h.emit_row + 1) * C * nb);
                h.s->results.push_back(std::move(r));
                srv->stats.results++;
            }
            h.s->queued--;
            if (h.emit_row >= 0) h.s->queued_windows--;
        }
        srv->stats.batches++;
        srv->stats.hops += fl.hops.size();
        srv->stats.max_batch_hops = std::max<uint64_t>(srv->stats.max_batch_hops, fl.hops.size());
        srv->stats.max_batch_ns = std::max<uint64_t>(srv->stats.max_batch_ns, t_done - fl.t_formed);
        st.busy = false;
        srv->flight.pop_front();
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
    o->max_session_windows = 4;
    return CWT_OK;
}

extern "C" int cwt_server_create(cwt_server **out, size_t budget, const cwt_server_opts *opts,
                                 void *stream)
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
    if (o.max_session_windows == 0) o.max_session_windows = 4;
    if (o.max_session_windows < 1 || o.max_session_windows > 64)
        return fail(CWT_E_INVALID, "windows per session per launch must be in [1, 64]");
    if (budget == 0) return fail(CWT_E_INVALID, "hbm_budget_bytes must be > 0");
    const DevMem m{o.alloc, o.free, o.alloc_ctx};
    int rc = check_dev_mem(m);
    if (rc != CWT_OK) return rc;
    int dev = 0;
    rc = check_device(&dev);
    if (rc != CWT_OK) return rc;
    cwt_server *srv = new (std::nothrow) cwt_server();
    if (!srv) return fail(CWT_E_NOMEM, "host allocation of the server failed");
    srv->budget = budget;
    srv->opts = o;
    srv->mem = m;
    srv->device = dev;
    if (stream) {
        srv->stream = (hipStream_t)stream;
    } else {
        hipError_t e = hipStreamCreateWithFlags(&srv->stream, hipStreamNonBlocking);
        if (e != hipSuccess) {
            delete srv;
            return hip_fail(e, "server stream creation");
        }
        srv->own_stream = true;
    }
    srv->stats.hbm_budget_bytes = budget;
    srv->launcher = std::thread(launcher_main, srv);
    srv->completer = std::thread(completer_main, srv);
    *out = srv;
    return CWT_OK;
}

static void release_session_locked(cwt_server *srv, cwt_session *s)
{
    dev_free(srv->mem, s->d_ring, s->ring_bytes, srv->stream);  // after the launches using it
    srv->used -= s->ring_bytes;
    StreamClass *k = s->cls;
    if (k && --k->n_sessions == 0) {
        srv->used -= k->dev_bytes;
        for (size_t i = 0; i < srv->classes.size(); ++i)
            if (srv->classes[i].get() == k) {
                free_class(srv, *k);
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
    srv->cv_done.notify_all();
    if (srv->launcher.joinable()) srv->launcher.join();
    if (srv->completer.joinable()) srv->completer.join();
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        while (!srv->sessions.empty()) release_session_locked(srv, srv->sessions.back());
        for (auto &k : srv->classes) free_class(srv, *k);
        srv->classes.clear();
    }
    if (srv->own_stream) {
        // the stream-ordered frees above complete before the stream goes
        (void)hipStreamSynchronize(srv->stream);
        (void)hipStreamDestroy(srv->stream);
    }
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
    if (plan->n_seg)
        return fail(CWT_E_UNSUPPORTED, "stream windows must fit one transform (n <= %d)",
                    CWT_MAX_LEN);
    if (plan->user)
        return fail(CWT_E_UNSUPPORTED,
                    "stream sessions need a closed-form wavelet (plans from sampled wavelets "
                    "have complex spectra)");
    const int64_t W = plan->n;
    if (C < 1 || C > 4096) return fail(CWT_E_INVALID, "C must be in [1, 4096]");
    if (hop < 1 || hop > W) return fail(CWT_E_INVALID, "hop must be in [1, n = %lld]", (long long)W);
    if ((size_t)plan->max_bins * 8 > (size_t)kStreamMaxLds)
        return fail(CWT_E_UNSUPPORTED, "spectrum band too wide for the stream kernel's LDS");
    std::lock_guard<std::mutex> lk(srv->mu);
    if (srv->error != CWT_OK) return fail(srv->error, "server failed: %s", srv->error_msg.c_str());
    const int mb = srv->opts.max_batch;
    const int64_t R = W + (int64_t)(srv->opts.max_session_windows - 1) * hop;
    if ((int64_t)mb * C * W > (int64_t)INT32_MAX || (int64_t)mb * C * hop > (int64_t)INT32_MAX ||
        R > (int64_t)INT32_MAX / 2)
        return fail(CWT_E_UNSUPPORTED, "max_batch x C x n exceeds the index range");
    StreamClass *cls = nullptr;
    for (auto &k : srv->classes)
        if (k->plan == plan && k->C == C && k->hop == hop) cls = k.get();
    const int Lh = plan->L / 2 + 1;
    const size_t ring_bytes = align256((size_t)C * R * 4);
    const int ng = plan->grp_off.empty() ? 0 : plan->grp_off.back();
    std::unique_ptr<StreamClass> fresh;
    size_t cls_bytes = 0;
    if (!cls) {
        fresh.reset(new (std::nothrow) StreamClass());
        if (!fresh) return fail(CWT_E_NOMEM, "host allocation of the stream class failed");
        fresh->plan = plan;
        fresh->C = (int)C;
        fresh->hop = (int)hop;
        fresh->W = (int)W;
        fresh->R = (int)R;
        fresh->Lh = Lh;
        fresh->nb = plan->n_bands;
        fresh->ng = ng;
        fresh->max_batch = mb;
        for (const DevBuf &b : class_dev_bufs(*fresh)) cls_bytes += b.n;
        fresh->dev_bytes = cls_bytes;
    }
    if (srv->used + ring_bytes + cls_bytes > srv->budget)
        return fail(CWT_E_BUDGET, "session needs %zu bytes, %zu of %zu in use",
                    ring_bytes + cls_bytes, srv->used, srv->budget);
    // the plan's tables may still be in flight on the stream that made them
    int rc = wait_plan_ready(*plan, srv->stream);
    if (rc != CWT_OK) return rc;
    cwt_session *s = new (std::nothrow) cwt_session();
    if (!s) return fail(CWT_E_NOMEM, "host allocation of the session failed");
    if (fresh) {
        rc = alloc_class(srv, *fresh);
        if (rc != CWT_OK) {
            free_class(srv, *fresh);
            delete s;
            return rc;
        }
        cls = fresh.get();
    }
    // stream-ordered allocation and clearing (no wait): every launch that
    // reads the ring is enqueued after these on the same stream
    rc = dev_alloc(srv->mem, (void **)&s->d_ring, ring_bytes, srv->stream, "session ring");
    if (rc == CWT_OK) {
        hipError_t e = hipMemsetAsync(s->d_ring, 0, ring_bytes, srv->stream);
        if (e != hipSuccess) rc = hip_fail(e, "ring clear");
    }
    if (rc != CWT_OK) {
        dev_free(srv->mem, s->d_ring, ring_bytes, srv->stream);
        if (fresh) free_class(srv, *fresh);
        delete s;
        return rc;
    }
    if (fresh) srv->classes.push_back(std::move(fresh));
    cls->n_sessions++;
    s->srv = srv;
    s->plan = plan;
    s->cls = cls;
    s->C = (int)C;
    s->W = (int)W;
    s->R = (int)R;
    s->hop = (int)hop;
    s->nb = plan->n_bands;
    s->ring_bytes = ring_bytes;
    // the first hop lands so that the ring's last W slots hold the window of
    // zeros preceding it (positions are taken mod R)
    s->ring_pos = 0;
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
        // Hops before the first full window only fill the ring and are not
        // held against max_pending: new hop i (1-based) ends at base + i hop,
        // and produces a window once that reaches W.
        const int64_t base = (int64_t)s->samples_in - s->acc_fill;
        int64_t fill_only = 0;
        if (base < s->W) fill_only = (s->W - base + s->hop - 1) / s->hop - 1;
        const int emitting = (int)std::max<int64_t>(0, new_hops - fill_only);
        if (s->queued_windows + emitting > srv->opts.max_pending) {
            srv->stats.rejected++;
            return fail(CWT_E_AGAIN, "session has %d window hops queued (max_pending %d)",
                        s->queued_windows, srv->opts.max_pending);
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
                s->queued_windows += h.emit ? 1 : 0;
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
    srv->cv_done.wait(lk, [&] {
        return srv->pending.empty() && srv->flight.empty() && srv->launching == 0;
    });
    if (srv->error != CWT_OK) return fail(srv->error, "server failed: %s", srv->error_msg.c_str());
    return CWT_OK;
}

extern "C" int cwt_stream_close(cwt_session *s)
{
    if (!s) return CWT_OK;
    cwt_server *srv = s->srv;
    std::unique_lock<std::mutex> lk(srv->mu);
    // drop this session's pending hops, then wait for those already launched
    std::deque<PendingHop> keep;
    for (auto &h : srv->pending) {
        if (h.s == s) {
            s->queued--;
            if (h.emit) s->queued_windows--;
        } else {
            keep.push_back(std::move(h));
        }
    }
    srv->pending.swap(keep);
    srv->cv_done.notify_all();  // a launcher waiting for a slot re-reads the queue
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
