// Batched form of libcwt: recordings of uneven length, channel count and
// frequency grid in one graph launch.
//
// The host builds, in the caller's workspace, a parameter table per item and
// two task lists (channel pairs for the forward transforms, runs of output
// rows of one channel for the transforms), sorted by estimated cost so that
// the long tasks start first.  Tasks are grouped into classes by workgroup
// size; each class runs one persistent forward kernel whose workgroups claim
// tasks through an atomic counter, and one transform kernel: persistent in
// the same way for the 16-value classes, one row per workgroup (handed out
// by the hardware dispatcher, one class per output mode) for the 24-value
// classes, whose persistent kernel would not fit in its registers.  The
// launches are captured once into a HIP graph per (workspace, layout) and
// replayed.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <tuple>
#include <vector>

#include "../../include/cwt.h"
#include "cwt_internal.hpp"
#include "cwt_kernels.hpp"

using namespace cwtk;
using namespace cwtrt;

namespace {

size_t al(size_t b) { return (b + 255) & ~(size_t)255; }

// Workgroup-size classes: a task may run with more threads than its plan
// needs (each thread then holds fewer butterflies), never fewer.
// Workgroup size of a class: the plan's rounded up to 64, 128, 256, 512 or
// the largest workgroup of its values-per-thread class (1024, or 768 for 32
// values per thread, whose kernels are compiled for at most 768 threads).
int class_threads(int t, int maxv)
{
    const int tmax = generic_max_threads(maxv);
    for (int c : {64, 128, 256, 512})
        if (t <= c) return c;
    return tmax;
}

struct ClassInfo {
    int threads = 0, maxv = 16;
    int max_L = 1;
    // 24-value classes run one row per workgroup (k_batch_rows, one output
    // mode per class): their persistent kernel would spill registers
    bool rows = false;
    int mode = -1;
    std::vector<BatchTask> fwd, main;
    std::vector<double> fwd_cost, main_cost;  // sort keys (larger first)
    double total = 0;                          // sum of main_cost
};

// Estimated cost of one transform row of a plan: L log2 L (FFT work).
double row_cost(const cwt_plan &P) { return P.L * std::log2((double)std::max(2, P.L)); }

// Rows per transform task: enough consecutive rows of one channel that a
// task is worth an atomic claim and a barrier, few enough to balance.
constexpr double kTaskCost = 1 << 20;

struct Layout {
    size_t counters = 0, fwd_items = 0, main_items = 0, fwd_tasks = 0, main_tasks = 0, xh = 0,
           total = 0;
    std::vector<size_t> xh_off;  // per item, bytes from ws
};

Layout make_layout(const cwt_batch_item *items, int n, size_t n_fwd, size_t n_main)
{
    Layout Lo;
    size_t off = 0;
    Lo.counters = off;
    off += al(64 * sizeof(int));
    Lo.fwd_items = off;
    off += al((size_t)n * sizeof(FwdParams));
    Lo.main_items = off;
    off += al((size_t)n * sizeof(MainParams));
    Lo.fwd_tasks = off;
    off += al(n_fwd * sizeof(BatchTask));
    Lo.main_tasks = off;
    off += al(n_main * sizeof(BatchTask));
    Lo.xh = off;
    Lo.xh_off.resize(n);
    for (int i = 0; i < n; ++i) {
        Lo.xh_off[i] = off;
        off += workspace_bytes(*items[i].plan, items[i].C);
    }
    Lo.total = off;
    return Lo;
}

int validate(const cwt_batch_item *items, int n)
{
    if (n < 0) return fail(CWT_E_INVALID, "n must be >= 0");
    if (n > 0 && !items) return fail(CWT_E_INVALID, "items is NULL");
    for (int i = 0; i < n; ++i) {
        const cwt_batch_item &it = items[i];
        if (!it.plan) return fail(CWT_E_INVALID, "items[%d].plan is NULL", i);
        if (it.C < 0 || it.C > (int64_t)1 << 24) return fail(CWT_E_INVALID, "items[%d].C out of range", i);
        if (it.C > 0 && (!it.x || !it.out))
            return fail(CWT_E_INVALID, "items[%d] has a NULL device pointer", i);
        if (it.plan->opts.precision != CWT_PREC_FP32)
            return fail(CWT_E_UNSUPPORTED, "items[%d]: batches run the FP32 path", i);
        if (it.plan->n_seg)
            return fail(CWT_E_UNSUPPORTED,
                        "items[%d]: segmented plans (padded length above %d) run through "
                        "cwt_execute", i, CWT_MAX_LEN);
        const int64_t rows =
            (it.plan->opts.out == CWT_OUT_BANDPOWER_F32) ? it.plan->n_bands : it.plan->F;
        if (it.C * rows > (int64_t)INT32_MAX)
            return fail(CWT_E_UNSUPPORTED, "items[%d]: C x rows exceeds the task range", i);
    }
    return CWT_OK;
}

// Graph cache: one instantiated graph per (workspace, layout, classes).
struct GraphKey {
    void *ws;
    int device;
    std::vector<int64_t> shape;
    bool operator<(const GraphKey &o) const
    {
        return std::tie(ws, device, shape) < std::tie(o.ws, o.device, o.shape);
    }
};

struct GraphCache {
    std::mutex mu;
    std::map<GraphKey, hipGraphExec_t> execs;
    std::map<int, hipStream_t> cap_streams;
};

GraphCache &cache()
{
    static GraphCache *c = new GraphCache();  // lives until process exit
    return *c;
}

// Pinned host staging of the tables, one per device, reused after the
// previous upload from it has completed.
struct Staging {
    std::mutex mu;
    void *host = nullptr;
    size_t cap = 0;
    hipEvent_t done = nullptr;
};

Staging &staging(int dev)
{
    static std::mutex m;
    static std::map<int, Staging *> s;
    std::lock_guard<std::mutex> lk(m);
    Staging *&p = s[dev];
    if (!p) p = new Staging();
    return *p;
}

// Side streams and fork/join events of one device: each class runs on its
// own stream so that the classes overlap (in a captured graph they become
// parallel branches between the counter reset and the join).
struct Fork {
    std::vector<hipStream_t> side;
    std::vector<hipEvent_t> join;
    hipEvent_t fork = nullptr;
};

int get_fork(int dev, size_t n, Fork *&out)
{
    static std::mutex m;
    static std::map<int, Fork *> forks;  // live until process exit
    std::lock_guard<std::mutex> lk(m);
    Fork *&f = forks[dev];
    if (!f) f = new Fork();
    hipError_t e = hipSuccess;
    const unsigned flags = hipEventDisableTiming | hipEventDisableSystemFence;
    if (!f->fork) e = hipEventCreateWithFlags(&f->fork, flags);
    while (e == hipSuccess && f->side.size() < n) {
        hipStream_t st = nullptr;
        hipEvent_t ev = nullptr;
        e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);  // default priority
        if (e == hipSuccess) e = hipEventCreateWithFlags(&ev, flags);
        if (e == hipSuccess) {
            f->side.push_back(st);
            f->join.push_back(ev);
        }
    }
    if (e != hipSuccess) return hip_fail(e, "batch side streams");
    out = f;
    return CWT_OK;
}

int enqueue_kernels(const std::vector<ClassInfo> &classes, char *ws, const Layout &Lo,
                    hipStream_t s)
{
    hipError_t e = launch_zero_counters(reinterpret_cast<int *>(ws + Lo.counters),
                                        2 * (int)classes.size(), s);
    if (e != hipSuccess) return hip_fail(e, "counter reset");
    const bool fork = classes.size() > 1;
    Fork *fk = nullptr;
    if (fork) {
        int dev = 0;
        (void)hipGetDevice(&dev);
        int rc = get_fork(dev, classes.size(), fk);
        if (rc != CWT_OK) return rc;
        e = hipEventRecord(fk->fork, s);
        if (e != hipSuccess) return hip_fail(e, "batch fork");
    }
    size_t f_off = 0, m_off = 0;
    for (size_t k = 0; k < classes.size(); ++k) {
        const ClassInfo &c = classes[k];
        hipStream_t sk = s;
        if (fork) {
            sk = fk->side[k];
            e = hipStreamWaitEvent(sk, fk->fork, 0);
            if (e != hipSuccess) return hip_fail(e, "batch fork wait");
        }
        int *ctr = reinterpret_cast<int *>(ws + Lo.counters) + 2 * k;
        const size_t lds = generic_lds_bytes(c.max_L);
        e = launch_batch_forward(reinterpret_cast<const FwdParams *>(ws + Lo.fwd_items),
                                 reinterpret_cast<const BatchTask *>(ws + Lo.fwd_tasks) + f_off,
                                 (int)c.fwd.size(), ctr, c.threads, c.maxv, lds, sk);
        if (e != hipSuccess) return hip_fail(e, "batch forward launch");
        if (c.rows)
            e = launch_batch_rows(reinterpret_cast<const MainParams *>(ws + Lo.main_items),
                                  reinterpret_cast<const BatchTask *>(ws + Lo.main_tasks) + m_off,
                                  (int)c.main.size(), c.threads, c.maxv, c.mode, lds, sk);
        else
            e = launch_batch_main(reinterpret_cast<const MainParams *>(ws + Lo.main_items),
                                  reinterpret_cast<const BatchTask *>(ws + Lo.main_tasks) + m_off,
                                  (int)c.main.size(), ctr + 1, c.threads, c.maxv, lds, sk);
        if (e != hipSuccess) return hip_fail(e, "batch transform launch");
        if (fork) {
            e = hipEventRecord(fk->join[k], sk);
            if (e == hipSuccess) e = hipStreamWaitEvent(s, fk->join[k], 0);
            if (e != hipSuccess) return hip_fail(e, "batch join");
        }
        f_off += c.fwd.size();
        m_off += c.main.size();
    }
    return CWT_OK;
}

// One item as its own pair of launches (the default form).
struct ItemLaunch {
    int item;
    int fwd_blocks, main_blocks, threads, maxv, mode;
    size_t lds;
    double cost;
};

// Items longest first, each assigned to the least loaded of up to four
// branches (the process's hardware queues); each branch runs its items'
// forward and transform launches in order.
int enqueue_items(const std::vector<ItemLaunch> &its, char *ws, const Layout &Lo, hipStream_t s)
{
    const int nb = (int)std::min<size_t>(4, its.size());
    const bool fork = nb > 1;
    Fork *fk = nullptr;
    hipError_t e;
    if (fork) {
        int dev = 0;
        (void)hipGetDevice(&dev);
        int rc = get_fork(dev, nb, fk);
        if (rc != CWT_OK) return rc;
        e = hipEventRecord(fk->fork, s);
        if (e != hipSuccess) return hip_fail(e, "batch fork");
        for (int b = 0; b < nb; ++b) {
            e = hipStreamWaitEvent(fk->side[b], fk->fork, 0);
            if (e != hipSuccess) return hip_fail(e, "batch fork wait");
        }
    }
    std::vector<double> load(nb, 0.0);
    const FwdParams *fi = reinterpret_cast<const FwdParams *>(ws + Lo.fwd_items);
    const MainParams *mi = reinterpret_cast<const MainParams *>(ws + Lo.main_items);
    for (const ItemLaunch &it : its) {
        const int b = (int)(std::min_element(load.begin(), load.end()) - load.begin());
        load[b] += it.cost;
        hipStream_t sb = fork ? fk->side[b] : s;
        e = launch_item_forward(fi, it.item, it.fwd_blocks, it.threads, it.maxv, it.lds, sb);
        if (e != hipSuccess) return hip_fail(e, "batch item forward launch");
        e = launch_item_main(mi, it.item, it.main_blocks, it.threads, it.maxv, it.mode, it.lds, sb);
        if (e != hipSuccess) return hip_fail(e, "batch item transform launch");
    }
    if (fork)
        for (int b = 0; b < nb; ++b) {
            e = hipEventRecord(fk->join[b], fk->side[b]);
            if (e == hipSuccess) e = hipStreamWaitEvent(s, fk->join[b], 0);
            if (e != hipSuccess) return hip_fail(e, "batch join");
        }
    return CWT_OK;
}

}  // namespace

extern "C" size_t cwt_batch_workspace_size(const cwt_batch_item *items, int32_t n)
{
    if (validate(items, n) != CWT_OK) return 0;
    size_t n_fwd = 0, n_main = 0;
    for (int i = 0; i < n; ++i) {
        const cwt_plan &P = *items[i].plan;
        const int64_t rows = (P.opts.out == CWT_OUT_BANDPOWER_F32) ? P.n_bands : P.F;
        n_fwd += (size_t)((items[i].C + 1) / 2);
        n_main += (size_t)(items[i].C * rows);
    }
    return make_layout(items, n, n_fwd, n_main).total;
}

extern "C" int cwt_execute_batch(const cwt_batch_item *items, int32_t n, void *ws,
                                 size_t ws_bytes, void *stream)
{
    clear_error();
    int rc = validate(items, n);
    if (rc != CWT_OK) return rc;
    if (n == 0) return CWT_OK;
    if (!ws) return fail(CWT_E_INVALID, "ws is NULL");
    if (((uintptr_t)ws & 255) != 0) return fail(CWT_E_INVALID, "ws must be 256-byte aligned");
    hipStream_t s = (hipStream_t)stream;

    // Form: one launch pair per item (default), or the persistent class
    // kernels (CWT_BATCH_KERNELS=persistent), which alone need task lists.
    const char *km = std::getenv("CWT_BATCH_KERNELS");
    const bool persistent = km && std::strcmp(km, "persistent") == 0;

    // Tasks, grouped by workgroup-size class (and output mode for the
    // one-row-per-workgroup classes).
    std::map<std::tuple<int, int, int>, ClassInfo> by_class;
    for (int i = 0; i < n && persistent; ++i) {
        const cwt_plan &P = *items[i].plan;
        if (items[i].C == 0) continue;
        const int thr = class_threads(P.rp.threads, P.rp.maxv);
        const bool one_row = P.rp.maxv > 16;
        ClassInfo &c = by_class[{thr, P.rp.maxv, one_row ? (int)P.opts.out : -1}];
        c.threads = thr;
        c.maxv = P.rp.maxv;
        c.rows = one_row;
        c.mode = one_row ? (int)P.opts.out : -1;
        c.max_L = std::max(c.max_L, P.L);
        const int rows = (P.opts.out == CWT_OUT_BANDPOWER_F32) ? P.n_bands : P.F;
        const double per_row = row_cost(P);
        for (int pr = 0; pr < (int)((items[i].C + 1) / 2); ++pr) {
            c.fwd.push_back({i, pr, 0, 1});
            c.fwd_cost.push_back(per_row);
        }
        // band-power rows cost their number of frequencies
        auto freqs_in = [&](int r) {
            return (P.opts.out == CWT_OUT_BANDPOWER_F32) ? P.grp_off[r + 1] - P.grp_off[r] : 1;
        };
        for (int ch = 0; ch < (int)items[i].C; ++ch)
            for (int r = 0; r < rows;) {
                int nr = 0;
                double cost = 0;
                while (r + nr < rows &&
                       (nr == 0 || (!c.rows && cost + freqs_in(r + nr) * per_row <= kTaskCost))) {
                    cost += freqs_in(r + nr) * per_row;
                    ++nr;
                }
                c.main.push_back({i, ch, r, nr});
                c.main_cost.push_back(cost);
                c.total += cost;
                r += nr;
            }
    }
    std::vector<ClassInfo> classes;
    size_t n_fwd = 0, n_main = 0;
    for (auto &kv : by_class) {
        ClassInfo c = std::move(kv.second);
        auto sort_by_cost = [](std::vector<BatchTask> &t, const std::vector<double> &cost) {
            std::vector<size_t> ix(t.size());
            for (size_t k = 0; k < ix.size(); ++k) ix[k] = k;
            std::stable_sort(ix.begin(), ix.end(),
                             [&](size_t a, size_t b) { return cost[a] > cost[b]; });
            std::vector<BatchTask> out(t.size());
            for (size_t k = 0; k < ix.size(); ++k) out[k] = t[ix[k]];
            t.swap(out);
        };
        sort_by_cost(c.fwd, c.fwd_cost);
        sort_by_cost(c.main, c.main_cost);
        n_fwd += c.fwd.size();
        n_main += c.main.size();
        classes.push_back(std::move(c));
    }
    // The costliest class first: it is the critical path, and the classes
    // launched after it fill the CUs it leaves free.
    std::stable_sort(classes.begin(), classes.end(),
                     [](const ClassInfo &a, const ClassInfo &b) { return a.total > b.total; });
    if (classes.size() > 32) return fail(CWT_E_UNSUPPORTED, "too many task classes");
    for (const ClassInfo &c : classes)
        if (c.main.size() > (size_t)INT32_MAX || c.fwd.size() > (size_t)INT32_MAX)
            return fail(CWT_E_UNSUPPORTED, "too many tasks in one class");
    const Layout Lo = make_layout(items, n, n_fwd, n_main);
    if (ws_bytes < Lo.total)
        return fail(CWT_E_INVALID, "workspace too small: %zu < %zu bytes", ws_bytes, Lo.total);

    // Host tables.
    const size_t table_bytes = Lo.xh;  // everything before the spectra
    int dev = 0;
    (void)hipGetDevice(&dev);
    Staging &st = staging(dev);
    std::lock_guard<std::mutex> slk(st.mu);
    hipError_t e;
    if (st.done) {
        e = hipEventSynchronize(st.done);  // previous upload from the staging buffer
        if (e != hipSuccess) return hip_fail(e, "staging event");
    } else {
        e = hipEventCreateWithFlags(&st.done, hipEventDisableTiming);
        if (e != hipSuccess) return hip_fail(e, "staging event");
    }
    if (st.cap < table_bytes) {
        if (st.host) (void)hipHostFree(st.host);
        st.host = nullptr;
        st.cap = 0;
        if (hipHostMalloc(&st.host, table_bytes, hipHostMallocDefault) != hipSuccess)
            return fail(CWT_E_NOMEM, "pinned staging of %zu bytes failed", table_bytes);
        st.cap = table_bytes;
    }
    char *h = static_cast<char *>(st.host);
    std::memset(h, 0, Lo.fwd_items);
    char *dws = static_cast<char *>(ws);
    FwdParams *fi = reinterpret_cast<FwdParams *>(h + Lo.fwd_items);
    MainParams *mi = reinterpret_cast<MainParams *>(h + Lo.main_items);
    for (int i = 0; i < n; ++i) {
        const cwt_plan &P = *items[i].plan;
        float2 *Xh = reinterpret_cast<float2 *>(dws + Lo.xh_off[i]);
        FwdParams f{};
        f.x = items[i].x;
        f.C = (int)items[i].C;
        f.N = (int)P.n;
        f.x_stride = P.n;
        f.Xh = Xh;
        f.Lh = P.L / 2 + 1;
        f.tw = P.d_tw;
        f.rp = P.rp;
        fi[i] = f;
        MainParams m{};
        m.Xh = Xh;
        m.Lh = P.L / 2 + 1;
        m.H = P.d_H;
        m.Hc = P.d_Hc;
        m.band = P.d_band;
        m.tw = P.d_tw;
        m.out = items[i].out;
        m.out_mode = P.opts.out;
        m.N = (int)P.n;
        m.F = P.F;
        m.C = (int)items[i].C;
        m.n_rows = (P.opts.out == CWT_OUT_BANDPOWER_F32) ? P.n_bands : P.F;
        m.grp_freq = P.d_grp_freq;
        m.grp_off = P.d_grp_off;
        m.rp = P.rp;
        m.variant = 0;
        mi[i] = m;
    }
    BatchTask *ft = reinterpret_cast<BatchTask *>(h + Lo.fwd_tasks);
    BatchTask *mt = reinterpret_cast<BatchTask *>(h + Lo.main_tasks);
    std::vector<int64_t> shape;
    for (const ClassInfo &c : classes) {
        std::copy(c.fwd.begin(), c.fwd.end(), ft);
        ft += c.fwd.size();
        std::copy(c.main.begin(), c.main.end(), mt);
        mt += c.main.size();
        shape.insert(shape.end(), {c.threads, c.maxv, c.max_L, c.mode, (int64_t)c.fwd.size(),
                                   (int64_t)c.main.size()});
    }
    std::vector<ItemLaunch> its;
    if (!persistent) {
        for (int i = 0; i < n; ++i) {
            const cwt_plan &P = *items[i].plan;
            if (items[i].C == 0) continue;
            const int64_t rows = (P.opts.out == CWT_OUT_BANDPOWER_F32) ? P.n_bands : P.F;
            ItemLaunch it;
            it.item = i;
            it.fwd_blocks = (int)((items[i].C + 1) / 2);
            it.main_blocks = (int)(items[i].C * rows);
            it.threads = P.rp.threads;
            it.maxv = P.rp.maxv;
            it.mode = (int)P.opts.out;
            it.lds = generic_lds_bytes(P.L);
            it.cost = (double)items[i].C * rows * row_cost(P);
            if ((int64_t)it.main_blocks * it.threads >= ((int64_t)1 << 32))
                return fail(CWT_E_UNSUPPORTED,
                            "items[%d]: C x rows x threads reaches 2^32 work-items; split C", i);
            its.push_back(it);
        }
        std::stable_sort(its.begin(), its.end(),
                         [](const ItemLaunch &a, const ItemLaunch &b) { return a.cost > b.cost; });
        shape.push_back(-1);
        for (const ItemLaunch &it : its)
            shape.insert(shape.end(), {it.item, it.fwd_blocks, it.main_blocks, it.threads,
                                       it.maxv, it.mode, (int64_t)it.lds});
    }
    shape.insert(shape.end(), {(int64_t)Lo.total, n});
    // The items' plans may have been created on other streams: s waits for
    // any whose tables are still being written.
    {
        std::vector<const cwt_plan *> seen;
        for (int i = 0; i < n; ++i) {
            const cwt_plan *P = items[i].plan;
            if (std::find(seen.begin(), seen.end(), P) != seen.end()) continue;
            seen.push_back(P);
            rc = wait_plan_ready(*P, s);
            if (rc != CWT_OK) return rc;
        }
    }
    e = hipMemcpyAsync(dws + Lo.fwd_items, h + Lo.fwd_items, table_bytes - Lo.fwd_items,
                       hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return hip_fail(e, "batch table upload");
    e = hipEventRecord(st.done, s);
    if (e != hipSuccess) return hip_fail(e, "staging event record");

    // Launch: replay the cached graph, or capture one.
    const char *g = std::getenv("CWT_BATCH_GRAPH");
    const bool use_graph = !(g && g[0] == '0');
    auto enqueue = [&](hipStream_t q) {
        return persistent ? enqueue_kernels(classes, dws, Lo, q) : enqueue_items(its, dws, Lo, q);
    };
    if (!use_graph) return enqueue(s);
    GraphCache &gc = cache();
    std::lock_guard<std::mutex> glk(gc.mu);
    GraphKey key{ws, dev, shape};
    auto it = gc.execs.find(key);
    if (it == gc.execs.end()) {
        hipStream_t &cs = gc.cap_streams[dev];
        if (!cs) {
            e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
            if (e != hipSuccess) return hip_fail(e, "capture stream");
        }
        e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) return hip_fail(e, "hipStreamBeginCapture");
        rc = enqueue(cs);
        hipGraph_t graph = nullptr;
        e = hipStreamEndCapture(cs, &graph);
        if (rc != CWT_OK) {
            if (graph) (void)hipGraphDestroy(graph);
            return rc;
        }
        if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
        hipGraphExec_t exec = nullptr;
        e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (e != hipSuccess) return hip_fail(e, "hipGraphInstantiate");
        if (gc.execs.size() >= 32) {  // bounded cache
            (void)hipGraphExecDestroy(gc.execs.begin()->second);
            gc.execs.erase(gc.execs.begin());
        }
        it = gc.execs.emplace(key, exec).first;
    }
    e = hipGraphLaunch(it->second, s);
    if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
    return CWT_OK;
}
