// Autotuner of libcwt: times candidate kernel configurations of a plan and
// keeps the fastest; optional cache file keyed by (device, L, output, precision).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/cwt.h"
#include "cwt_internal.hpp"
#include "cwt_kernels.hpp"

using namespace cwtk;
using namespace cwtrt;

namespace {

std::mutex g_cache_mu;

struct Config {
    bool use_fixed;
    int variant;
    RadixPlan rp;
};

std::string arch_name(int dev)
{
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return "unknown";
    std::string a = prop.gcnArchName;
    const size_t colon = a.find(':');
    return colon == std::string::npos ? a : a.substr(0, colon);
}

// One cache line: arch L out precision kernel variant threads maxv n r0 r1 ...
std::string key_of(const std::string &arch, const cwt_plan &P)
{
    char buf[128];
    snprintf(buf, sizeof buf, "%s %d %d %d", arch.c_str(), P.L, P.opts.out, P.opts.precision);
    return buf;
}

}  // namespace

namespace cwtrt {

void apply_tuning_cache(cwt_plan &P)
{
    const char *path = std::getenv("CWT_AUTOTUNE_CACHE");
    if (!path || !*path || P.opts.precision != CWT_PREC_FP32) return;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return;
    const std::string key = key_of(arch_name(dev), P);
    std::lock_guard<std::mutex> lk(g_cache_mu);
    FILE *f = std::fopen(path, "r");
    if (!f) return;
    char line[512];
    Config best{};
    bool found = false;
    while (std::fgets(line, sizeof line, f)) {
        char arch[64];
        int L, out, prec, kernel, variant, threads, maxv, n;
        int off = 0;
        if (std::sscanf(line, "%63s %d %d %d %d %d %d %d %d%n", arch, &L, &out, &prec, &kernel,
                        &variant, &threads, &maxv, &n, &off) != 9)
            continue;
        char k2[128];
        snprintf(k2, sizeof k2, "%s %d %d %d", arch, L, out, prec);
        if (key != k2 || n < 1 || n > kMaxPasses) continue;
        RadixPlan rp{};
        rp.L = L;
        rp.n_pass = n;
        rp.threads = threads;
        rp.maxv = maxv;
        int prod = 1, ok = 1;
        const char *q = line + off;
        for (int i = 0; i < n && ok; ++i) {
            int r, used = 0;
            if (std::sscanf(q, "%d%n", &r, &used) != 1) ok = 0;
            q += used;
            // radices the passes implement
            if (ok && !(r == 1 || r == 2 || r == 3 || r == 4 || r == 5 || r == 6 || r == 7 ||
                        r == 8 || r == 9 || r == 10 || r == 12 || r == 14 || r == 15 || r == 16 ||
                        ((r == 20 || r == 21 || r == 24) && r <= maxv)))
                ok = 0;
            if (!ok) break;
            rp.radix[i] = r;
            prod *= r;
        }
        if (!ok || prod != L || threads < 64 || (maxv != 16 && maxv != 24 && maxv != 32) ||
            threads > generic_max_threads(maxv))
            continue;
        // every pass's butterflies fit the workgroup (as the planner requires)
        for (int i = 0; i < n && ok; ++i) {
            const int S = L / rp.radix[i];
            if ((S + threads - 1) / threads > std::max(1, maxv / rp.radix[i])) ok = 0;
        }
        if (!ok) continue;
        if (kernel == 1 && !reg_main_available(L)) continue;
        best = Config{kernel == 1, variant, rp};
        found = true;  // the last matching line wins
    }
    std::fclose(f);
    if (found) {
        P.use_fixed = best.use_fixed;
        P.variant = best.variant;
        if (!best.use_fixed) P.rp = best.rp;
    }
}

}  // namespace cwtrt

extern "C" int cwt_plan_autotune(cwt_plan *P, int64_t C, void *stream, cwt_tune_result *res)
{
    clear_error();
    if (!P) return fail(CWT_E_INVALID, "cwt_plan_autotune: plan is NULL");
    if (C < 1) return fail(CWT_E_INVALID, "C must be >= 1");
    if (res) std::memset(res, 0, sizeof *res);
    if (P->opts.precision != CWT_PREC_FP32) return CWT_OK;
    if (P->n_seg)
        return fail(CWT_E_UNSUPPORTED,
                    "segmented plans (padded length above %d) are not autotuned", CWT_MAX_LEN);
    hipStream_t s = (hipStream_t)stream;
    const int64_t Ct = C < 16 ? C : 16;
    const int64_t rows = (P->opts.out == CWT_OUT_BANDPOWER_F32) ? P->n_bands : P->F;
    const size_t out_b = (size_t)Ct * rows * P->n * ((P->opts.out == CWT_OUT_COMPLEX64) ? 8 : 4);
    const size_t x_b = (size_t)Ct * P->n * 4;
    const size_t ws_b = workspace_bytes(*P, Ct);
    void *x = nullptr, *out = nullptr, *ws = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    // temporaries from the plan's allocator, freed in stream order on s
    auto cleanup = [&]() {
        dev_free(P->mem, x, x_b, s);
        dev_free(P->mem, out, out_b, s);
        dev_free(P->mem, ws, ws_b, s);
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
    };
    int arc = dev_alloc(P->mem, &x, x_b, s, "autotune input");
    if (arc == CWT_OK) arc = dev_alloc(P->mem, &out, out_b, s, "autotune output");
    if (arc == CWT_OK) arc = dev_alloc(P->mem, &ws, ws_b, s, "autotune workspace");
    if (arc != CWT_OK) {
        cleanup();
        return arc;
    }
    hipError_t e = hipMemsetAsync(x, 0, x_b, s);
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    if (e != hipSuccess) {
        cleanup();
        return hip_fail(e, "autotune setup");
    }
    std::vector<Config> cands;
    const Config orig{P->use_fixed, P->variant, P->rp};
    cands.push_back(orig);
    if (reg_main_available(P->L)) {
        cands.push_back(Config{true, 0, P->rp});
        cands.push_back(Config{true, 1, P->rp});
    }
    std::vector<RadixPlan> rps;
    radix_candidates(P->L, rps);
    for (const RadixPlan &rp : rps) cands.push_back(Config{false, 0, rp});
    float best_ms = 1e30f, orig_ms = 0.f;
    size_t best_i = 0;
    int rc = CWT_OK;
    for (size_t i = 0; i < cands.size() && rc == CWT_OK; ++i) {
        P->use_fixed = cands[i].use_fixed;
        P->variant = cands[i].variant;
        P->rp = cands[i].rp;
        float t_min = 1e30f;
        for (int rep = 0; rep < 4 && rc == CWT_OK; ++rep) {
            e = hipEventRecord(e0, s);
            if (e == hipSuccess) rc = enqueue_execute(*P, (const float *)x, Ct, P->n, out, ws, s);
            if (rc == CWT_OK && e == hipSuccess) e = hipEventRecord(e1, s);
            if (rc == CWT_OK && e == hipSuccess) e = hipEventSynchronize(e1);
            float ms = 0.f;
            if (rc == CWT_OK && e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
            if (e != hipSuccess && rc == CWT_OK) rc = hip_fail(e, "autotune timing");
            if (rep > 0 && ms < t_min) t_min = ms;  // the first run warms up
        }
        if (i == 0) orig_ms = t_min;
        if (t_min < best_ms) {
            best_ms = t_min;
            best_i = i;
        }
    }
    cleanup();
    const Config &b = (rc == CWT_OK) ? cands[best_i] : orig;
    P->use_fixed = b.use_fixed;
    P->variant = b.variant;
    P->rp = b.rp;
    if (rc != CWT_OK) return rc;
    if (res) {
        res->n_candidates = (int)cands.size();
        res->kernel = b.use_fixed ? 1 : 0;
        res->variant = b.variant;
        res->threads = b.use_fixed ? reg_row_threads(P->L) : b.rp.threads;
        res->n_passes = b.rp.n_pass;
        for (int i = 0; i < b.rp.n_pass && i < 16; ++i) res->radix[i] = b.rp.radix[i];
        res->best_ms = best_ms;
        res->default_ms = orig_ms;
    }
    const char *path = std::getenv("CWT_AUTOTUNE_CACHE");
    if (path && *path) {
        int dev = 0;
        (void)hipGetDevice(&dev);
        std::lock_guard<std::mutex> lk(g_cache_mu);
        FILE *f = std::fopen(path, "a");
        if (f) {
            std::fprintf(f, "%s %d %d %d %d %d", key_of(arch_name(dev), *P).c_str(),
                         b.use_fixed ? 1 : 0, b.variant, b.rp.threads, b.rp.maxv, b.rp.n_pass);
            for (int i = 0; i < b.rp.n_pass; ++i) std::fprintf(f, " %d", b.rp.radix[i]);
            std::fprintf(f, "\n");
            std::fclose(f);
        }
    }
    return CWT_OK;
}
