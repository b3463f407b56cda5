// C ABI of libfhw (declared in include/fhw.h): context, planner and the
// entry points of the hot path.  Host logic only; every arithmetic step of
// the method runs in the kernels of geometry/assemble/lu/solve/field/synth.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <cstdio>
#include <new>
#include <mutex>
#include <set>

#include "fhw_internal.h"

namespace {

struct zd { double re, im; };   // complex128 element (host view)

struct chunk_t {
    int32_t j0 = 0, count = 0, maxN = 0;
    // device metadata (inside ctx->meta)
    int32_t* d_N = nullptr;
    int64_t *d_aoff = nullptr, *d_pivoff = nullptr, *d_linvoff = nullptr, *d_voff = nullptr;
    fhw_assemble_item* d_items = nullptr;
    int64_t* d_asm_prefix = nullptr;
    int32_t* d_lu_prefix = nullptr;
    int64_t asm_blocks = 0;
    fhw_lu_sched sched;
    int64_t psi_base = 0;       // element offset of psi_j0
    int64_t vec_elems = 0;      // sum N over the chunk
    hipGraphExec_t lu_graph = nullptr;   // the factorization's launches, captured once per plan
};

struct plan_ext {
    std::vector<chunk_t> chunks;
    fhw_field_item* d_field_items = nullptr;
    fhw_field_item* d_lf_items = nullptr;   // graded nodes 1 .. lf_M lf_N (the last is omega_c)
};

// per-context plan extension; contexts may live on different host threads
// (one per stream), so lookups go through one lock (map nodes do not move)
std::mutex g_plans_mu;
std::map<const fhw_ctx*, plan_ext> g_plans;

plan_ext& plan_of(const fhw_ctx* c) {
    std::lock_guard<std::mutex> lk(g_plans_mu);
    return g_plans[c];
}

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

int64_t linv_elems(int32_t N) { return (int64_t)((N + FHW_LU_NB - 1) / FHW_LU_NB) * FHW_LU_NB * FHW_LU_NB; }

size_t freq_bytes(int32_t N, int precision) {
    size_t NN = (size_t)N * N;
    size_t b = NN * 16;                                       // FP64 matrix
    if (precision == FHW_FP32_REFINE) b += NN * 8;             // FP32 factors
    b += (size_t)linv_elems(N) * (precision == FHW_FP64 ? 16 : 8);
    b += (size_t)N * 4;                                       // pivots
    b += (size_t)N * 16 * 2 * FHW_INC_GROUP;                  // g, r per incidence of a group
    b += 256;                                                 // metadata
    return b;
}

void curve_eval_host(const fhw_host_curve& cv, double s, double& x1, double& x2, double& d1, double& d2) {
    x1 = x2 = d1 = d2 = 0.0;
    for (int d = 0; d <= cv.degree; ++d) {
        double cs = cos(d * s), sn = sin(d * s);
        x1 += cv.cx[d] * cs + cv.sx[d] * sn;
        x2 += cv.cy[d] * cs + cv.sy[d] * sn;
        d1 += d * (cv.sx[d] * cs - cv.cx[d] * sn);
        d2 += d * (cv.sy[d] * cs - cv.cy[d] * sn);
    }
}

void free_plan(fhw_ctx* c) {
    {
        std::lock_guard<std::mutex> lk(g_plans_mu);
        auto it = g_plans.find(c);
        if (it != g_plans.end()) {
            for (auto& ch : it->second.chunks)
                if (ch.lu_graph) (void)hipGraphExecDestroy(ch.lu_graph);
            g_plans.erase(it);
        }
    }
    // geometry, curve coefficients and the small per-plan buffers stay for
    // the next plan (fhw_destroy frees them): freeing device memory
    // synchronizes the device, which would stall other streams' work
    c->geoms.clear();
    c->curves.clear();
    c->planned = false;
    c->factors_resident = false;
}

void free_caches(fhw_ctx* c) {
    for (auto& kv : c->geo_cache) {
        (void)hipFree(kv.second.e.geom);
        (void)hipFree(kv.second.e.R);
        (void)hipFree(kv.second.e.logtab);
    }
    c->geo_cache.clear();
    c->geo_cache_bytes = 0;
    for (auto& kv : c->curve_cache) (void)hipFree(kv.second.d);
    c->curve_cache.clear();
    void* ptrs[] = {c->meta, c->d_status, c->d_norms, c->d_done, c->d_sweeps, c->d_rpart, c->d_rcount};
    for (void* p : ptrs)
        if (p) (void)hipFree(p);
    c->meta = nullptr; c->d_status = nullptr; c->d_norms = nullptr; c->d_done = nullptr; c->d_sweeps = nullptr;
    c->d_rpart = nullptr; c->d_rcount = nullptr;
    for (size_t& k : c->small_cap) k = 0;
}

// A small per-plan buffer (index k of small_cap) of at least `bytes`, kept
// across plans and reallocated only when a plan outgrows it; zero-filled
// (on the context's stream) when `zero` and newly allocated.
int grow_small(fhw_ctx* c, void** p, int k, size_t bytes, bool zero = false) {
    bytes = std::max<size_t>(bytes, 256);
    if (*p && c->small_cap[k] >= bytes) return FHW_OK;
    if (*p) {
        FHW_HIP(c, hipStreamSynchronize(c->stream));
        (void)hipFree(*p);
        *p = nullptr;
    }
    c->small_cap[k] = 0;
    const size_t nb = align_up(bytes + bytes / 2, 4096);
    FHW_HIP(c, hipMalloc(p, nb));
    c->small_cap[k] = nb;
    if (zero) FHW_HIP(c, hipMemsetAsync(*p, 0, nb, c->stream));
    return FHW_OK;
}

// device-to-host copy on the context's stream, then wait for it
int copy_d2h(fhw_ctx* c, void* dst, const void* src, size_t bytes) {
    FHW_HIP(c, hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, c->stream));
    FHW_HIP(c, hipStreamSynchronize(c->stream));
    return FHW_OK;
}

// Several device-to-host copies through the context's pinned staging buffer
// with one wait: the copies are queued on the stream, then the host waits
// once and unpacks (each pageable copy would wait on its own).
struct d2h_item {
    void* dst;
    const void* src;
    size_t bytes;
};
int readback(fhw_ctx* c, std::initializer_list<d2h_item> items) {
    size_t total = 0;
    for (const d2h_item& it : items) total += align_up(it.bytes, 64);
    if (total > c->h_stage_bytes) {
        FHW_HIP(c, hipStreamSynchronize(c->stream));
        if (c->h_stage) (void)hipHostFree(c->h_stage);
        c->h_stage = nullptr;
        c->h_stage_bytes = 0;
        const size_t nb = align_up(total + total / 2, 4096);
        FHW_HIP(c, hipHostMalloc(&c->h_stage, nb, hipHostMallocDefault));
        c->h_stage_bytes = nb;
    }
    size_t o = 0;
    for (const d2h_item& it : items) {
        if (it.bytes) FHW_HIP(c, hipMemcpyAsync((char*)c->h_stage + o, it.src, it.bytes, hipMemcpyDeviceToHost, c->stream));
        o += align_up(it.bytes, 64);
    }
    FHW_HIP(c, hipStreamSynchronize(c->stream));
    o = 0;
    for (const d2h_item& it : items) {
        if (it.bytes) memcpy(it.dst, (char*)c->h_stage + o, it.bytes);
        o += align_up(it.bytes, 64);
    }
    return FHW_OK;
}

uint64_t curve_fingerprint(const fhw_host_curve& cv) {
    uint64_t h = 1469598103934665603ull;
    auto mix = [&](const void* p, size_t n) {
        const unsigned char* b = (const unsigned char*)p;
        for (size_t i = 0; i < n; ++i) { h ^= b[i]; h *= 1099511628211ull; }
    };
    mix(&cv.degree, sizeof(cv.degree));
    for (const std::vector<double>* v : {&cv.cx, &cv.sx, &cv.cy, &cv.sy}) mix(v->data(), v->size() * sizeof(double));
    return h;
}

void** workspace_slot(fhw_ctx* c, int k) {
    void** slots[6] = {&c->A64, &c->A32, &c->linv, (void**)&c->piv, &c->x, &c->r};
    return slots[k];
}

void free_workspace(fhw_ctx* c) {
    for (int k = 0; k < 6; ++k) {
        void** p = workspace_slot(c, k);
        if (*p) (void)hipFree(*p);
        *p = nullptr;
        c->ws_cap[k] = 0;
    }
}

// The six large work buffers of a plan (bytes in need[]), reusing those of the
// previous plan that are big enough: a stream of plans (one per request, say)
// then allocates only when it outgrows them.  If what would be kept plus what
// must grow exceeds the budget, everything is released and allocated afresh.
int ensure_workspace(fhw_ctx* c, const size_t need[6]) {
    size_t keep = 0, grow = 0;
    for (int k = 0; k < 6; ++k) {
        if (need[k] <= c->ws_cap[k]) keep += c->ws_cap[k];
        else grow += need[k];
    }
    if (grow > 0 && keep + grow > c->budget) free_workspace(c);
    for (int k = 0; k < 6; ++k) {
        if (need[k] == 0 || need[k] <= c->ws_cap[k]) continue;
        void** p = workspace_slot(c, k);
        if (*p) (void)hipFree(*p);
        *p = nullptr;
        c->ws_cap[k] = 0;
        FHW_HIP(c, hipMalloc(p, need[k]));
        c->ws_cap[k] = need[k];
    }
    return FHW_OK;
}

int lds_limit(fhw_ctx* c) {
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, c->device) != hipSuccess) v = 65536;
    return v;
}

}  // namespace

// The status words of fhw_solve_range_noalloc live in this fixed device array,
// one per GPU the library runs on, instead of memory the library allocates.
// On the host, the array's name is only a stand-in for the device symbol:
// host code never passes it to a kernel or a copy.  Its device address on each
// device is looked up once, at the first fhw_create on that device (with the
// device current), with hipGetSymbolAddress; only that address is used.
static __device__ __align__(256) unsigned char noalloc_scratch[FHW_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int kNoallocDevices = 64;
std::mutex g_noalloc_mu;
void* g_noalloc_addr[kNoallocDevices] = {};

// device address of noalloc_scratch on `device` (the current device)
void* noalloc_address(int device, std::string* err) {
    if (device < 0 || device >= kNoallocDevices) {
        *err = "allocation-free solves: device index out of range";
        return nullptr;
    }
    std::lock_guard<std::mutex> lk(g_noalloc_mu);
    if (!g_noalloc_addr[device]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(noalloc_scratch));
        if (e != hipSuccess || !p) {
            *err = std::string("allocation-free solves: hipGetSymbolAddress failed: ") + hipGetErrorString(e);
            return nullptr;
        }
        g_noalloc_addr[device] = p;
    }
    return g_noalloc_addr[device];
}

// turns the stage timers off for one call (their events would be created on demand)
struct prof_pause {
    fhw_prof& p;
    bool was;
    explicit prof_pause(fhw_prof& q) : p(q), was(q.on) { p.on = false; }
    ~prof_pause() { p.on = was; }
};
}  // namespace

hipEvent_t fhw_prof::take() {
    if (!pool.empty()) {
        hipEvent_t e = pool.back();
        pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

void fhw_prof::begin(int stage, hipStream_t s) {
    open_stage = stage;
    open_a = take();
    if (open_a) (void)hipEventRecord(open_a, s);
}

void fhw_prof::end(hipStream_t s) {
    if (open_stage < 0 || !open_a) return;
    hipEvent_t b = take();
    if (!b) return;
    (void)hipEventRecord(b, s);
    recs.push_back(rec{open_stage, open_a, b});
    open_stage = -1;
    open_a = nullptr;
}

int fhw_fail(fhw_ctx* ctx, int code, const std::string& msg) {
    if (ctx) ctx->err = msg;
    return code;
}

int fhw_hip_check(fhw_ctx* ctx, hipError_t e, const char* what) {
    if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation)
        return fhw_fail(ctx, FHW_E_NOMEM, std::string("device memory exhausted: ") + what);
    return fhw_fail(ctx, FHW_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

int fhw_ensure_scratch(fhw_ctx* ctx, size_t bytes) {
    if (bytes <= ctx->scratch_bytes) return FHW_OK;
    FHW_HIP(ctx, hipStreamSynchronize(ctx->stream));
    if (ctx->scratch) (void)hipFree(ctx->scratch);
    ctx->scratch = nullptr;
    ctx->scratch_bytes = 0;
    size_t nb = align_up(bytes, 1 << 20);
    FHW_HIP(ctx, hipMalloc(&ctx->scratch, nb));
    ctx->scratch_bytes = nb;
    return FHW_OK;
}

#define STAGE(c, st, call)                                               \
    do {                                                                 \
        prof_begin(&(c)->prof, (st), (c)->stream);                       \
        hipError_t _e = (call);                                          \
        prof_end(&(c)->prof, (c)->stream);                               \
        if (_e != hipSuccess) return fhw_hip_check((c), _e, #call);      \
    } while (0)

extern "C" {

int fhw_version(void) { return 1; }

int fhw_profile(fhw_ctx* c, int32_t enable) {
    if (!c) return FHW_E_INVALID;
    FHW_HIP(c, hipStreamSynchronize(c->stream));
    for (auto& r : c->prof.recs) {
        c->prof.pool.push_back(r.a);
        c->prof.pool.push_back(r.b);
    }
    c->prof.recs.clear();
    c->prof.on = enable != 0;
    return FHW_OK;
}

int fhw_profile_read(fhw_ctx* c, double* ms, int64_t* launches) {
    if (!c || !ms || !launches) return FHW_E_INVALID;
    FHW_HIP(c, hipStreamSynchronize(c->stream));
    for (int q = 0; q < FHW_N_STAGES; ++q) {
        ms[q] = 0.0;
        launches[q] = 0;
    }
    for (auto& r : c->prof.recs) {
        float t = 0.0f;
        FHW_HIP(c, hipEventElapsedTime(&t, r.a, r.b));
        if (r.stage >= 0 && r.stage < FHW_N_STAGES) {
            ms[r.stage] += (double)t;
            launches[r.stage] += 1;
        }
        c->prof.pool.push_back(r.a);
        c->prof.pool.push_back(r.b);
    }
    c->prof.recs.clear();
    return FHW_OK;
}

int fhw_create(fhw_ctx** out, void* hip_stream, size_t hbm_budget_bytes) {
    if (!out) return FHW_E_INVALID;
    *out = nullptr;
    fhw_ctx* c = new (std::nothrow) fhw_ctx();
    if (!c) return FHW_E_NOMEM;
    c->stream = (hipStream_t)hip_stream;
    if (hipGetDevice(&c->device) != hipSuccess) {
        delete c;
        return FHW_E_HIP;
    }
    size_t fr = 0, tot = 0;
    if (hipMemGetInfo(&fr, &tot) != hipSuccess) {
        delete c;
        return FHW_E_HIP;
    }
    c->budget = hbm_budget_bytes ? hbm_budget_bytes : (size_t)(0.9 * (double)fr);
    if (hipMalloc((void**)&c->d_pending, sizeof(int32_t)) != hipSuccess ||
        hipHostMalloc((void**)&c->h_pending, sizeof(int32_t), hipHostMallocDefault) != hipSuccess) {
        if (c->d_pending) (void)hipFree(c->d_pending);
        delete c;
        return FHW_E_NOMEM;
    }
    // the other calls work without it: a failed lookup fails only
    // fhw_solve_range_noalloc, with this message
    c->noalloc = noalloc_address(c->device, &c->noalloc_err);
    *out = c;
    return FHW_OK;
}

int fhw_destroy(fhw_ctx* c) {
    if (!c) return FHW_OK;
    (void)hipStreamSynchronize(c->stream);
    free_plan(c);
    free_workspace(c);
    free_caches(c);
    if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
    if (c->scratch) (void)hipFree(c->scratch);
    if (c->d_pending) (void)hipFree(c->d_pending);
    if (c->h_pending) (void)hipHostFree(c->h_pending);
    if (c->h_stage) (void)hipHostFree(c->h_stage);
    for (auto& r : c->prof.recs) {
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
    }
    for (hipEvent_t e : c->prof.pool) (void)hipEventDestroy(e);
    delete c;
    return FHW_OK;
}

const char* fhw_last_error(const fhw_ctx* c) { return c ? c->err.c_str() : "null context"; }

// Plan n_curves scatterers with one problem: system s = curve * F + j; or,
// with sys != NULL, the n_sys systems listed there (any curve, frequency, N).
static int plan_impl(fhw_ctx* c, const fhw_curve* curves, int32_t n_curves, const fhw_problem* p, int32_t* N_out,
                     int64_t* psi_off_out, const fhw_system* sys = nullptr, int32_t n_sys = 0) {
    if (!c) return FHW_E_INVALID;
    if (!curves || n_curves < 1 || !p) return fhw_fail(c, FHW_E_INVALID, "plan: missing curve/problem");
    if (sys) {
        if (n_sys < 1) return fhw_fail(c, FHW_E_INVALID, "plan_systems: need at least one system");
        for (int s = 0; s < n_sys; ++s) {
            if (sys[s].curve < 0 || sys[s].curve >= n_curves)
                return fhw_fail(c, FHW_E_INVALID, "plan_systems: curve index out of range");
            if (!(sys[s].omega > 0) || !isfinite(sys[s].omega))
                return fhw_fail(c, FHW_E_INVALID, "plan_systems: need a finite omega > 0");
            if (sys[s].N < 4 || (sys[s].N & 1) || sys[s].N > 4096)
                return fhw_fail(c, FHW_E_INVALID, "plan_systems: N must be even, 4 <= N <= 4096");
        }
    }
    for (int k = 0; k < n_curves; ++k) {
        const fhw_curve* curve = curves + k;
        if (curve->degree < 1 || !curve->cx || !curve->sx || !curve->cy || !curve->sy)
            return fhw_fail(c, FHW_E_INVALID, "plan: missing curve coefficients");
    }
    if (!(p->c > 0) || !isfinite(p->c)) return fhw_fail(c, FHW_E_INVALID, "plan: need c > 0");
    if (!sys && (!(p->W > 0) || p->F < 1 || !isfinite(p->W)))
        return fhw_fail(c, FHW_E_INVALID, "plan: need W > 0, F >= 1");
    if (p->precision != FHW_FP64 && p->precision != FHW_FP32_REFINE)
        return fhw_fail(c, FHW_E_INVALID, "plan: unknown precision");
    if (!isfinite(p->direction[0]) || !isfinite(p->direction[1]))
        return fhw_fail(c, FHW_E_INVALID, "plan: direction not finite");
    if (p->j_first < 0) return fhw_fail(c, FHW_E_INVALID, "plan: j_first must be >= 0");
    if (p->formulation != FHW_FORM_DIRECT && p->formulation != FHW_FORM_COMBINED)
        return fhw_fail(c, FHW_E_INVALID, "plan: unknown formulation");
    if (p->formulation == FHW_FORM_COMBINED && (sys || n_curves != 1 || p->j_first != 0 || p->N_fixed <= 0))
        return fhw_fail(c, FHW_E_INVALID, "plan: the combined formulation needs one curve on the DFT grid with "
                                          "a fixed N");
    const bool lowfreq = p->lf_M > 0;
    if (p->lf_M < 0) return fhw_fail(c, FHW_E_INVALID, "plan: lf_M must be >= 0");
    if (lowfreq) {
        if (sys || n_curves != 1 || p->j_first != 0)
            return fhw_fail(c, FHW_E_INVALID, "plan: the graded low-frequency nodes need a one-curve plan on the DFT grid");
        if (p->lf_N < 1 || p->lf_N > 32 || !(p->lf_q > 0) || !isfinite(p->lf_q) || p->lf_jc < 1 ||
            p->F - p->lf_jc + 1 < 20 || (int64_t)p->lf_M * p->lf_N > 4096)
            return fhw_fail(c, FHW_E_INVALID, "plan: need 1 <= lf_N <= 32, lf_q > 0, lf_jc >= 1, F - lf_jc + 1 >= 20, "
                                              "lf_M lf_N <= 4096");
    }
    (void)hipStreamSynchronize(c->stream);
    free_plan(c);
    c->prob = *p;
    c->curves.resize(n_curves);
    for (int k = 0; k < n_curves; ++k) {
        const fhw_curve* curve = curves + k;
        fhw_host_curve& cv = c->curves[k];
        cv.degree = curve->degree;
        const int D1 = curve->degree + 1;
        cv.cx.assign(curve->cx, curve->cx + D1);
        cv.sx.assign(curve->sx, curve->sx + D1);
        cv.cy.assign(curve->cy, curve->cy + D1);
        cv.sy.assign(curve->sy, curve->sy + D1);
        for (int d = 0; d < D1; ++d)
            if (!isfinite(cv.cx[d]) || !isfinite(cv.sx[d]) || !isfinite(cv.cy[d]) || !isfinite(cv.sy[d]))
                return fhw_fail(c, FHW_E_INVALID, "plan: curve coefficients not finite");
        // curve length (trapezoidal rule on the periodic speed), orientation check
        const int nq = 4096;
        double L = 0.0, area = 0.0, minsp = 1e300;
        for (int q = 0; q < nq; ++q) {
            double s = 2.0 * M_PI * q / nq, x1, x2, d1, d2;
            curve_eval_host(cv, s, x1, x2, d1, d2);
            double sp = sqrt(d1 * d1 + d2 * d2);
            L += sp;
            area += x1 * d2 - x2 * d1;
            minsp = std::min(minsp, sp);
        }
        L *= 2.0 * M_PI / nq;
        area *= 0.5 * 2.0 * M_PI / nq;
        if (!(minsp > 0.0) || !(area > 0.0))
            return fhw_fail(c, FHW_E_INVALID, "plan: curve must be counter-clockwise, non-degenerate");
        cv.length = L;
    }
    // frequencies, sizes, coupling per system
    const int F = sys ? n_sys : p->F;
    const double dw = p->W / (double)F;
    // graded low-frequency nodes (eq. gradedmesh): Clenshaw-Curtis points of
    // each [mu_j, mu_{j+1}], ascending, shared ends once
    c->lf_extra = 0;
    c->lf_mu.clear();
    c->lf_nodes.clear();
    if (lowfreq) {
        const int M = p->lf_M, Nn = p->lf_N;
        c->lf_omega_c = dw * (double)p->lf_jc;
        c->lf_mu.resize(M + 1);
        for (int j = 0; j <= M; ++j) c->lf_mu[j] = c->lf_omega_c * pow((double)j / (double)M, p->lf_q);
        for (int j = 0; j < M; ++j) {
            const double a = c->lf_mu[j], b = c->lf_mu[j + 1];
            for (int i = 0; i < Nn; ++i)   // Clenshaw-Curtis point Nn - i: cos(pi (Nn - i) / Nn) ascends with i
                c->lf_nodes.push_back(0.5 * (a + b) + 0.5 * (b - a) * cos(M_PI * (double)(Nn - i) / (double)Nn));
        }
        c->lf_nodes.push_back(c->lf_omega_c);
        c->lf_nodes[0] = 0.0;
        for (size_t g = 1; g < c->lf_nodes.size(); ++g)
            if (!(c->lf_nodes[g] > c->lf_nodes[g - 1]))
                return fhw_fail(c, FHW_E_INVALID, "plan: graded nodes not increasing (lf_q too large for lf_M)");
        c->lf_extra = M * Nn - 1;
    }
    const int S = sys ? n_sys : n_curves * F + c->lf_extra;
    c->kappa.resize(S);
    c->eta.resize(S);
    c->Ns.resize(S);
    c->sys_curve.resize(S);
    c->system_plan = sys != nullptr;
    for (int s = 0; sys && s < S; ++s) {
        c->kappa[s] = sys[s].omega / p->c;
        c->eta[s] = std::max(c->kappa[s], 1.0);
        c->Ns[s] = sys[s].N;
        c->sys_curve[s] = sys[s].curve;
    }
    for (int k = 0; !sys && k < n_curves; ++k)
        for (int j = 0; j < F; ++j) {
            const int sy = k * F + j;
            c->sys_curve[sy] = k;
            double om = dw * (double)(p->j_first + j + 1);
            c->kappa[sy] = om / p->c;
            c->eta[sy] = std::max(c->kappa[sy], 1.0);
            int N;
            if (p->N_fixed > 0) {
                N = p->N_fixed;
            } else {
                if (p->n_mult < 1 || p->n_min < 2 || p->n_cap < p->n_min || !(p->ppw > 0))
                    return fhw_fail(c, FHW_E_INVALID, "plan: bad N rule");
                double raw = p->ppw * c->curves[k].length * c->kappa[sy] / (2.0 * M_PI);
                double m = ceil(raw / (double)p->n_mult) * (double)p->n_mult;
                N = (int)std::min<double>(std::max<double>(m, p->n_min), p->n_cap);
            }
            if (N < 4 || (N & 1) || N > 4096)
                return fhw_fail(c, FHW_E_INVALID, "plan: N must be even, 4 <= N <= 4096");
            c->Ns[sy] = N;
        }
    for (int e = 0; e < c->lf_extra; ++e) {
        // graded node e + 1 (ascending), on curve 0, N by the same rule
        const int sy = F + e;
        c->sys_curve[sy] = 0;
        c->kappa[sy] = c->lf_nodes[e + 1] / p->c;
        c->eta[sy] = std::max(c->kappa[sy], 1.0);
        int N;
        if (p->N_fixed > 0) {
            N = p->N_fixed;
        } else {
            if (p->n_mult < 1 || p->n_min < 2 || p->n_cap < p->n_min || !(p->ppw > 0))
                return fhw_fail(c, FHW_E_INVALID, "plan: bad N rule");
            double raw = p->ppw * c->curves[0].length * c->kappa[sy] / (2.0 * M_PI);
            double m = ceil(raw / (double)p->n_mult) * (double)p->n_mult;
            N = (int)std::min<double>(std::max<double>(m, p->n_min), p->n_cap);
        }
        if (N < 4 || (N & 1) || N > 4096) return fhw_fail(c, FHW_E_INVALID, "plan: N must be even, 4 <= N <= 4096");
        c->Ns[sy] = N;
    }
    c->psi_off.assign(S + 1, 0);
    for (int j = 0; j < S; ++j) c->psi_off[j + 1] = c->psi_off[j] + c->Ns[j];
    int maxN = *std::max_element(c->Ns.begin(), c->Ns.end());
    if ((size_t)maxN * 16 + FHW_SOLVE_STATIC_LDS > (size_t)lds_limit(c))
        return fhw_fail(c, FHW_E_INVALID, "plan: N too large for the LDS-resident solve vector");

    // curve coefficients on device, geometry + Kress tables per (curve, distinct N)
    // (kept across plans: a curve's coefficients and its nodes and Kress
    // tables at each N are computed once per context)
    size_t geo = 0;
    if (c->geo_cache_bytes > ((size_t)1 << 30)) {
        FHW_HIP(c, hipStreamSynchronize(c->stream));
        for (auto& kv : c->geo_cache) {
            (void)hipFree(kv.second.e.geom);
            (void)hipFree(kv.second.e.R);
            (void)hipFree(kv.second.e.logtab);
        }
        c->geo_cache.clear();
        c->geo_cache_bytes = 0;
    }
    for (int k = 0; k < n_curves; ++k) {
        fhw_host_curve& cv = c->curves[k];
        const int D1 = cv.degree + 1;
        std::vector<double> hc(4 * D1);
        for (int d = 0; d < D1; ++d) {
            hc[d] = cv.cx[d]; hc[D1 + d] = cv.sx[d]; hc[2 * D1 + d] = cv.cy[d]; hc[3 * D1 + d] = cv.sy[d];
        }
        const uint64_t fp = curve_fingerprint(cv);
        auto cit = c->curve_cache.find(fp);
        if (cit == c->curve_cache.end() || cit->second.coef != hc) {
            if (cit != c->curve_cache.end()) {
                // a different curve with the same fingerprint: drop the old entry
                FHW_HIP(c, hipStreamSynchronize(c->stream));
                (void)hipFree(cit->second.d);
                c->curve_cache.erase(cit);
            }
            fhw_curve_cache_entry ce;
            ce.coef = hc;
            FHW_HIP(c, hipMalloc((void**)&ce.d, sizeof(double) * 4 * D1));
            FHW_HIP(c, hipMemcpyAsync(ce.d, ce.coef.data(), sizeof(double) * 4 * D1, hipMemcpyHostToDevice,
                                      c->stream));
            FHW_HIP(c, hipStreamSynchronize(c->stream));
            cit = c->curve_cache.emplace(fp, std::move(ce)).first;
        }
        cv.d_curve = cit->second.d;
        cv.fingerprint = fp;
        std::set<int32_t> distinct;
        for (int s = 0; s < S; ++s)
            if (c->sys_curve[s] == k) distinct.insert(c->Ns[s]);
        for (int32_t N : distinct) {
            auto git = c->geo_cache.find({fp, N});
            if (git == c->geo_cache.end()) {
                fhw_geo_cache_entry ge{};
                fhw_geom_entry& e = ge.e;
                e.N = N;
                FHW_HIP(c, hipMalloc(&e.geom, sizeof(double) * 9 * N));
                FHW_HIP(c, hipMalloc(&e.R, sizeof(double) * N));
                FHW_HIP(c, hipMalloc(&e.logtab, sizeof(double) * N));
                STAGE(c, FHW_STAGE_GEOMETRY, launch_geometry(c->stream, cv.d_curve, cv.degree, N, e.geom));
                STAGE(c, FHW_STAGE_KRESS, launch_kress(c->stream, N, e.R, e.logtab));
                git = c->geo_cache.emplace(std::make_pair(fp, N), ge).first;
                c->geo_cache_bytes += (size_t)N * 11 * 8;
            }
            c->geoms[fhw_geom_key(k, N)] = git->second.e;
            geo += (size_t)N * 11 * 8;
        }
    }

    // chunks over frequencies within the HBM budget
    const int prec = p->precision;
    plan_ext& px = plan_of(c);
    px.chunks.clear();
    {
        size_t avail = c->budget > geo ? c->budget - geo : 0;
        int j = 0;
        while (j < S) {
            chunk_t ch;
            ch.j0 = j;
            size_t used = 0;
            while (j < S) {
                size_t fb = freq_bytes(c->Ns[j], prec);
                if (ch.count > 0 && used + fb > avail) break;
                if (ch.count == 0 && fb > avail)
                    return fhw_fail(c, FHW_E_NOMEM, "plan: one frequency does not fit the HBM budget");
                used += fb;
                ch.count++;
                j++;
            }
            px.chunks.push_back(ch);
        }
    }
    // workspace sized for the largest chunk
    size_t wsA64 = 0, wsA32 = 0, wsL = 0, wsP = 0, wsV = 0;
    int maxcount = 0;
    for (auto& ch : px.chunks) {
        size_t a = 0, l = 0, pv = 0, v = 0;
        ch.maxN = 0;
        for (int q = 0; q < ch.count; ++q) {
            int N = c->Ns[ch.j0 + q];
            a += (size_t)N * N;
            l += linv_elems(N);
            pv += N;
            v += N;
            ch.maxN = std::max(ch.maxN, N);
        }
        ch.psi_base = c->psi_off[ch.j0];
        ch.vec_elems = (int64_t)v;
        wsA64 = std::max(wsA64, a);
        wsL = std::max(wsL, l);
        wsP = std::max(wsP, pv);
        wsV = std::max(wsV, v);
        maxcount = std::max(maxcount, ch.count);
    }
    wsA32 = prec == FHW_FP32_REFINE ? wsA64 : 0;
    c->chunk = maxcount;
    {
        // A64, A32 (FP32 path), linv, piv, x (g), r (residual / correction)
        const size_t need[6] = {wsA64 * 16, wsA32 * 8, wsL * (prec == FHW_FP64 ? 16 : 8), wsP * 4,
                                wsV * 16 * FHW_INC_GROUP, wsV * 16 * FHW_INC_GROUP};
        int rc = ensure_workspace(c, need);
        if (rc) return rc;
    }
    {
        int rc = grow_small(c, (void**)&c->d_status, 0, sizeof(int32_t) * 4);
        if (!rc) rc = grow_small(c, (void**)&c->d_norms, 1, sizeof(double) * 2 * S);
        if (!rc) rc = grow_small(c, (void**)&c->d_done, 2, sizeof(int32_t) * S);
        if (!rc) rc = grow_small(c, (void**)&c->d_sweeps, 3, sizeof(int32_t) * S);
        // residual: per-block partial norms and per-matrix block counters (zero;
        // every residual launch leaves them zero)
        c->ws_vec = (int64_t)wsV;
        c->rpart_stride = 2 * (int64_t)maxcount * ((maxN + 63) / 64);
        if (!rc) rc = grow_small(c, (void**)&c->d_rpart, 4, sizeof(double) * (size_t)c->rpart_stride * FHW_INC_GROUP);
        if (!rc) rc = grow_small(c, (void**)&c->d_rcount, 5, sizeof(int32_t) * (size_t)maxcount * FHW_INC_GROUP, true);
        if (rc) return rc;
    }
    c->ws_A64 = wsA64; c->ws_A32 = wsA32; c->ws_linv = wsL; c->ws_piv = wsP;

    // per-chunk metadata, built once and uploaded into one buffer
    std::vector<char> host;
    struct fix { chunk_t* ch; size_t oN, oA, oP, oL, oV, oI, oAP, oLP; };
    std::vector<fix> fixes;
    auto put = [&](const void* src, size_t bytes) {
        size_t o = align_up(host.size(), 64);
        host.resize(o + bytes);
        memcpy(host.data() + o, src, bytes);
        return o;
    };
    for (auto& ch : px.chunks) {
        std::vector<int32_t> Nv(ch.count);
        std::vector<int64_t> ao(ch.count), po(ch.count), lo(ch.count), vo(ch.count), ap(ch.count + 1);
        std::vector<fhw_assemble_item> items(ch.count);
        int64_t a = 0, pv = 0, l = 0, v = 0, blk = 0;
        for (int q = 0; q < ch.count; ++q) {
            int j = ch.j0 + q;
            int N = c->Ns[j];
            Nv[q] = N;
            ao[q] = a; po[q] = pv; lo[q] = l; vo[q] = v;
            const fhw_geom_entry& ge = c->geoms[fhw_geom_key(c->sys_curve[j], N)];
            items[q].geom = ge.geom;
            items[q].R = ge.R;
            items[q].logtab = ge.logtab;
            items[q].a_off = a;
            items[q].g_off = v;
            items[q].N = N;
            items[q].kappa = c->kappa[j];
            items[q].eta = c->eta[j];
            ap[q] = blk;
            blk += assemble_blocks_for(N);
            a += (int64_t)N * N; pv += N; l += linv_elems(N); v += N;
        }
        ap[ch.count] = blk;
        ch.asm_blocks = blk;
        lu_build_schedule(Nv.data(), ch.count, ch.sched);
        fix f;
        f.ch = &ch;
        f.oN = put(Nv.data(), Nv.size() * 4);
        f.oA = put(ao.data(), ao.size() * 8);
        f.oP = put(po.data(), po.size() * 8);
        f.oL = put(lo.data(), lo.size() * 8);
        f.oV = put(vo.data(), vo.size() * 8);
        f.oI = put(items.data(), items.size() * sizeof(fhw_assemble_item));
        f.oAP = put(ap.data(), ap.size() * 8);
        f.oLP = put(ch.sched.prefix.data(), std::max<size_t>(1, ch.sched.prefix.size()) * 4);
        fixes.push_back(f);
    }
    std::vector<fhw_field_item> fitems(S);
    for (int j = 0; j < S; ++j) {
        fitems[j].geom = c->geoms[fhw_geom_key(c->sys_curve[j], c->Ns[j])].geom;
        fitems[j].psi_off = c->psi_off[j];
        fitems[j].N = c->Ns[j];
        fitems[j].kappa = c->kappa[j];
        fitems[j].eta = c->eta[j];
    }
    size_t oF = put(fitems.data(), fitems.size() * sizeof(fhw_field_item));
    size_t oLF = 0;
    if (c->lf_extra > 0) {
        // graded nodes 1 .. lf_M lf_N: the extra systems, then omega_c (system lf_jc - 1)
        std::vector<fhw_field_item> lfi(c->lf_extra + 1);
        for (int e = 0; e < c->lf_extra; ++e) lfi[e] = fitems[F + e];
        lfi[c->lf_extra] = fitems[p->lf_jc - 1];
        oLF = put(lfi.data(), lfi.size() * sizeof(fhw_field_item));
    }
    c->meta_bytes = align_up(host.size(), 64);
    {
        int rc = grow_small(c, &c->meta, 6, c->meta_bytes);
        if (rc) return rc;
    }
    FHW_HIP(c, hipMemcpyAsync(c->meta, host.data(), host.size(), hipMemcpyHostToDevice, c->stream));
    char* mb = (char*)c->meta;
    for (auto& f : fixes) {
        f.ch->d_N = (int32_t*)(mb + f.oN);
        f.ch->d_aoff = (int64_t*)(mb + f.oA);
        f.ch->d_pivoff = (int64_t*)(mb + f.oP);
        f.ch->d_linvoff = (int64_t*)(mb + f.oL);
        f.ch->d_voff = (int64_t*)(mb + f.oV);
        f.ch->d_items = (fhw_assemble_item*)(mb + f.oI);
        f.ch->d_asm_prefix = (int64_t*)(mb + f.oAP);
        f.ch->d_lu_prefix = (int32_t*)(mb + f.oLP);
    }
    px.d_field_items = (fhw_field_item*)(mb + oF);
    px.d_lf_items = c->lf_extra > 0 ? (fhw_field_item*)(mb + oLF) : nullptr;
    FHW_HIP(c, hipStreamSynchronize(c->stream));
    c->planned = true;
    if (N_out)
        for (int j = 0; j < S; ++j) N_out[j] = c->Ns[j];
    if (psi_off_out)
        for (int j = 0; j <= S; ++j) psi_off_out[j] = c->psi_off[j];
    return FHW_OK;
}

int fhw_plan(fhw_ctx* c, const fhw_curve* curve, const fhw_problem* p, int32_t* N_out, int64_t* psi_off_out) {
    return plan_impl(c, curve, 1, p, N_out, psi_off_out);
}

int fhw_plan_curves(fhw_ctx* c, const fhw_curve* curves, int32_t n_curves, const fhw_problem* p, int32_t* N_out,
                    int64_t* psi_off_out) {
    return plan_impl(c, curves, n_curves, p, N_out, psi_off_out);
}

int fhw_plan_systems(fhw_ctx* c, const fhw_curve* curves, int32_t n_curves, const fhw_system* systems,
                     int32_t n_systems, const fhw_problem* p, int64_t* psi_off_out) {
    if (!c) return FHW_E_INVALID;
    if (!systems) return fhw_fail(c, FHW_E_INVALID, "plan_systems: no systems");
    return plan_impl(c, curves, n_curves, p, nullptr, psi_off_out, systems, n_systems);
}

// winding number of the planned curve about (a, b): 0 outside
static int winding_number(const fhw_host_curve& cv, double a, double b, double* min_dist) {
    const int M = 4096;
    double tot = 0.0, prev = 0.0, dmin = INFINITY;
    for (int k = 0; k <= M; ++k) {
        double x1, x2, d1, d2;
        curve_eval_host(cv, 2.0 * M_PI * (double)k / M, x1, x2, d1, d2);
        const double ang = atan2(x2 - b, x1 - a);
        dmin = std::min(dmin, hypot(x1 - a, x2 - b));
        if (k > 0) {
            double da = ang - prev;
            if (da > M_PI) da -= 2.0 * M_PI;
            if (da < -M_PI) da += 2.0 * M_PI;
            tot += da;
        }
        prev = ang;
    }
    *min_dist = dmin;
    return (int)lround(tot / (2.0 * M_PI));
}

// The factorization of a chunk as one graph launch: its launch sequence (all
// kernels; no memory set or copy nodes) is captured on the context's capture
// stream at the first solve of the plan and replayed on the work stream
// afterwards.  The graph holds the plan's device pointers, so a new plan
// drops it (free_plan).
static int launch_factor_graph(fhw_ctx* c, chunk_t& ch, const fhw_batch_dev& bd, void* LU) {
    if (!ch.lu_graph) {
        if (!c->cap_stream) FHW_HIP(c, hipStreamCreate(&c->cap_stream));
        lu_prepare(c->prob.precision);
        // nothing executes during the capture; the graph runs on the work
        // stream, in order with the work before and after it
        FHW_HIP(c, hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeRelaxed));
        hipError_t e = launch_lu_factor(c->cap_stream, bd, ch.sched, ch.d_lu_prefix, LU, c->piv, c->linv,
                                        c->d_status, c->prob.precision, nullptr);
        hipGraph_t g = nullptr;
        hipError_t e2 = hipStreamEndCapture(c->cap_stream, &g);
        if (e == hipSuccess) e = e2;
        if (e == hipSuccess) e = hipGraphInstantiate(&ch.lu_graph, g, nullptr, nullptr, 0);
        if (g) (void)hipGraphDestroy(g);
        if (e != hipSuccess) {
            ch.lu_graph = nullptr;
            return fhw_hip_check(c, e, "factorization graph capture");
        }
    }
    FHW_HIP(c, hipGraphLaunch(ch.lu_graph, c->stream));
    return FHW_OK;
}

// Where the right-hand sides of a solve come from: incident fields (inc), the
// windows of sampled boundary data (bnd: window k_first + q is right-hand
// side q), or neither (the plan's plane wave, as the assembly left it).
struct rhs_src {
    const fhw_incidence* inc = nullptr;
    const fhw_boundary* bnd = nullptr;
    double H = 0.0;
    int64_t k_first = 0;
};

// The incidences on one factored batch, in groups of up to FHW_INC_GROUP
// (one launch per step for a whole group: a second grid dimension), each
// with its own slot of g and r: boundary data (inc == NULL: the plan's plane
// wave, as the assembly left it in slot 0), solves and, on the FP32 path,
// the refinement sweeps.  Vectors are addressed with the batch's offsets:
// incidence q's densities at x + q xs + v_off[b], of which the elements
// [voff0, voff0 + elems) belong to the batch; its norms at norms + 2 q fs
// and flags at done / sw + q fs (index b within the batch).
static int solve_groups(fhw_ctx* c, const fhw_batch_dev& bd, int32_t maxN, const fhw_assemble_item* d_items,
                        int64_t voff0, int64_t elems, const rhs_src& src, int32_t n_inc, zd* x, int64_t xs,
                        double* norms, int32_t* done, int32_t* sw, int64_t fs) {
    const fhw_incidence* inc = src.inc;
    const fhw_problem& p = c->prob;
    const bool fp32 = p.precision == FHW_FP32_REFINE;
    void* LU = fp32 ? c->A32 : c->A64;
    zd* g = (zd*)c->x;
    zd* r = (zd*)c->r;
    const int64_t sv = c->ws_vec;
    for (int q0 = 0; q0 < n_inc; q0 += FHW_INC_GROUP) {
        const int G = std::min(FHW_INC_GROUP, n_inc - q0);
        zd* xq = x + q0 * xs;     // solutions written in place into psi
        if (inc) {
            fhw_rhs_group rg{};
            rg.n = G;
            for (int q = 0; q < G; ++q) {
                rg.kind[q] = inc[q0 + q].kind;
                rg.v[q][0] = inc[q0 + q].v[0];
                rg.v[q][1] = inc[q0 + q].v[1];
            }
            STAGE(c, FHW_STAGE_ASSEMBLE, launch_rhs(c->stream, d_items, bd.batch, rg, sv, g));
        } else if (src.bnd) {
            const fhw_boundary& b = *src.bnd;
            STAGE(c, FHW_STAGE_ASSEMBLE, launch_boundary_rhs(c->stream, b.b, b.n_t, b.N, b.t0, b.dt, src.H,
                                                             src.k_first + q0, G, p.c, d_items, bd.batch, sv, g));
        }
        for (int q = 0; q < G; ++q)
            FHW_HIP(c, hipMemcpyAsync(xq + q * xs + voff0, g + q * sv + voff0, sizeof(zd) * elems,
                                      hipMemcpyDeviceToDevice, c->stream));
        fhw_grp gs;
        gs.n = G;
        gs.sv = xs;
        STAGE(c, FHW_STAGE_SOLVE, launch_lu_solve(c->stream, bd, maxN, LU, c->piv, c->linv, xq, nullptr,
                                                  p.precision, gs));
        if (!fp32) continue;
        double* nq = norms + 2 * (int64_t)q0 * fs;
        int32_t* dq = done + (int64_t)q0 * fs;
        int32_t* wq = sw + (int64_t)q0 * fs;
        fhw_grp gr;   // residual: x in psi, g and r in their slots
        gr.n = G;
        gr.sx = xs; gr.sg = sv; gr.sr = sv;
        gr.spart = c->rpart_stride; gr.scount = c->chunk; gr.snorm = 2 * fs; gr.sflag = fs;
        fhw_grp ga;   // correction: solve r in place, add into x, skip converged
        ga.n = G;
        ga.sv = sv; ga.sacc = xs; ga.sflag = fs;
        // sweep 0 measures the FP32 solution (never within a tight tolerance:
        // its correction always runs); from sweep 1 on, the number of systems
        // still above the tolerance comes back to the host, and the sweeps
        // stop as soon as it is zero, instead of launching idle ones
        const int maxs = std::max(0, p.refine_max);
        for (int it = 0; it <= maxs; ++it) {
            int32_t* pend = it >= 1 ? c->d_pending : nullptr;
            if (pend) FHW_HIP(c, hipMemsetAsync(pend, 0, sizeof(int32_t), c->stream));
            STAGE(c, FHW_STAGE_RESIDUAL, launch_residual_t(c->stream, bd, maxN, c->A64, xq, g, r, c->d_rpart,
                                                           c->d_rcount, nq, p.refine_tol, dq, wq, it, pend, gr));
            if (pend) {
                FHW_HIP(c, hipMemcpyAsync(c->h_pending, pend, sizeof(int32_t), hipMemcpyDeviceToHost, c->stream));
                FHW_HIP(c, hipStreamSynchronize(c->stream));
                if (*c->h_pending == 0) break;
            }
            if (it == maxs) break;
            STAGE(c, FHW_STAGE_SOLVE, launch_lu_solve_acc(c->stream, bd, maxN, LU, c->piv, c->linv, r, xq, dq,
                                                          p.precision, ga));
        }
    }
    return FHW_OK;
}

// The calls of the direct equation (incident waves, single-layer field)
// refuse a plan of the combined formulation.
static int direct_only(fhw_ctx* c, const char* what) {
    if (c->prob.formulation != FHW_FORM_DIRECT)
        return fhw_fail(c, FHW_E_STATE, std::string(what) + ": the plan is of the combined formulation (general "
                                                              "boundary data: fhw_solve_general and the window calls)");
    return FHW_OK;
}

// Densities for n_inc incidences (inc == NULL: the plan's plane wave, whose
// boundary data the assembly kernel writes).  psi holds n_inc blocks of
// psi_off[F] elements; resid / sweeps [host] are [n_inc][F].
static int solve_impl(fhw_ctx* c, const fhw_incidence* inc, int32_t n_inc, void* psi, double* resid,
                      int32_t* sweeps, int32_t compute_resid, bool reuse) {
    plan_ext& px = plan_of(c);
    const fhw_problem& p = c->prob;
    const int F = (int)c->Ns.size();   // systems (curves x frequencies)
    const bool fp32 = p.precision == FHW_FP32_REFINE;
    const int64_t total = c->psi_off[F];
    // per-(incidence, frequency) status: the plan's arrays for one incidence,
    // the scratch buffer for several
    int32_t *d_done = c->d_done, *d_sw = c->d_sweeps;
    double* d_norms = c->d_norms;
    if (n_inc > 1) {
        const size_t nf = (size_t)n_inc * F;
        const size_t off_sw = align_up(nf * 4, 256), off_nrm = off_sw + align_up(nf * 4, 256);
        int rc = fhw_ensure_scratch(c, off_nrm + nf * 16);
        if (rc) return rc;
        d_done = (int32_t*)c->scratch;
        d_sw = (int32_t*)((char*)c->scratch + off_sw);
        d_norms = (double*)((char*)c->scratch + off_nrm);
    }
    FHW_HIP(c, hipMemsetAsync(c->d_status, 0, sizeof(int32_t) * 4, c->stream));
    FHW_HIP(c, hipMemsetAsync(d_done, 0, sizeof(int32_t) * F * n_inc, c->stream));
    FHW_HIP(c, hipMemsetAsync(d_sw, 0, sizeof(int32_t) * F * n_inc, c->stream));
    zd* psid = (zd*)psi;
    zd* g = (zd*)c->x;
    zd* r = (zd*)c->r;
    for (auto& ch : px.chunks) {
        fhw_batch_dev bd{ch.d_N, ch.d_aoff, ch.d_pivoff, ch.d_linvoff, ch.d_voff, ch.count};
        void* LU = fp32 ? c->A32 : c->A64;
        if (!reuse) {
            c->factors_resident = false;
            STAGE(c, FHW_STAGE_ASSEMBLE, launch_assemble_blocks(c->stream, ch.d_items, ch.d_asm_prefix, ch.count,
                                                                ch.asm_blocks, p.direction[0], p.direction[1], c->A64,
                                                                fp32 ? c->A32 : nullptr, g, p.formulation == FHW_FORM_COMBINED));
            if (c->prof.on) {
                // per-stage timers need the launches one by one
                FHW_HIP(c, launch_lu_factor(c->stream, bd, ch.sched, ch.d_lu_prefix, LU, c->piv, c->linv,
                                            c->d_status, p.precision, &c->prof));
            } else {
                int rc = launch_factor_graph(c, ch, bd, LU);
                if (rc) return rc;
            }
        }
        {
            rhs_src src;
            src.inc = inc;
            int rc = solve_groups(c, bd, ch.maxN, ch.d_items, 0, ch.vec_elems, src, n_inc, psid + ch.psi_base, total,
                                  d_norms + 2 * (int64_t)ch.j0, d_done + ch.j0, d_sw + ch.j0, F);
            if (rc) return rc;
        }
        if (!fp32 && compute_resid) {
            // the factorization overwrote A: assemble it again for the residuals
            // (which also ends the residency of the FP64 factors)
            STAGE(c, FHW_STAGE_ASSEMBLE, launch_assemble_blocks(c->stream, ch.d_items, ch.d_asm_prefix, ch.count, ch.asm_blocks,
                                              p.direction[0], p.direction[1], c->A64, nullptr, g,
                                              p.formulation == FHW_FORM_COMBINED));
            const int64_t sv = c->ws_vec;
            for (int q0 = 0; q0 < n_inc; q0 += FHW_INC_GROUP) {
                const int G = std::min(FHW_INC_GROUP, n_inc - q0);
                if (inc) {
                    fhw_rhs_group rg{};
                    rg.n = G;
                    for (int q = 0; q < G; ++q) {
                        rg.kind[q] = inc[q0 + q].kind;
                        rg.v[q][0] = inc[q0 + q].v[0];
                        rg.v[q][1] = inc[q0 + q].v[1];
                    }
                    STAGE(c, FHW_STAGE_ASSEMBLE, launch_rhs(c->stream, ch.d_items, ch.count, rg, sv, g));
                }
                double* norms = d_norms + 2 * ((int64_t)q0 * F + ch.j0);
                fhw_grp gr;
                gr.n = G;
                gr.sx = total; gr.sg = sv; gr.sr = sv;
                gr.spart = c->rpart_stride; gr.scount = c->chunk; gr.snorm = 2 * (int64_t)F;
                STAGE(c, FHW_STAGE_RESIDUAL, launch_residual_t(c->stream, bd, ch.maxN, c->A64,
                                                               psid + q0 * total + ch.psi_base, g, r, c->d_rpart,
                                                               c->d_rcount, norms, 0.0, nullptr, nullptr, 0, nullptr,
                                                               gr));
            }
        }
    }
    int32_t st[4];
    const size_t nf = (size_t)F * n_inc;
    const bool have_norms = fp32 || compute_resid;
    std::vector<double> nrm(have_norms ? 2 * nf : 0);
    std::vector<int32_t> done(fp32 ? nf : 0), sw(fp32 ? nf : 0);
    {
        int rc = readback(c, {{st, c->d_status, sizeof(st)},
                              {nrm.data(), d_norms, sizeof(double) * nrm.size()},
                              {done.data(), d_done, sizeof(int32_t) * done.size()},
                              {sw.data(), d_sw, sizeof(int32_t) * sw.size()}});
        if (rc) return rc;
    }
    // factors stay usable when the whole plan fits one chunk and nothing
    // overwrote them (FP64 residuals re-assemble A in place)
    if (!reuse) c->factors_resident = px.chunks.size() == 1 && !(!fp32 && compute_resid) && !st[0];
    for (size_t j = 0; j < nf; ++j) {
        if (resid) resid[j] = have_norms ? (nrm[2 * j + 1] > 0 ? nrm[2 * j] / nrm[2 * j + 1] : 0.0) : -1.0;
        if (sweeps) sweeps[j] = fp32 ? (done[j] ? sw[j] : p.refine_max) : 0;
    }
    if (st[0]) return fhw_fail(c, FHW_E_SINGULAR, "solve: exactly zero pivot in an LU factorization");
    if (fp32)
        for (size_t j = 0; j < nf; ++j)
            if (!done[j]) return fhw_fail(c, FHW_E_NOCONV, "solve: refinement did not reach refine_tol");
    return FHW_OK;
}

int fhw_solve_densities(fhw_ctx* c, void* psi, double* resid, int32_t* sweeps, int32_t compute_resid) {
    if (!c) return FHW_E_INVALID;
    if (!c->planned) return fhw_fail(c, FHW_E_STATE, "solve: no plan");
    if (int rc_d = direct_only(c, "solve_densities")) return rc_d;
    if (!psi) return fhw_fail(c, FHW_E_INVALID, "solve: psi is null");
    return solve_impl(c, nullptr, 1, psi, resid, sweeps, compute_resid, false);
}

static int check_incidences(fhw_ctx* c, const fhw_incidence* inc, int32_t n_inc, const void* psi) {
    if (!inc || n_inc < 1 || !psi) return fhw_fail(c, FHW_E_INVALID, "solve: need n_inc >= 1 incidences and psi");
    for (int q = 0; q < n_inc; ++q) {
        const double a = inc[q].v[0], b = inc[q].v[1];
        if (!isfinite(a) || !isfinite(b)) return fhw_fail(c, FHW_E_INVALID, "solve: incidence not finite");
        if (inc[q].kind == FHW_INC_PLANE) {
            if (fabs(hypot(a, b) - 1.0) > 1e-12) return fhw_fail(c, FHW_E_INVALID, "solve: direction not a unit vector");
        } else if (inc[q].kind == FHW_INC_POINT) {
            for (const fhw_host_curve& cv : c->curves) {
                double dmin;
                if (winding_number(cv, a, b, &dmin) != 0 || !(dmin > 0.0))
                    return fhw_fail(c, FHW_E_INVALID, "solve: point source on or inside a curve");
            }
        } else {
            return fhw_fail(c, FHW_E_INVALID, "solve: unknown incidence kind");
        }
    }
    return FHW_OK;
}

int fhw_solve_incidences(fhw_ctx* c, const fhw_incidence* inc, int32_t n_inc, void* psi, double* resid,
                         int32_t* sweeps, int32_t compute_resid) {
    if (!c) return FHW_E_INVALID;
    if (!c->planned) return fhw_fail(c, FHW_E_STATE, "solve: no plan");
    if (int rc_d = direct_only(c, "solve_incidences")) return rc_d;
    int rc = check_incidences(c, inc, n_inc, psi);
    if (rc) return rc;
    return solve_impl(c, inc, n_inc, psi, resid, sweeps, compute_resid, false);
}

int fhw_solve_cached(fhw_ctx* c, const fhw_incidence* inc, int32_t n_inc, void* psi, double* resid,
                     int32_t* sweeps) {
    if (!c) return FHW_E_INVALID;
    if (!c->planned) return fhw_fail(c, FHW_E_STATE, "solve: no plan");
    if (int rc_d = direct_only(c, "solve_cached")) return rc_d;
    if (!c->factors_resident)
        return fhw_fail(c, FHW_E_STATE, "solve_cached: no resident factors (no solve yet, several chunks, "
                                        "or FP64 residuals overwrote them)");
    int rc = check_incidences(c, inc, n_inc, psi);
    if (rc) return rc;
    return solve_impl(c, inc, n_inc, psi, resid, sweeps, 0, true);
}

int fhw_factor(fhw_ctx* c) {
    if (!c) return FHW_E_INVALID;
    if (!c->planned) return fhw_fail(c, FHW_E_STATE, "factor: no plan");
    if (plan_of(c).chunks.size() != 1)
        return fhw_fail(c, FHW_E_NOMEM, "factor: the plan does not fit one workspace chunk");
    return solve_impl(c, nullptr, 0, nullptr, nullptr, nullptr, 0, false);
}

// Systems s0 .. s0 + count - 1 on the resident factors for n right-hand
// sides from src; psi holds the range's densities per right-hand side
// (element e of right-hand side q at psi + q elems + e).  what names the
// entry point in messages.
static int range_solve(fhw_ctx* c, const char* what, int32_t s0, int32_t count, const rhs_src& src, int32_t n,
                       void* psi, double* resid, int32_t* sweeps) {
    plan_ext& px = plan_of(c);
    const chunk_t& ch = px.chunks[0];
    const fhw_problem& p = c->prob;
    const bool fp32 = p.precision == FHW_FP32_REFINE;
    // the range as a sub-batch of the resident chunk: its rows of the
    // per-matrix device tables, vectors addressed with the chunk's offsets
    const int b0 = s0 - ch.j0;
    fhw_batch_dev bd{ch.d_N + b0, ch.d_aoff + b0, ch.d_pivoff + b0, ch.d_linvoff + b0, ch.d_voff + b0, count};
    int32_t maxN = 0;
    for (int s = s0; s < s0 + count; ++s) maxN = std::max(maxN, c->Ns[s]);
    const int64_t voff0 = c->psi_off[s0] - ch.psi_base;
    const int64_t elems = c->psi_off[s0 + count] - c->psi_off[s0];
    const size_t nf = (size_t)n * count;
    const size_t off_sw = align_up(nf * 4, 256), off_nrm = off_sw + align_up(nf * 4, 256);
    int rc = fhw_ensure_scratch(c, off_nrm + nf * 16);
    if (rc) return rc;
    int32_t* d_done = (int32_t*)c->scratch;
    int32_t* d_sw = (int32_t*)((char*)c->scratch + off_sw);
    double* d_norms = (double*)((char*)c->scratch + off_nrm);
    FHW_HIP(c, hipMemsetAsync(d_done, 0, sizeof(int32_t) * nf, c->stream));
    FHW_HIP(c, hipMemsetAsync(d_sw, 0, sizeof(int32_t) * nf, c->stream));
    zd* x = (zd*)psi - voff0;
    rc = solve_groups(c, bd, maxN, ch.d_items + b0, voff0, elems, src, n, x, elems, d_norms, d_done, d_sw, count);
    if (rc) return rc;
    std::vector<double> nrm(fp32 ? 2 * nf : 0);
    std::vector<int32_t> done(fp32 ? nf : 0), sw(fp32 ? nf : 0);
    rc = readback(c, {{nrm.data(), d_norms, sizeof(double) * nrm.size()},
                      {done.data(), d_done, sizeof(int32_t) * done.size()},
                      {sw.data(), d_sw, sizeof(int32_t) * sw.size()}});
    if (rc) return rc;
    for (size_t j = 0; j < nf; ++j) {
        if (resid) resid[j] = fp32 ? (nrm[2 * j + 1] > 0 ? nrm[2 * j] / nrm[2 * j + 1] : 0.0) : -1.0;
        if (sweeps) sweeps[j] = fp32 ? (done[j] ? sw[j] : p.refine_max) : 0;
    }
    if (fp32)
        for (size_t j = 0; j < nf; ++j)
            if (!done[j]) return fhw_fail(c, FHW_E_NOCONV, std::string(what) + ": refinement did not reach refine_tol");
    return FHW_OK;
}

int fhw_solve_range(fhw_ctx* c, int32_t s0, int32_t count, const fhw_incidence* inc, int32_t n_inc, void* psi,
                    double* resid, int32_t* sweeps) {
    if (!c) return FHW_E_INVALID;
    if (!c->planned) return fhw_fail(c, FHW_E_STATE, "solve_range: no plan");
    if (int rc_d = direct_only(c, "solve_range")) return rc_d;
    if (!c->factors_resident)
        return fhw_fail(c, FHW_E_STATE, "solve_range: no resident factors (fhw_factor first)");
    const int S = (int)c->Ns.size();
    if (s0 < 0 || count < 1 || s0 > S - count) return fhw_fail(c, FHW_E_INVALID, "solve_range: systems out of range");
    int rc = check_incidences(c, inc, n_inc, psi);
    if (rc) return rc;
    rhs_src src;
    src.inc = inc;
    return range_solve(c, "solve_range", s0, count, src, n_inc, psi, resid, sweeps);
}

int fhw_window_range(double t_lo, double t_hi, double H, int64_t* k_first, int32_t* n_win) {
    if (!k_first || !n_win || !isfinite(t_lo) || !isfinite(t_hi) || !(t_hi >= t_lo) || !(H > 0) || !isfinite(H))
        return FHW_E_INVALID;
    const double span = 1.5 * H;
    int64_t k_lo = (int64_t)floor((t_lo - H) / span);
    int64_t k_hi = (int64_t)ceil((t_hi + H) / span) + 2;
    while (k_lo <= k_hi && !(span * ((double)k_lo - 1.0) + H >= t_lo)) ++k_lo;
    while (k_hi >= k_lo && !(span * ((double)k_hi - 1.0) - H <= t_hi)) --k_hi;
    if (k_hi - k_lo + 1 > INT32_MAX) return FHW_E_INVALID;
    *k_first = k_lo;
    *n_win = (int32_t)(k_hi - k_lo + 1);
    return FHW_OK;
}

// A plan the general-data path takes: the combined formulation, one curve,
// the DFT grid, the same N at every frequency (the boundary samples' nodes).
static int general_plan_check(fhw_ctx* c, const char* what) {
    if (!c->planned) return fhw_fail(c, FHW_E_STATE, std::string(what) + ": no plan");
    if (c->prob.formulation != FHW_FORM_COMBINED || c->prob.j_first != 0 || c->system_plan || c->curves.size() != 1)
        return fhw_fail(c, FHW_E_STATE, std::string(what) + ": needs a plan of the combined formulation (one "
                                                              "curve on the DFT grid)");
    for (int32_t N : c->Ns)
        if (N != c->Ns[0])
            return fhw_fail(c, FHW_E_STATE, std::string(what) + ": needs the same N at every frequency");
    return FHW_OK;
}

int fhw_solve_general(fhw_ctx* c, const fhw_boundary* bnd, double H, int64_t k_first, int32_t n_win, void* psi,
                      double* resid, int32_t* sweeps) {
    if (!c) return FHW_E_INVALID;
    int rc = general_plan_check(c, "solve_general");
    if (rc) return rc;
    if (!c->factors_resident)
        return fhw_fail(c, FHW_E_STATE, "solve_general: no resident factors (fhw_factor first)");
    if (!bnd || !bnd->b || !psi || n_win < 1)
        return fhw_fail(c, FHW_E_INVALID, "solve_general: need boundary data, psi and n_win >= 1");
    if (bnd->N != c->Ns[0]) return fhw_fail(c, FHW_E_INVALID, "solve_general: boundary data at another N");
    if (bnd->n_t < 2 || !(bnd->dt > 0) || !isfinite(bnd->dt) || !isfinite(bnd->t0))
        return fhw_fail(c, FHW_E_INVALID, "solve_general: need n_t >= 2, dt > 0 and a finite t0");
    if (!(H > 0) || !isfinite(H) || !isfinite(1.5 * H * ((double)k_first - 1.0)) ||
        !isfinite(1.5 * H * ((double)k_first + n_win)))
        return fhw_fail(c, FHW_E_INVALID, "solve_general: bad windows");
    rhs_src src;
    src.bnd = bnd;
    src.H = H;
    src.k_first = k_first;
    return range_solve(c, "solve_general", 0, (int32_t)c->Ns.size(), src, n_win, psi, resid, sweeps);
}

int fhw_eval_field_windows(fhw_ctx* c, const void* psi, int32_t n_win, const double* obs, int32_t N_r, void* V) {
    if (!c) return FHW_E_INVALID;
    int rc = general_plan_check(c, "field_windows");
    if (rc) return rc;
    if (n_win < 0 || N_r < 0 || (n_win > 0 && N_r > 0 && (!psi || !obs || !V)))
        return fhw_fail(c, FHW_E_INVALID, "field_windows: bad arguments");
    if (n_win == 0 || N_r == 0) return FHW_OK;
    if (n_win > 65535 * 8) return fhw_fail(c, FHW_E_INVALID, "field_windows: too many windows");
    for (int q = 0; q < 2 * N_r; ++q)
        if (!isfinite(obs[q])) return fhw_fail(c, FHW_E_INVALID, "field_windows: observation point not finite");
    rc = fhw_ensure_scratch(c, (size_t)N_r * 16);
    if (rc) return rc;
    const int F = c->prob.F;
    FHW_HIP(c, hipMemcpyAsync(c->scratch, obs, (size_t)N_r * 16, hipMemcpyHostToDevice, c->stream));
    STAGE(c, FHW_STAGE_FIELD, launch_field_blocks(c->stream, plan_of(c).d_field_items, F, psi,
                                                  c->psi_off[c->Ns.size()], n_win, (const double*)c->scratch, N_r,
                                                  0.0, V, (int64_t)N_r * 2 * F));
    FHW_HIP(c, hipStreamSynchronize(c->stream));
    return FHW_OK;
}

// fhw_solve_range with its status words in the fixed device array: the same
// solves (solve_groups), no allocation.  Layout of the array for nf =
// n_inc * count pairs: done | sweeps | norms (2 nf) | resid out | sweeps out |
// counter, each at a 256-byte boundary.
int fhw_solve_range_noalloc(fhw_ctx* c, int32_t s0, int32_t count, const fhw_incidence* inc, int32_t n_inc,
                            void* psi, double* resid, int32_t* sweeps) {
    if (!c) return FHW_E_INVALID;
    if (!c->planned) return fhw_fail(c, FHW_E_STATE, "solve_range_noalloc: no plan");
    if (int rc_d = direct_only(c, "solve_range_noalloc")) return rc_d;
    if (!c->factors_resident)
        return fhw_fail(c, FHW_E_STATE, "solve_range_noalloc: no resident factors (fhw_factor first)");
    const int S = (int)c->Ns.size();
    if (s0 < 0 || count < 1 || s0 > S - count)
        return fhw_fail(c, FHW_E_INVALID, "solve_range_noalloc: systems out of range");
    int rc = check_incidences(c, inc, n_inc, psi);
    if (rc) return rc;
    if ((int64_t)n_inc * count > FHW_NOALLOC_MAX_PAIRS)
        return fhw_fail(c, FHW_E_INVALID, "solve_range_noalloc: n_inc * count = " +
                                              std::to_string((int64_t)n_inc * count) + " exceeds " +
                                              std::to_string(FHW_NOALLOC_MAX_PAIRS));
    if (!c->noalloc) return fhw_fail(c, FHW_E_HIP, c->noalloc_err);
    const size_t nf = (size_t)n_inc * count;
    const size_t o_done = 0, o_sw = align_up(o_done + nf * 4, 256), o_nrm = align_up(o_sw + nf * 4, 256);
    const size_t o_res = align_up(o_nrm + nf * 16, 256), o_swo = align_up(o_res + nf * 8, 256);
    const size_t o_cnt = align_up(o_swo + nf * 4, 256);
    static_assert(FHW_NOALLOC_MAX_PAIRS * 36 + 6 * 256 <= FHW_NOALLOC_SCRATCH_BYTES, "status array too small");
    if (o_cnt + 4 > FHW_NOALLOC_SCRATCH_BYTES) return fhw_fail(c, FHW_E_INVALID, "solve_range_noalloc: too many pairs");
    char* sb = (char*)c->noalloc;
    int32_t* d_done = (int32_t*)(sb + o_done);
    int32_t* d_sw = (int32_t*)(sb + o_sw);
    double* d_norms = (double*)(sb + o_nrm);
    double* d_res = (double*)(sb + o_res);
    int32_t* d_swo = (int32_t*)(sb + o_swo);
    int32_t* d_cnt = (int32_t*)(sb + o_cnt);
    prof_pause pause(c->prof);
    plan_ext& px = plan_of(c);
    const chunk_t& ch = px.chunks[0];
    const fhw_problem& p = c->prob;
    const bool fp32 = p.precision == FHW_FP32_REFINE;
    const int b0 = s0 - ch.j0;
    fhw_batch_dev bd{ch.d_N + b0, ch.d_aoff + b0, ch.d_pivoff + b0, ch.d_linvoff + b0, ch.d_voff + b0, count};
    int32_t maxN = 0;
    for (int s = s0; s < s0 + count; ++s) maxN = std::max(maxN, c->Ns[s]);
    const int64_t voff0 = c->psi_off[s0] - ch.psi_base;
    const int64_t elems = c->psi_off[s0 + count] - c->psi_off[s0];
    FHW_HIP(c, launch_status_clear(c->stream, d_done, d_sw, d_cnt, (int64_t)nf));
    zd* x = (zd*)psi - voff0;
    rhs_src src;
    src.inc = inc;
    rc = solve_groups(c, bd, maxN, ch.d_items + b0, voff0, elems, src, n_inc, x, elems, d_norms, d_done, d_sw, count);
    if (rc) return rc;
    FHW_HIP(c, launch_status_finish(c->stream, d_done, d_sw, d_norms, (int64_t)nf, fp32 ? 1 : 0, p.refine_max, d_res,
                                    d_swo, d_cnt));
    if (resid) FHW_HIP(c, hipMemcpyAsync(resid, d_res, nf * 8, hipMemcpyDeviceToHost, c->stream));
    if (sweeps) FHW_HIP(c, hipMemcpyAsync(sweeps, d_swo, nf * 4, hipMemcpyDeviceToHost, c->stream));
    FHW_HIP(c, hipMemcpyAsync(c->h_pending, d_cnt, 4, hipMemcpyDeviceToHost, c->stream));
    FHW_HIP(c, hipStreamSynchronize(c->stream));
    if (fp32 && *c->h_pending != 0)
        return fhw_fail(c, FHW_E_NOCONV, "solve_range_noalloc: refinement did not reach refine_tol");
    return FHW_OK;
}

int fhw_eval_field_curve(fhw_ctx* c, int32_t curve, const void* psi, const double* obs, int32_t N_r,
                         double zero_value, void* V) {
    if (!c) return FHW_E_INVALID;
    if (!c->planned) return fhw_fail(c, FHW_E_STATE, "field: no plan");
    if (int rc_d = direct_only(c, "field")) return rc_d;
    if (c->prob.j_first != 0 || c->system_plan)
        return fhw_fail(c, FHW_E_STATE, "field: the plan is a band or a list of systems (no DFT grid)");
    if (curve < 0 || curve >= (int)c->curves.size()) return fhw_fail(c, FHW_E_INVALID, "field: no such curve");
    if (N_r < 0 || (N_r > 0 && (!psi || !obs || !V))) return fhw_fail(c, FHW_E_INVALID, "field: bad arguments");
    if (N_r == 0) return FHW_OK;
    for (int q = 0; q < 2 * N_r; ++q)
        if (!isfinite(obs[q])) return fhw_fail(c, FHW_E_INVALID, "field: observation point not finite");
    int rc = fhw_ensure_scratch(c, (size_t)N_r * 16);
    if (rc) return rc;
    FHW_HIP(c, hipMemcpyAsync(c->scratch, obs, (size_t)N_r * 16, hipMemcpyHostToDevice, c->stream));
    STAGE(c, FHW_STAGE_FIELD, launch_field(c->stream, plan_of(c).d_field_items + (int64_t)curve * c->prob.F,
                                           c->prob.F, psi, (const double*)c->scratch, N_r, zero_value, V));
    FHW_HIP(c, hipStreamSynchronize(c->stream));
    return FHW_OK;
}

int fhw_eval_field(fhw_ctx* c, const void* psi, const double* obs, int32_t N_r, double zero_value, void* V) {
    return fhw_eval_field_curve(c, 0, psi, obs, N_r, zero_value, V);
}

int fhw_eval_field_lowfreq(fhw_ctx* c, const void* psi, const double* obs, int32_t N_r, double zero_value,
                           void* V_sing) {
    if (!c) return FHW_E_INVALID;
    if (!c->planned) return fhw_fail(c, FHW_E_STATE, "field_lowfreq: no plan");
    if (int rc_d = direct_only(c, "field_lowfreq")) return rc_d;
    if (c->lf_extra <= 0) return fhw_fail(c, FHW_E_STATE, "field_lowfreq: the plan has no graded low-frequency nodes");
    if (N_r < 0 || (N_r > 0 && (!psi || !obs || !V_sing)) || !isfinite(zero_value))
        return fhw_fail(c, FHW_E_INVALID, "field_lowfreq: bad arguments");
    if (N_r == 0) return FHW_OK;
    for (int q = 0; q < 2 * N_r; ++q)
        if (!isfinite(obs[q])) return fhw_fail(c, FHW_E_INVALID, "field_lowfreq: observation point not finite");
    int rc = fhw_ensure_scratch(c, (size_t)N_r * 16);
    if (rc) return rc;
    FHW_HIP(c, hipMemcpyAsync(c->scratch, obs, (size_t)N_r * 16, hipMemcpyHostToDevice, c->stream));
    STAGE(c, FHW_STAGE_FIELD, launch_field_list(c->stream, plan_of(c).d_lf_items, c->lf_extra + 1, psi,
                                                (const double*)c->scratch, N_r, zero_value, V_sing, false));
    FHW_HIP(c, hipStreamSynchronize(c->stream));
    return FHW_OK;
}

// Windows k whose support [s_k - H, s_k + H], s_k = 1.5 H (k - 1), meets the
// signal's sample range (Sec. 3.1); empty when k_lo > k_hi.
static void signal_windows(const fhw_signal* sig, double H, int64_t* k_lo_out, int64_t* k_hi_out) {
    const double tlo = sig->t0, thi = sig->t0 + sig->dt * (double)(sig->n - 1);
    const double span = 1.5 * H;
    int64_t k_lo = (int64_t)floor((tlo - H) / span) + 1 - 1;
    int64_t k_hi = (int64_t)ceil((thi + H) / span) + 1 + 1;
    while (k_lo <= k_hi && !(1.5 * H * ((double)k_lo - 1.0) + H >= tlo)) ++k_lo;
    while (k_hi >= k_lo && !(1.5 * H * ((double)k_hi - 1.0) - H <= thi)) --k_hi;
    *k_lo_out = k_lo;
    *k_hi_out = k_hi;
}

int fhw_synthesize(fhw_ctx* c, const fhw_signal* sig, const fhw_windows* win, const void* V, int32_t N_r,
                   const double* times, int32_t N_t, double* u) {
    if (!c) return FHW_E_INVALID;
    if (!c->planned) return fhw_fail(c, FHW_E_STATE, "synthesize: no plan");
    if (c->prob.j_first != 0 || c->system_plan)
        return fhw_fail(c, FHW_E_STATE, "synthesize: the plan is a band or a list of systems (no DFT grid)");
    if (!sig || !win || N_r < 0 || N_t < 0) return fhw_fail(c, FHW_E_INVALID, "synthesize: bad arguments");
    if (N_r == 0 || N_t == 0) return FHW_OK;
    if (!V || !times || !u || !sig->f || sig->n < 2 || !(sig->dt > 0) || !isfinite(sig->t0))
        return fhw_fail(c, FHW_E_INVALID, "synthesize: bad signal or buffers");
    const double H = win->H, tau0 = win->tau0, ttol = win->track_tol;
    if (!(H > 0) || !isfinite(H) || !isfinite(tau0)) return fhw_fail(c, FHW_E_INVALID, "synthesize: bad windows");
    if (!(ttol >= 0) || !isfinite(ttol)) return fhw_fail(c, FHW_E_INVALID, "synthesize: track_tol must be >= 0");
    const bool track = ttol > 0;
    const int F = c->prob.F;
    const int M = 2 * F;
    if (M & (M - 1)) return fhw_fail(c, FHW_E_INVALID, "synthesize: 2F must be a power of two");
    if (M > 8192 || (size_t)M * 16 > (size_t)lds_limit(c)) return fhw_fail(c, FHW_E_INVALID, "synthesize: 2F too large");
    const double W = c->prob.W;
    int64_t k_lo, k_hi;
    signal_windows(sig, H, &k_lo, &k_hi);
    const double span = 1.5 * H;
    const double P = M_PI / (W / (double)F);
    std::vector<int32_t> slot;
    std::vector<int64_t> klist;
    if (k_hi >= k_lo) {
        slot.assign(k_hi - k_lo + 1, -1);
        std::vector<char> need(k_hi - k_lo + 1, 0);
        for (int q = 0; q < N_t; ++q) {
            const double t = times[q];
            if (!isfinite(t)) return fhw_fail(c, FHW_E_INVALID, "synthesize: time not finite");
            int64_t ka = (int64_t)floor((t - tau0 - P) / span) + 1 - 1;
            int64_t kb = (int64_t)ceil((t - tau0 + P) / span) + 1 + 1;
            for (int64_t k = std::max(ka, k_lo); k <= std::min(kb, k_hi); ++k) {
                const double sk = 1.5 * H * ((double)k - 1.0);
                if (fabs(t - sk - tau0) <= P) need[k - k_lo] = 1;
            }
        }
        for (int64_t k = k_lo; k <= k_hi; ++k)
            if (need[k - k_lo]) {
                slot[k - k_lo] = (int32_t)klist.size();
                klist.push_back(k);
            }
    }
    const int count = (int)klist.size();
    // scratch layout: times | slot | klist | B | c
    size_t o_t = 0;
    size_t o_s = align_up(o_t + (size_t)N_t * 8, 256);
    size_t o_k = align_up(o_s + std::max<size_t>(1, slot.size()) * 4, 256);
    size_t o_B = align_up(o_k + std::max<size_t>(1, klist.size()) * 8, 256);
    size_t o_c = align_up(o_B + (size_t)count * M * 16, 256);
    size_t o_bnd = align_up(o_c + (size_t)count * N_r * M * 8, 256);   // real parts of c
    size_t o_max = align_up(o_bnd + (size_t)count * N_r * 8, 256);      // tracking bounds
    size_t o_wm = align_up(o_max + 16, 256);                            // window maxima
    size_t total = align_up(o_wm + (size_t)std::max(count, 1) * 8, 256);
    int rc = fhw_ensure_scratch(c, total);
    if (rc) return rc;
    char* sb = (char*)c->scratch;
    FHW_HIP(c, hipMemcpyAsync(sb + o_t, times, (size_t)N_t * 8, hipMemcpyHostToDevice, c->stream));
    if (!slot.empty())
        FHW_HIP(c, hipMemcpyAsync(sb + o_s, slot.data(), slot.size() * 4, hipMemcpyHostToDevice, c->stream));
    if (count > 0)
        FHW_HIP(c, hipMemcpyAsync(sb + o_k, klist.data(), klist.size() * 8, hipMemcpyHostToDevice, c->stream));
    STAGE(c, FHW_STAGE_SPECTRA, launch_window_spectra(c->stream, sig->f, sig->n, sig->t0, sig->dt, H, 0, (const int64_t*)(sb + o_k),
                                     count, W, F, sb + o_B));
    double* bnd = track ? (double*)(sb + o_bnd) : nullptr;
    unsigned long long* gmax = track ? (unsigned long long*)(sb + o_max) : nullptr;
    if (track) FHW_HIP(c, hipMemsetAsync(gmax, 0, 16, c->stream));   // gmax and the window-level max
    STAGE(c, FHW_STAGE_COEFFS, launch_fourier_coeffs(c->stream, sb + o_B, count, V, N_r, W, F, tau0, nullptr,
                                                     (double*)(sb + o_c), bnd, gmax, (double*)(sb + o_wm),
                                                     gmax ? gmax + 1 : nullptr, ttol));
    c->trk_pairs = (int64_t)count * N_r;
    c->trk_active = c->trk_pairs;
    if (count == 0) {
        FHW_HIP(c, hipMemsetAsync(u, 0, sizeof(double) * (size_t)N_r * N_t, c->stream));
    } else {
        STAGE(c, FHW_STAGE_SYNTH, launch_synth(c->stream, sb + o_c, (const int32_t*)(sb + o_s), k_lo, k_hi, count, N_r,
                                (const double*)(sb + o_t), N_t, W, F, H, tau0, u, bnd, gmax, ttol));
    }
    FHW_HIP(c, hipStreamSynchronize(c->stream));
    if (track && count > 0) {
        // pairs kept, for fhw_synth_active_pairs
        std::vector<double> b((size_t)count * N_r);
        unsigned long long mx = 0;
        if (int rc_ = copy_d2h(c, b.data(), bnd, 8 * b.size())) return rc_;
        if (int rc_ = copy_d2h(c, &mx, gmax, 8)) return rc_;
        double gm;
        memcpy(&gm, &mx, 8);
        int64_t n = 0;
        for (double v : b) n += v > ttol * gm ? 1 : 0;
        c->trk_active = n;
    }
    return FHW_OK;
}

int fhw_eval_field_windows_lowfreq(fhw_ctx* c, const void* psi, int32_t n_win, const double* obs, int32_t N_r,
                                   void* V_sing) {
    if (!c) return FHW_E_INVALID;
    int rc = general_plan_check(c, "field_windows_lowfreq");
    if (rc) return rc;
    if (c->lf_extra <= 0)
        return fhw_fail(c, FHW_E_STATE, "field_windows_lowfreq: the plan has no graded low-frequency nodes");
    if (n_win < 0 || N_r < 0 || (n_win > 0 && N_r > 0 && (!psi || !obs || !V_sing)))
        return fhw_fail(c, FHW_E_INVALID, "field_windows_lowfreq: bad arguments");
    if (n_win == 0 || N_r == 0) return FHW_OK;
    if (n_win > 65535 * 8) return fhw_fail(c, FHW_E_INVALID, "field_windows_lowfreq: too many windows");
    for (int q = 0; q < 2 * N_r; ++q)
        if (!isfinite(obs[q])) return fhw_fail(c, FHW_E_INVALID, "field_windows_lowfreq: observation point not finite");
    rc = fhw_ensure_scratch(c, (size_t)N_r * 16);
    if (rc) return rc;
    FHW_HIP(c, hipMemcpyAsync(c->scratch, obs, (size_t)N_r * 16, hipMemcpyHostToDevice, c->stream));
    const int64_t ps = c->psi_off[c->Ns.size()], vs = (int64_t)N_r * (c->lf_extra + 2);
    STAGE(c, FHW_STAGE_FIELD, launch_field_blocks(c->stream, plan_of(c).d_lf_items, c->lf_extra + 1, psi, ps, n_win,
                                                  (const double*)c->scratch, N_r, 0.0, V_sing, vs, true));
    FHW_HIP(c, hipStreamSynchronize(c->stream));
    return FHW_OK;
}

// Synthesis with each window's own field (general boundary data): the
// coefficient kernel on V_k e^{-i omega tau0} (no spectra), then the sinc
// sum over the windows active at each time.
int fhw_synthesize_windows(fhw_ctx* c, const fhw_windows* win, int64_t k_first, int32_t n_win, const void* V,
                           int32_t N_r, const double* times, int32_t N_t, double* u) {
    if (!c) return FHW_E_INVALID;
    int rc = general_plan_check(c, "synthesize_windows");
    if (rc) return rc;
    if (!win || n_win < 0 || N_r < 0 || N_t < 0) return fhw_fail(c, FHW_E_INVALID, "synthesize_windows: bad arguments");
    if (N_r == 0 || N_t == 0) return FHW_OK;
    if (!times || !u || (n_win > 0 && !V)) return fhw_fail(c, FHW_E_INVALID, "synthesize_windows: bad buffers");
    const double H = win->H, tau0 = win->tau0;
    if (!(H > 0) || !isfinite(H) || !isfinite(tau0)) return fhw_fail(c, FHW_E_INVALID, "synthesize_windows: bad windows");
    if (win->track_tol != 0.0) return fhw_fail(c, FHW_E_INVALID, "synthesize_windows: track_tol must be 0");
    const int F = c->prob.F;
    const int M = 2 * F;
    if (M & (M - 1)) return fhw_fail(c, FHW_E_INVALID, "synthesize_windows: 2F must be a power of two");
    if (M > 8192 || (size_t)M * 16 > (size_t)lds_limit(c))
        return fhw_fail(c, FHW_E_INVALID, "synthesize_windows: 2F too large");
    const double W = c->prob.W;
    const double span = 1.5 * H;
    const double P = M_PI / (W / (double)F);
    // windows active at some sample time get a coefficient slot
    std::vector<int32_t> slot((size_t)std::max(n_win, 1), -1);
    std::vector<char> need((size_t)std::max(n_win, 1), 0);
    for (int q = 0; q < N_t; ++q) {
        const double t = times[q];
        if (!isfinite(t)) return fhw_fail(c, FHW_E_INVALID, "synthesize_windows: time not finite");
        const int64_t ka = (int64_t)floor((t - tau0 - P) / span), kb = (int64_t)ceil((t - tau0 + P) / span) + 2;
        for (int64_t k = std::max(ka, k_first); k <= std::min<int64_t>(kb, k_first + n_win - 1); ++k)
            if (fabs(t - span * ((double)k - 1.0) - tau0) <= P) need[k - k_first] = 1;
    }
    // coefficients are computed for the run of windows from the first to the
    // last active one (contiguous in V), inactive ones inside it included
    int32_t q_lo = n_win, q_hi = -1;
    for (int32_t q = 0; q < n_win; ++q)
        if (need[q]) {
            q_lo = std::min(q_lo, q);
            q_hi = q;
        }
    const int count = q_hi >= q_lo ? q_hi - q_lo + 1 : 0;
    for (int32_t q = q_lo; q <= q_hi; ++q) slot[q] = q - q_lo;
    size_t o_t = 0;
    size_t o_s = align_up(o_t + (size_t)N_t * 8, 256);
    size_t o_c = align_up(o_s + slot.size() * 4, 256);
    size_t total = align_up(o_c + (size_t)count * N_r * M * 8, 256);
    rc = fhw_ensure_scratch(c, total);
    if (rc) return rc;
    char* sb = (char*)c->scratch;
    FHW_HIP(c, hipMemcpyAsync(sb + o_t, times, (size_t)N_t * 8, hipMemcpyHostToDevice, c->stream));
    FHW_HIP(c, hipMemcpyAsync(sb + o_s, slot.data(), slot.size() * 4, hipMemcpyHostToDevice, c->stream));
    c->trk_pairs = (int64_t)count * N_r;
    c->trk_active = c->trk_pairs;
    if (count == 0) {
        FHW_HIP(c, hipMemsetAsync(u, 0, sizeof(double) * (size_t)N_r * N_t, c->stream));
    } else {
        const int64_t vq = (int64_t)N_r * M;
        STAGE(c, FHW_STAGE_COEFFS, launch_fourier_coeffs(c->stream, nullptr, count, (const zd*)V + q_lo * vq, N_r, W, F,
                                                         tau0, nullptr, (double*)(sb + o_c), nullptr, nullptr,
                                                         nullptr, nullptr, 0.0, vq));
        STAGE(c, FHW_STAGE_SYNTH, launch_synth(c->stream, sb + o_c, (const int32_t*)(sb + o_s), k_first,
                                               k_first + n_win - 1, count, N_r, (const double*)(sb + o_t), N_t, W, F,
                                               H, tau0, u, nullptr, nullptr, 0.0));
    }
    FHW_HIP(c, hipStreamSynchronize(c->stream));
    return FHW_OK;
}

// 2D time samples with the low-frequency decomposition: window spectra at the
// smooth grid of [omega_c, W] and at the graded nodes, the continuation's
// Fourier coefficients and the Filon-Clenshaw-Curtis data per (window,
// point), then every (point, time) summed over all windows (lowfreq.hip).
// The low-frequency synthesis for windows k_lo .. k_lo + K - 1: the
// continuation coefficients and Filon-Clenshaw-Curtis data per (window,
// point), then every (point, time) summed over all windows.  sig != NULL: the
// plane-path form, F_k = B_k V with the window spectra of the signal; sig ==
// NULL: each window's own fields (V + q vq, Vs + q vsq), F_k = V_k.
static int lowfreq_synth_impl(fhw_ctx* c, const char* what, const fhw_signal* sig, int64_t k_lo, int K, double H,
                              double tau0, const void* V, const void* V_sing, int64_t vq, int64_t vsq, int32_t N_r,
                              const double* times, int32_t N_t, double* u) {
    const fhw_problem& p = c->prob;
    const int F = p.F, M = p.lf_M, nc = p.lf_N, jc = p.lf_jc;
    const int n = F - jc + 1, L = n + lf_fc_points();
    const size_t lds_coef = (size_t)2 * L * 16, lds_syn = ((size_t)2 * L + (size_t)M * 3 * (nc + 1)) * 16;
    if (n > lf_max_points() || lds_coef > 65536 || lds_syn > 65536)
        return fhw_fail(c, FHW_E_INVALID, std::string(what) + ": F - lf_jc + 1 too large for the kernels' 64 KiB of LDS");
    if (K <= 0) {
        FHW_HIP(c, hipMemsetAsync(u, 0, sizeof(double) * (size_t)N_r * N_t, c->stream));
        FHW_HIP(c, hipStreamSynchronize(c->stream));
        return FHW_OK;
    }
    std::vector<int64_t> klist(K);
    for (int q = 0; q < K; ++q) klist[q] = k_lo + q;
    const double h = p.W / (double)F;
    const int n_om = n + M * nc + 1;
    std::vector<double> om(n_om);
    for (int i = 0; i < n; ++i) om[i] = c->lf_omega_c + h * (double)i;
    for (int g = 0; g <= M * nc; ++g) om[n + g] = c->lf_nodes[g];
    // moments of x^p against T_k on [-1, 1]: row 0 from int T_k = 2/(1 - k^2)
    // (even k), then x T_k = (T_{k+1} + T_{|k-1|}) / 2
    const int PT = lf_taylor_terms();
    const int KT = nc + PT + 1;
    std::vector<double> Sp(KT, 0.0), Sn(KT, 0.0), tay((size_t)(nc + 1) * PT);
    for (int k = 0; k < KT; ++k) Sp[k] = (k % 2 == 0) ? 2.0 / (1.0 - (double)k * (double)k) : 0.0;
    for (int pw = 0; pw < PT; ++pw) {
        for (int k = 0; k <= nc; ++k) tay[(size_t)k * PT + pw] = Sp[k];
        for (int k = 0; k + 1 < KT; ++k) Sn[k] = 0.5 * (Sp[k + 1] + Sp[k == 0 ? 1 : k - 1]);
        std::swap(Sp, Sn);
    }
    size_t o_t = 0;
    size_t o_k = align_up(o_t + (size_t)N_t * 8, 256);
    size_t o_om = align_up(o_k + (size_t)K * 8, 256);
    size_t o_mu = align_up(o_om + (size_t)n_om * 8, 256);
    size_t o_ty = align_up(o_mu + (size_t)(M + 1) * 8, 256);
    size_t o_B = align_up(o_ty + tay.size() * 8, 256);
    size_t o_cf = align_up(o_B + (sig ? (size_t)K * n_om * 16 : 0), 256);
    size_t o_ch = align_up(o_cf + (size_t)K * N_r * L * 16, 256);
    size_t total = align_up(o_ch + (size_t)K * N_r * M * 3 * (nc + 1) * 16, 256);
    int rc = fhw_ensure_scratch(c, total);
    if (rc) return rc;
    char* sb = (char*)c->scratch;
    FHW_HIP(c, hipMemcpyAsync(sb + o_t, times, (size_t)N_t * 8, hipMemcpyHostToDevice, c->stream));
    FHW_HIP(c, hipMemcpyAsync(sb + o_k, klist.data(), (size_t)K * 8, hipMemcpyHostToDevice, c->stream));
    FHW_HIP(c, hipMemcpyAsync(sb + o_om, om.data(), (size_t)n_om * 8, hipMemcpyHostToDevice, c->stream));
    FHW_HIP(c, hipMemcpyAsync(sb + o_mu, c->lf_mu.data(), (size_t)(M + 1) * 8, hipMemcpyHostToDevice, c->stream));
    FHW_HIP(c, hipMemcpyAsync(sb + o_ty, tay.data(), tay.size() * 8, hipMemcpyHostToDevice, c->stream));
    if (sig)
        STAGE(c, FHW_STAGE_SPECTRA, launch_window_spectra_at(c->stream, sig->f, sig->n, sig->t0, sig->dt, H,
                                                             (const int64_t*)(sb + o_k), K, (const double*)(sb + o_om),
                                                             n_om, sb + o_B));
    STAGE(c, FHW_STAGE_COEFFS, launch_lf_coeffs(c->stream, sig ? sb + o_B : nullptr, (const double*)(sb + o_om), n_om,
                                                V, V_sing, N_r, F, jc, n, M, nc, tau0, K, sb + o_cf, sb + o_ch, vq,
                                                vsq));
    STAGE(c, FHW_STAGE_SYNTH, launch_lf_synth(c->stream, sb + o_cf, sb + o_ch, (const int64_t*)(sb + o_k), K,
                                              (const double*)(sb + o_mu), (const double*)(sb + o_ty),
                                              (const double*)(sb + o_t), N_t, N_r, n, M, nc, h, c->lf_omega_c, H,
                                              tau0, u));
    FHW_HIP(c, hipStreamSynchronize(c->stream));
    c->trk_pairs = (int64_t)K * N_r;
    c->trk_active = c->trk_pairs;
    return FHW_OK;
}

int fhw_synthesize_lowfreq(fhw_ctx* c, const fhw_signal* sig, const fhw_windows* win, const void* V,
                           const void* V_sing, int32_t N_r, const double* times, int32_t N_t, double* u) {
    if (!c) return FHW_E_INVALID;
    if (!c->planned) return fhw_fail(c, FHW_E_STATE, "synthesize_lowfreq: no plan");
    if (c->lf_extra <= 0)
        return fhw_fail(c, FHW_E_STATE, "synthesize_lowfreq: the plan has no graded low-frequency nodes");
    if (!sig || !win || N_r < 0 || N_t < 0) return fhw_fail(c, FHW_E_INVALID, "synthesize_lowfreq: bad arguments");
    if (N_r == 0 || N_t == 0) return FHW_OK;
    if (!V || !V_sing || !times || !u || !sig->f || sig->n < 2 || !(sig->dt > 0) || !isfinite(sig->t0))
        return fhw_fail(c, FHW_E_INVALID, "synthesize_lowfreq: bad signal or buffers");
    const double H = win->H, tau0 = win->tau0;
    if (!(H > 0) || !isfinite(H) || !isfinite(tau0) || win->track_tol != 0.0)
        return fhw_fail(c, FHW_E_INVALID, "synthesize_lowfreq: bad windows (track_tol must be 0)");
    if (N_r > 65535) return fhw_fail(c, FHW_E_INVALID, "synthesize_lowfreq: at most 65535 points");
    for (int q = 0; q < N_t; ++q)
        if (!isfinite(times[q])) return fhw_fail(c, FHW_E_INVALID, "synthesize_lowfreq: time not finite");
    int64_t k_lo, k_hi;
    signal_windows(sig, H, &k_lo, &k_hi);
    const int K = k_hi >= k_lo ? (int)(k_hi - k_lo + 1) : 0;
    return lowfreq_synth_impl(c, "synthesize_lowfreq", sig, k_lo, K, H, tau0, V, V_sing, 0, 0, N_r, times, N_t, u);
}

int fhw_synthesize_windows_lowfreq(fhw_ctx* c, const fhw_windows* win, int64_t k_first, int32_t n_win,
                                   const void* V, const void* V_sing, int32_t N_r, const double* times, int32_t N_t,
                                   double* u) {
    if (!c) return FHW_E_INVALID;
    int rc = general_plan_check(c, "synthesize_windows_lowfreq");
    if (rc) return rc;
    if (c->lf_extra <= 0)
        return fhw_fail(c, FHW_E_STATE, "synthesize_windows_lowfreq: the plan has no graded low-frequency nodes");
    if (!win || n_win < 0 || N_r < 0 || N_t < 0)
        return fhw_fail(c, FHW_E_INVALID, "synthesize_windows_lowfreq: bad arguments");
    if (N_r == 0 || N_t == 0) return FHW_OK;
    if (!times || !u || (n_win > 0 && (!V || !V_sing)))
        return fhw_fail(c, FHW_E_INVALID, "synthesize_windows_lowfreq: bad buffers");
    const double H = win->H, tau0 = win->tau0;
    if (!(H > 0) || !isfinite(H) || !isfinite(tau0) || win->track_tol != 0.0)
        return fhw_fail(c, FHW_E_INVALID, "synthesize_windows_lowfreq: bad windows (track_tol must be 0)");
    if (N_r > 65535) return fhw_fail(c, FHW_E_INVALID, "synthesize_windows_lowfreq: at most 65535 points");
    for (int q = 0; q < N_t; ++q)
        if (!isfinite(times[q])) return fhw_fail(c, FHW_E_INVALID, "synthesize_windows_lowfreq: time not finite");
    const int64_t vq = (int64_t)N_r * 2 * c->prob.F, vsq = (int64_t)N_r * (c->lf_extra + 2);
    return lowfreq_synth_impl(c, "synthesize_windows_lowfreq", nullptr, k_first, n_win, H, tau0, V, V_sing, vq, vsq,
                              N_r, times, N_t, u);
}

// Time samples on the uniform grid t_n = t_first + n t_step by the fast scaled
// convolution: the windows, spectra, coefficients and active sets of
// fhw_synthesize, then per window and point the sum over m by an L-point FFT
// and a chirp-z convolution (frft.hip) instead of the direct sinc sum.
int fhw_synthesize_uniform(fhw_ctx* c, const fhw_signal* sig, const fhw_windows* win, const void* V, int32_t N_r,
                           double t_first, double t_step, int32_t N_t, int32_t L, double* u) {
    if (!c) return FHW_E_INVALID;
    if (!c->planned) return fhw_fail(c, FHW_E_STATE, "synthesize_uniform: no plan");
    if (c->prob.j_first != 0 || c->system_plan)
        return fhw_fail(c, FHW_E_STATE, "synthesize_uniform: the plan is a band or a list of systems (no DFT grid)");
    if (!sig || !win || N_r < 0 || N_t < 0) return fhw_fail(c, FHW_E_INVALID, "synthesize_uniform: bad arguments");
    if (N_r == 0 || N_t == 0) return FHW_OK;
    if (!V || !u || !sig->f || sig->n < 2 || !(sig->dt > 0) || !isfinite(sig->t0))
        return fhw_fail(c, FHW_E_INVALID, "synthesize_uniform: bad signal or buffers");
    if (!isfinite(t_first) || !(t_step > 0) || !isfinite(t_step))
        return fhw_fail(c, FHW_E_INVALID, "synthesize_uniform: bad time grid");
    const double H = win->H, tau0 = win->tau0, ttol = win->track_tol;
    if (!(H > 0) || !isfinite(H) || !isfinite(tau0))
        return fhw_fail(c, FHW_E_INVALID, "synthesize_uniform: bad windows");
    if (!(ttol >= 0) || !isfinite(ttol))
        return fhw_fail(c, FHW_E_INVALID, "synthesize_uniform: track_tol must be >= 0");
    const bool track = ttol > 0;
    if (N_r > 65535) return fhw_fail(c, FHW_E_INVALID, "synthesize_uniform: at most 65535 points");
    const int F = c->prob.F;
    const int M = 2 * F;
    if (M & (M - 1)) return fhw_fail(c, FHW_E_INVALID, "synthesize_uniform: 2F must be a power of two");
    const int qmax = frft_max_q(lds_limit(c));
    if (L == 0) L = std::max(2 * M, 8);
    if (L < 2 * M || L < 8 || (L & (L - 1)) || 2 * L > qmax)
        return fhw_fail(c, FHW_E_INVALID, "synthesize_uniform: L must be a power of two with max(4F, 8) <= L <= " +
                                              std::to_string(qmax / 2));
    const double W = c->prob.W;
    const double span = 1.5 * H;
    const double P = M_PI / (W / (double)F);
    const double beta = W * t_step / M_PI;
    int64_t k_lo, k_hi;
    signal_windows(sig, H, &k_lo, &k_hi);
    // active grid range of each window, by the same test as the direct sum
    struct wrange { int64_t k; int64_t a, b; };
    std::vector<wrange> wr;
    auto tn = [&](int64_t n) {
        const double prod = (double)n * t_step;
        return t_first + prod;
    };
    for (int64_t k = k_lo; k <= k_hi; ++k) {
        const double sk = 1.5 * H * ((double)k - 1.0);
        const double lo = (sk + tau0 - P - t_first) / t_step, hi = (sk + tau0 + P - t_first) / t_step;
        if (!(hi >= -2.0) || !(lo <= (double)N_t + 1.0)) continue;
        int64_t a = std::max<int64_t>(0, (int64_t)floor(std::max(lo, -2.0)) - 1);
        int64_t b = std::min<int64_t>(N_t - 1, (int64_t)ceil(std::min(hi, (double)N_t + 1.0)) + 1);
        while (a <= b && !(fabs(tn(a) - sk - tau0) <= P)) ++a;
        while (b >= a && !(fabs(tn(b) - sk - tau0) <= P)) --b;
        if (a <= b) wr.push_back({k, a, b});
    }
    const int count = (int)wr.size();
    int64_t nk_max = 1;
    for (const wrange& w : wr) nk_max = std::max(nk_max, w.b - w.a + 1);
    int Q = L;
    while (Q < qmax && (int64_t)Q < (int64_t)L + nk_max - 1) Q <<= 1;
    const int NC = Q - L + 1;
    // windows k and k + j overlap in time iff j span <= 2P: passes of windows
    // k mod NP hold disjoint time ranges
    const double np_d = floor(2.0 * P / span) + 1.0;
    const int64_t NP = np_d < 4e18 ? (int64_t)np_d : INT64_MAX;
    std::vector<std::pair<int64_t, int>> order(count);   // (pass, slot), windows of one pass together
    for (int q = 0; q < count; ++q) order[q] = {((wr[q].k % NP) + NP) % NP, q};
    std::stable_sort(order.begin(), order.end(),
                     [](const std::pair<int64_t, int>& x, const std::pair<int64_t, int>& y) { return x.first < y.first; });
    std::vector<fhw_frft_chunk> chunks;
    std::vector<int32_t> pass_first;   // first chunk of each non-empty pass, then the total
    for (int i = 0; i < count; ++i) {
        if (i == 0 || order[i].first != order[i - 1].first) pass_first.push_back((int32_t)chunks.size());
        const int q = order[i].second;
        const wrange& w = wr[q];
        const double sk = 1.5 * H * ((double)w.k - 1.0);
        for (int64_t n0 = w.a; n0 <= w.b; n0 += NC) {
            fhw_frft_chunk ch;
            ch.slot = q;
            ch.n0 = (int32_t)n0;
            ch.n = (int32_t)std::min<int64_t>(NC, w.b - n0 + 1);
            ch.pad = 0;
            ch.xs = W * (tn(n0) - sk - tau0) / M_PI;
            chunks.push_back(ch);
        }
    }
    pass_first.push_back((int32_t)chunks.size());
    // scratch layout: klist | B | c (real parts) | chirp spectrum | chirps | chunks | tracking
    size_t o_k = 0;
    size_t o_B = align_up(o_k + (size_t)std::max(count, 1) * 8, 256);
    size_t o_c = align_up(o_B + (size_t)count * M * 16, 256);
    size_t o_hs = align_up(o_c + (size_t)count * N_r * M * 8, 256);
    size_t o_ci = align_up(o_hs + (size_t)Q * 16, 256);
    size_t o_co = align_up(o_ci + (size_t)L * 16, 256);
    size_t o_ch = align_up(o_co + (size_t)NC * 16, 256);
    size_t o_bnd = align_up(o_ch + std::max<size_t>(1, chunks.size()) * sizeof(fhw_frft_chunk), 256);
    size_t o_max = align_up(o_bnd + (size_t)count * N_r * 8, 256);   // tracking bounds, their maxima
    size_t o_wm = align_up(o_max + 16, 256);                           // window maxima
    size_t total = align_up(o_wm + (size_t)std::max(count, 1) * 8, 256);
    int rc = fhw_ensure_scratch(c, total);
    if (rc) return rc;
    char* sb = (char*)c->scratch;
    FHW_HIP(c, hipMemsetAsync(u, 0, sizeof(double) * (size_t)N_r * N_t, c->stream));
    c->trk_pairs = (int64_t)count * N_r;
    c->trk_active = c->trk_pairs;
    if (count == 0) return FHW_OK;
    std::vector<int64_t> klist(count);
    for (int q = 0; q < count; ++q) klist[q] = wr[q].k;
    FHW_HIP(c, hipMemcpyAsync(sb + o_k, klist.data(), klist.size() * 8, hipMemcpyHostToDevice, c->stream));
    FHW_HIP(c, hipMemcpyAsync(sb + o_ch, chunks.data(), chunks.size() * sizeof(fhw_frft_chunk), hipMemcpyHostToDevice,
                              c->stream));
    STAGE(c, FHW_STAGE_SPECTRA, launch_window_spectra(c->stream, sig->f, sig->n, sig->t0, sig->dt, H, 0,
                                                      (const int64_t*)(sb + o_k), count, W, F, sb + o_B));
    double* bnd = track ? (double*)(sb + o_bnd) : nullptr;
    unsigned long long* gmax = track ? (unsigned long long*)(sb + o_max) : nullptr;
    if (track) FHW_HIP(c, hipMemsetAsync(gmax, 0, 16, c->stream));   // gmax and the window-level max
    STAGE(c, FHW_STAGE_COEFFS, launch_fourier_coeffs(c->stream, sb + o_B, count, V, N_r, W, F, tau0, nullptr,
                                                     (double*)(sb + o_c), bnd, gmax, (double*)(sb + o_wm),
                                                     gmax ? gmax + 1 : nullptr, ttol));
    STAGE(c, FHW_STAGE_SYNTH, launch_frft_setup(c->stream, L, NC, Q, beta, sb + o_hs, sb + o_ci, sb + o_co));
    const fhw_frft_chunk* d_ch = (const fhw_frft_chunk*)(sb + o_ch);
    for (size_t ps = 0; ps + 1 < pass_first.size(); ++ps) {
        const int32_t n = pass_first[ps + 1] - pass_first[ps];
        if (n == 0) continue;
        STAGE(c, FHW_STAGE_SYNTH, launch_frft(c->stream, (const double*)(sb + o_c), d_ch + pass_first[ps], n, N_r, F,
                                              L, Q, beta, W / M_PI, sb + o_hs, sb + o_ci, sb + o_co, u,
                                              N_t, bnd, gmax, ttol));
    }
    FHW_HIP(c, hipStreamSynchronize(c->stream));
    if (track) {
        // pairs kept, for fhw_synth_active_pairs
        std::vector<double> b((size_t)count * N_r);
        unsigned long long mx = 0;
        if (int rc_ = copy_d2h(c, b.data(), bnd, 8 * b.size())) return rc_;
        if (int rc_ = copy_d2h(c, &mx, gmax, 8)) return rc_;
        double gm;
        memcpy(&gm, &mx, 8);
        int64_t n = 0;
        for (double v : b) n += v > ttol * gm ? 1 : 0;
        c->trk_active = n;
    }
    return FHW_OK;
}

// The whole hot path of a single-curve plane-wave plan in one call (steps
// F1-F5, T0-T6): densities, field at the observation points (V(r, 0) = 1,
// the plane-wave limit) and the time samples, in the order of the separate
// calls and with the same kernels.
int fhw_run(fhw_ctx* c, const fhw_signal* sig, const fhw_windows* win, const double* obs, int32_t N_r,
            const double* times, int32_t N_t, void* psi, void* V, double* u, double* resid, int32_t* sweeps) {
    if (!c) return FHW_E_INVALID;
    if (!c->planned) return fhw_fail(c, FHW_E_STATE, "run: no plan");
    if (c->curves.size() != 1) return fhw_fail(c, FHW_E_INVALID, "run: plans of one curve only");
    int rc = fhw_solve_densities(c, psi, resid, sweeps, 0);
    if (rc) return rc;
    rc = fhw_eval_field(c, psi, obs, N_r, 1.0, V);
    if (rc) return rc;
    return fhw_synthesize(c, sig, win, V, N_r, times, N_t, u);
}

int fhw_synth_active_pairs(fhw_ctx* c, int64_t* pairs, int64_t* active) {
    if (!c) return FHW_E_INVALID;
    if (!pairs || !active) return fhw_fail(c, FHW_E_INVALID, "synth_active_pairs: null output");
    if (c->trk_pairs < 0) return fhw_fail(c, FHW_E_STATE, "synth_active_pairs: no synthesis yet");
    *pairs = c->trk_pairs;
    *active = c->trk_active;
    return FHW_OK;
}

// ----------------------------- stage entry points ---------------------------

int fhw_geometry(fhw_ctx* c, int32_t N, double* geom) {
    if (!c) return FHW_E_INVALID;
    if (!c->planned) return fhw_fail(c, FHW_E_STATE, "geometry: no plan");
    if (N < 4 || (N & 1) || !geom) return fhw_fail(c, FHW_E_INVALID, "geometry: bad arguments");
    STAGE(c, FHW_STAGE_GEOMETRY, launch_geometry(c->stream, c->curves[0].d_curve, c->curves[0].degree, N, geom));
    FHW_HIP(c, hipStreamSynchronize(c->stream));
    return FHW_OK;
}

int fhw_kress_weights(fhw_ctx* c, int32_t N, double* R, double* logtab) {
    if (!c) return FHW_E_INVALID;
    if (N < 4 || (N & 1) || !R || !logtab) return fhw_fail(c, FHW_E_INVALID, "kress: bad arguments");
    STAGE(c, FHW_STAGE_KRESS, launch_kress(c->stream, N, R, logtab));
    FHW_HIP(c, hipStreamSynchronize(c->stream));
    return FHW_OK;
}

int fhw_assemble(fhw_ctx* c, int32_t j0, int32_t count, void* A, const int64_t* A_off, void* g,
                 const int64_t* g_off) {
    if (!c) return FHW_E_INVALID;
    if (!c->planned) return fhw_fail(c, FHW_E_STATE, "assemble: no plan");
    if (j0 < 0 || count < 0 || j0 + count > (int)c->Ns.size() || (count > 0 && (!A || !A_off || !g || !g_off)))
        return fhw_fail(c, FHW_E_INVALID, "assemble: bad arguments");
    if (count == 0) return FHW_OK;
    std::vector<fhw_assemble_item> items(count);
    std::vector<int64_t> pre(count + 1);
    int64_t blk = 0;
    for (int q = 0; q < count; ++q) {
        int j = j0 + q;
        const fhw_geom_entry& ge = c->geoms[fhw_geom_key(c->sys_curve[j], c->Ns[j])];
        items[q] = fhw_assemble_item{ge.geom, ge.R, ge.logtab, A_off[q], g_off[q], c->Ns[j], c->kappa[j], c->eta[j]};
        pre[q] = blk;
        blk += assemble_blocks_for(c->Ns[j]);
    }
    pre[count] = blk;
    size_t oi = 0, op = align_up(sizeof(fhw_assemble_item) * count, 256);
    int rc = fhw_ensure_scratch(c, op + 8 * (count + 1));
    if (rc) return rc;
    char* sb = (char*)c->scratch;
    FHW_HIP(c, hipMemcpyAsync(sb + oi, items.data(), sizeof(fhw_assemble_item) * count, hipMemcpyHostToDevice,
                              c->stream));
    FHW_HIP(c, hipMemcpyAsync(sb + op, pre.data(), 8 * (count + 1), hipMemcpyHostToDevice, c->stream));
    STAGE(c, FHW_STAGE_ASSEMBLE, launch_assemble_blocks(c->stream, (const fhw_assemble_item*)(sb + oi), (const int64_t*)(sb + op), count,
                                      blk, c->prob.direction[0], c->prob.direction[1], A, nullptr, g,
                                      c->prob.formulation == FHW_FORM_COMBINED));
    FHW_HIP(c, hipStreamSynchronize(c->stream));
    return FHW_OK;
}

static int upload_batch(fhw_ctx* c, int32_t batch, const int32_t* N, const int64_t* a_off, const int64_t* piv_off,
                        const int64_t* linv_off, const int64_t* v_off, const std::vector<int32_t>* prefix,
                        fhw_batch_dev& bd, int32_t** d_prefix) {
    size_t o[7];
    size_t pos = 0;
    auto nxt = [&](size_t bytes) { size_t r = align_up(pos, 256); pos = r + bytes; return r; };
    o[0] = nxt(4 * batch);
    o[1] = nxt(8 * batch);
    o[2] = nxt(8 * batch);
    o[3] = nxt(8 * batch);
    o[4] = nxt(8 * batch);
    o[5] = nxt(prefix ? 4 * std::max<size_t>(1, prefix->size()) : 4);
    o[6] = nxt(16);   // status
    int rc = fhw_ensure_scratch(c, pos);
    if (rc) return rc;
    char* sb = (char*)c->scratch;
    std::vector<int64_t> zero(batch, 0);
    FHW_HIP(c, hipMemcpyAsync(sb + o[0], N, 4 * batch, hipMemcpyHostToDevice, c->stream));
    FHW_HIP(c, hipMemcpyAsync(sb + o[1], a_off, 8 * batch, hipMemcpyHostToDevice, c->stream));
    FHW_HIP(c, hipMemcpyAsync(sb + o[2], piv_off ? piv_off : zero.data(), 8 * batch, hipMemcpyHostToDevice, c->stream));
    FHW_HIP(c, hipMemcpyAsync(sb + o[3], linv_off ? linv_off : zero.data(), 8 * batch, hipMemcpyHostToDevice,
                              c->stream));
    FHW_HIP(c, hipMemcpyAsync(sb + o[4], v_off ? v_off : zero.data(), 8 * batch, hipMemcpyHostToDevice, c->stream));
    if (prefix && !prefix->empty())
        FHW_HIP(c, hipMemcpyAsync(sb + o[5], prefix->data(), 4 * prefix->size(), hipMemcpyHostToDevice, c->stream));
    FHW_HIP(c, hipMemsetAsync(sb + o[6], 0, 16, c->stream));
    bd = fhw_batch_dev{(const int32_t*)(sb + o[0]), (const int64_t*)(sb + o[1]), (const int64_t*)(sb + o[2]),
                       (const int64_t*)(sb + o[3]), (const int64_t*)(sb + o[4]), batch};
    if (d_prefix) *d_prefix = (int32_t*)(sb + o[5]);
    // status word at o[6]
    c->status_len = o[6];
    FHW_HIP(c, hipStreamSynchronize(c->stream));
    return FHW_OK;
}

int fhw_lu_factor(fhw_ctx* c, int32_t batch, const int32_t* N, const int64_t* A_off, void* A, const int64_t* piv_off,
                  int32_t* piv, const int64_t* linv_off, void* linv, int32_t precision) {
    if (!c) return FHW_E_INVALID;
    if (batch < 0 || (batch > 0 && (!N || !A_off || !A || !piv_off || !piv || !linv_off || !linv)))
        return fhw_fail(c, FHW_E_INVALID, "lu_factor: bad arguments");
    if (precision != FHW_FP64 && precision != FHW_FP32_REFINE)
        return fhw_fail(c, FHW_E_INVALID, "lu_factor: unknown precision");
    if (batch == 0) return FHW_OK;
    for (int q = 0; q < batch; ++q)
        if (N[q] < 1 || N[q] > 4096) return fhw_fail(c, FHW_E_INVALID, "lu_factor: need 1 <= N <= 4096");
    fhw_lu_sched sch;
    lu_build_schedule(N, batch, sch);
    fhw_batch_dev bd;
    int32_t* d_prefix = nullptr;
    int rc = upload_batch(c, batch, N, A_off, piv_off, linv_off, nullptr, &sch.prefix, bd, &d_prefix);
    if (rc) return rc;
    int32_t* d_st = (int32_t*)((char*)c->scratch + c->status_len);
    FHW_HIP(c, launch_lu_factor(c->stream, bd, sch, d_prefix, A, piv, linv, d_st, precision, &c->prof));
    FHW_HIP(c, hipStreamSynchronize(c->stream));
    int32_t st = 0;
    if (int rc_ = copy_d2h(c, &st, d_st, 4)) return rc_;
    if (st) return fhw_fail(c, FHW_E_SINGULAR, "lu_factor: exactly zero pivot");
    return FHW_OK;
}

int fhw_lu_solve(fhw_ctx* c, int32_t batch, const int32_t* N, const int64_t* A_off, const void* LU,
                 const int64_t* piv_off, const int32_t* piv, const int64_t* linv_off, const void* linv,
                 const int64_t* b_off, void* b, int32_t precision) {
    if (!c) return FHW_E_INVALID;
    if (batch < 0 || (batch > 0 && (!N || !A_off || !LU || !piv_off || !piv || !linv_off || !linv || !b_off || !b)))
        return fhw_fail(c, FHW_E_INVALID, "lu_solve: bad arguments");
    if (precision != FHW_FP64 && precision != FHW_FP32_REFINE)
        return fhw_fail(c, FHW_E_INVALID, "lu_solve: unknown precision");
    if (batch == 0) return FHW_OK;
    int32_t maxN = 0;
    for (int q = 0; q < batch; ++q) {
        if (N[q] < 1 || N[q] > 4096) return fhw_fail(c, FHW_E_INVALID, "lu_solve: need 1 <= N <= 4096");
        maxN = std::max(maxN, N[q]);
    }
    if ((size_t)maxN * 16 + FHW_SOLVE_STATIC_LDS > (size_t)lds_limit(c)) return fhw_fail(c, FHW_E_INVALID, "lu_solve: N too large");
    fhw_batch_dev bd;
    int rc = upload_batch(c, batch, N, A_off, piv_off, linv_off, b_off, nullptr, bd, nullptr);
    if (rc) return rc;
    STAGE(c, FHW_STAGE_SOLVE, launch_lu_solve(c->stream, bd, maxN, LU, piv, linv, b, nullptr, precision));
    FHW_HIP(c, hipStreamSynchronize(c->stream));
    return FHW_OK;
}

int fhw_window_spectra(fhw_ctx* c, const fhw_signal* sig, const fhw_windows* win, int64_t k_first, int32_t count,
                       void* B) {
    if (!c) return FHW_E_INVALID;
    if (!c->planned) return fhw_fail(c, FHW_E_STATE, "window_spectra: no plan");
    if (c->system_plan) return fhw_fail(c, FHW_E_STATE, "window_spectra: the plan is a list of systems (no DFT grid)");
    if (!sig || !win || count < 0 || (count > 0 && (!B || !sig->f)) || sig->n < 2 || !(sig->dt > 0) || !(win->H > 0))
        return fhw_fail(c, FHW_E_INVALID, "window_spectra: bad arguments");
    STAGE(c, FHW_STAGE_SPECTRA, launch_window_spectra(c->stream, sig->f, sig->n, sig->t0, sig->dt, win->H, k_first, nullptr, count,
                                     c->prob.W, c->prob.F, B));
    FHW_HIP(c, hipStreamSynchronize(c->stream));
    return FHW_OK;
}

int fhw_fourier_coefficients(fhw_ctx* c, const void* B, int32_t count, const void* V, int32_t N_r, double tau0,
                             void* cc) {
    if (!c) return FHW_E_INVALID;
    if (!c->planned) return fhw_fail(c, FHW_E_STATE, "fourier_coefficients: no plan");
    if (c->system_plan) return fhw_fail(c, FHW_E_STATE, "fourier_coefficients: the plan is a list of systems (no DFT grid)");
    const int M = 2 * c->prob.F;
    if (M & (M - 1)) return fhw_fail(c, FHW_E_INVALID, "fourier_coefficients: 2F must be a power of two");
    if (M > 8192 || (size_t)M * 16 > (size_t)lds_limit(c))
        return fhw_fail(c, FHW_E_INVALID, "fourier_coefficients: 2F too large");
    if (count < 0 || N_r < 0 || ((count > 0 && N_r > 0) && (!B || !V || !cc)) || !isfinite(tau0))
        return fhw_fail(c, FHW_E_INVALID, "fourier_coefficients: bad arguments");
    STAGE(c, FHW_STAGE_COEFFS, launch_fourier_coeffs(c->stream, B, count, V, N_r, c->prob.W, c->prob.F, tau0, cc,
                                                     nullptr));
    FHW_HIP(c, hipStreamSynchronize(c->stream));
    return FHW_OK;
}

int fhw_hankel01(fhw_ctx* c, const double* z, int64_t n, void* h) {
    if (!c) return FHW_E_INVALID;
    if (n < 0 || (n > 0 && (!z || !h))) return fhw_fail(c, FHW_E_INVALID, "hankel01: bad arguments");
    FHW_HIP(c, launch_hankel01(c->stream, z, n, h));
    FHW_HIP(c, hipStreamSynchronize(c->stream));
    return FHW_OK;
}

}  // extern "C"
