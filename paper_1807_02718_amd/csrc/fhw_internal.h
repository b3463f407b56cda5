// Host-side internals of libfhw: context, plan, and the kernel launchers
// each .hip translation unit provides.
#pragma once
#include <hip/hip_runtime.h>

#include <atomic>
#include <initializer_list>
#include <stdint.h>

#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/fhw.h"

// Outer LU panel width (columns per panel factorization / trailing update).
#define FHW_LU_NB 64
// LDS of the solve kernels beside the N-long solution vector (at most)
#define FHW_SOLVE_STATIC_LDS 20480

struct fhw_batch_dev {
    // device arrays describing a ragged batch of square matrices
    const int32_t* N;         // [batch]
    const int64_t* a_off;     // [batch] element offsets of the (column-major) matrices
    const int64_t* piv_off;   // [batch]
    const int64_t* linv_off;  // [batch]
    const int64_t* v_off;     // [batch] vector offsets
    int32_t batch;
};

struct fhw_geom_entry {
    int32_t N;
    double* geom;    // [9][N]
    double* R;       // [N]
    double* logtab;  // [N]
};

// Per-stage launch timers (HIP events on the context stream).
struct fhw_prof {
    bool on = false;
    struct rec {
        int stage;
        hipEvent_t a, b;
    };
    std::vector<rec> recs;
    std::vector<hipEvent_t> pool;
    int open_stage = -1;
    hipEvent_t open_a = nullptr;
    hipEvent_t take();
    void begin(int stage, hipStream_t s);
    void end(hipStream_t s);
};
// helpers usable with a null profiler
inline void prof_begin(fhw_prof* p, int stage, hipStream_t s) {
    if (p && p->on) p->begin(stage, s);
}
inline void prof_end(fhw_prof* p, hipStream_t s) {
    if (p && p->on) p->end(s);
}

struct fhw_host_curve {
    int32_t degree = 0;
    std::vector<double> cx, sx, cy, sy;
    double length = 0.0;
    double* d_curve = nullptr;         // [4][degree+1] on the device (owned by the curve cache)
    uint64_t fingerprint = 0;
};
// kept across plans (freed by fhw_destroy)
struct fhw_curve_cache_entry {
    std::vector<double> coef;          // cx | sx | cy | sy
    double* d = nullptr;
};
struct fhw_geo_cache_entry {
    fhw_geom_entry e;
};
inline int64_t fhw_geom_key(int curve, int N) { return (int64_t)curve * 65536 + N; }

struct fhw_ctx {
    hipStream_t stream = nullptr;
    size_t budget = 0;
    std::string err;
    int device = 0;

    // plan
    bool planned = false;
    bool factors_resident = false;     // LU of every planned frequency in the workspace
    fhw_problem prob{};
    // systems: curve-major, system s = curve * F + j (frequency j of curve)
    std::vector<fhw_host_curve> curves;
    std::vector<double> kappa, eta;    // [systems]
    std::vector<int32_t> Ns;           // [systems]
    std::vector<int32_t> sys_curve;    // [systems] curve of each system
    bool system_plan = false;          // planned by fhw_plan_systems (no DFT grid)
    std::vector<int64_t> psi_off;      // [systems + 1]
    // graded low-frequency nodes (plans with lf_M > 0): systems F .. F + lf_extra - 1
    int32_t lf_extra = 0;              // lf_M lf_N - 1 (0: none)
    double lf_omega_c = 0.0;
    std::vector<double> lf_mu;         // [lf_M + 1] graded mesh
    std::vector<double> lf_nodes;      // [lf_M lf_N + 1] ascending, 0 .. omega_c
    std::map<int64_t, fhw_geom_entry> geoms;   // the plan's view, key: curve * 65536 + N
    std::map<uint64_t, fhw_curve_cache_entry> curve_cache;                       // by curve fingerprint
    std::map<std::pair<uint64_t, int32_t>, fhw_geo_cache_entry> geo_cache;       // by (fingerprint, N)
    size_t geo_cache_bytes = 0;
    size_t small_cap[7] = {0, 0, 0, 0, 0, 0, 0};   // status, norms, done, sweeps, rpart, rcount, meta

    // solve workspace (one chunk of frequencies)
    int32_t chunk = 0;                 // max frequencies per chunk
    size_t ws_A64 = 0, ws_A32 = 0, ws_linv = 0, ws_piv = 0;   // element counts
    void* A64 = nullptr;               // complex128 matrices
    void* A32 = nullptr;               // complex64 copies (FP32 path)
    void* linv = nullptr;              // inverse diagonal blocks (factor type)
    int32_t* piv = nullptr;
    void* x = nullptr;                 // complex128 boundary data g [FHW_INC_GROUP][chunk vectors]
    void* r = nullptr;                 // complex128 residuals [FHW_INC_GROUP][chunk vectors]
    int64_t ws_vec = 0;                // elements of one incidence's slot in x and r
    int64_t rpart_stride = 0;          // doubles of one incidence's residual partial norms
    // bytes allocated for A64, A32, linv, piv, x, r: these outlive a plan, and
    // a new plan reallocates only the ones it outgrows
    size_t ws_cap[6] = {0, 0, 0, 0, 0, 0};
    void* meta = nullptr;              // per-chunk device metadata
    size_t meta_bytes = 0;
    int32_t* d_status = nullptr;       // [0]: singular flag, [1..]: per-matrix flags
    size_t status_len = 0;
    double* d_norms = nullptr;         // [chunk][2] residual norms
    double* d_rpart = nullptr;         // residual partial norms [FHW_INC_GROUP][chunk][blocks][2]
    int32_t* d_rcount = nullptr;       // residual block counters [FHW_INC_GROUP][chunk] (kept zero)
    int32_t* d_done = nullptr;         // [chunk]
    int32_t* d_sweeps = nullptr;       // [chunk]
    int32_t* d_pending = nullptr;      // systems still above the refinement tolerance after a sweep
    int32_t* h_pending = nullptr;      // its pinned host copy
    void* h_stage = nullptr;           // pinned staging of the status read-backs
    size_t h_stage_bytes = 0;

    fhw_prof prof;
    hipStream_t cap_stream = nullptr;  // graph capture (created on first use, default priority)
    // the last fhw_synthesize's (window, point) pairs, and how many tracking kept
    int64_t trk_pairs = -1;            // -1: no synthesis yet
    int64_t trk_active = 0;

    // generic scratch (synthesis)
    void* scratch = nullptr;
    size_t scratch_bytes = 0;

    // device address of the library's fixed status array on this context's
    // device (fhw_solve_range_noalloc); nullptr if the lookup failed
    void* noalloc = nullptr;
    std::string noalloc_err;
};

int fhw_fail(fhw_ctx* ctx, int code, const std::string& msg);
int fhw_hip_check(fhw_ctx* ctx, hipError_t e, const char* what);
int fhw_ensure_scratch(fhw_ctx* ctx, size_t bytes);
#define FHW_HIP(ctx, call)                                                 \
    do {                                                                   \
        hipError_t _e = (call);                                            \
        if (_e != hipSuccess) return fhw_hip_check((ctx), _e, #call);      \
    } while (0)

// --- geometry.hip -----------------------------------------------------------
hipError_t launch_geometry(hipStream_t s, const double* curve, int32_t degree, int32_t N, double* geom);
hipError_t launch_kress(hipStream_t s, int32_t N, double* R, double* logtab);

// --- assemble.hip -----------------------------------------------------------
struct fhw_assemble_item {
    const double* geom;    // [9][N]
    const double* R;       // [N]
    const double* logtab;  // [N]
    int64_t a_off, g_off;  // element offsets (complex)
    int32_t N;
    double kappa, eta;
};
// write complex128 A (and optionally a complex64 copy A32 at the same offsets)
// and the plane-wave RHS g; d_prefix[q] = first block of item q; combined:
// the combined potential's matrix instead of the direct equation's
hipError_t launch_assemble_blocks(hipStream_t s, const fhw_assemble_item* d_items, const int64_t* d_prefix,
                                  int32_t n_items, int64_t total_blocks, double p1, double p2, void* A,
                                  void* A32, void* g, bool combined = false);
int64_t assemble_blocks_for(int32_t N);
// boundary data of one incidence (FHW_INC_PLANE: v = p; FHW_INC_POINT: v = r0)
// for every item, written at g + g_off
// Runs fn once per device for the given mask (kernel attributes such as the
// dynamic LDS limit are per device).  Contexts on several host threads may
// race here: the first caller runs fn under a lock, and the others wait for
// it before they launch.
inline std::mutex& fhw_attr_mutex() {
    static std::mutex m;
    return m;
}
template <class Fn>
inline void fhw_once_on_device(std::atomic<uint64_t>& mask, Fn&& fn) {
    int dev = 0;
    (void)hipGetDevice(&dev);
    const uint64_t bit = 1ull << (dev & 63);
    if (mask.load(std::memory_order_acquire) & bit) return;
    std::lock_guard<std::mutex> lk(fhw_attr_mutex());
    if (mask.load(std::memory_order_acquire) & bit) return;
    fn();
    mask.fetch_or(bit, std::memory_order_release);
}

// Incidences solved together: one more grid dimension over up to
// FHW_INC_GROUP incidences, each buffer advanced by its stride (elements).
#define FHW_INC_GROUP 16
struct fhw_grp {
    int32_t n = 1;
    int64_t sv = 0, sacc = 0, sflag = 0;      // solve: vector, accumulator; skip / done / sweeps flags
    int64_t sx = 0, sg = 0, sr = 0;           // residual: x, g, r
    int64_t spart = 0, scount = 0, snorm = 0; // residual: partial norms, block counters, norms
};
struct fhw_rhs_group {
    int32_t n;
    int32_t kind[FHW_INC_GROUP];
    double v[FHW_INC_GROUP][2];
};
// boundary data of n incidences (FHW_INC_PLANE: v = p; FHW_INC_POINT: v = r0)
// for every item, incidence q written at g + q sg + g_off
hipError_t launch_rhs(hipStream_t s, const fhw_assemble_item* d_items, int32_t n_items, const fhw_rhs_group& rg,
                      int64_t sg, void* g);

// --- lu.hip -----------------------------------------------------------------
// One launch of the batched factorization.  Panels go in pairs (2q, 2q+1):
// the pair's trailing block is updated once with depth 128 (see lu.hip).
enum { FHW_LU_OP_PANEL = 0, FHW_LU_OP_DIAGINV, FHW_LU_OP_SWAP, FHW_LU_OP_TRSM, FHW_LU_OP_SUB };
struct fhw_lu_op {
    int32_t kind;
    int32_t k0;                          // first column of the op's panel
    int32_t R;                           // PANEL: rows per thread
    int32_t K, roff, rlim, coff, clim;   // SUB: depth; rows k0+roff.., cols k0+coff..; limits (0 = to N)
    int32_t cbeg, ccount;                // SWAP: first column and count (0 = to N)
    int32_t grid;                        // GEMM tiles or SWAP column blocks
    int64_t prefix_off;                  // GEMM: offset of the op's tile prefix in prefix
};
struct fhw_lu_sched {
    // host-built launch schedule for one batched factorization
    int32_t nsteps;
    std::vector<fhw_lu_op> ops;
    std::vector<int32_t> prefix;         // concatenated per-op tile prefix arrays
};
void lu_build_schedule(const int32_t* N, int32_t batch, fhw_lu_sched& sch);
// kernel attributes the factorization needs, set outside any stream capture
void lu_prepare(int precision);
hipError_t launch_lu_factor(hipStream_t s, const fhw_batch_dev& b, const fhw_lu_sched& sch,
                            const int32_t* d_prefix, void* A, int32_t* piv, void* linv,
                            int32_t* d_status, int precision, fhw_prof* prof);
// grp (default: one incidence) gives the incidence count and the strides
// sv (x), sacc (acc), sflag (d_skip)
hipError_t launch_lu_solve(hipStream_t s, const fhw_batch_dev& b, int32_t maxN, const void* LU,
                           const int32_t* piv, const void* linv, void* x, const int32_t* d_skip,
                           int precision, const fhw_grp& grp = fhw_grp());
// as launch_lu_solve, but when acc != NULL adds the solution into acc (same
// offsets) and leaves x holding its input
hipError_t launch_lu_solve_acc(hipStream_t s, const fhw_batch_dev& b, int32_t maxN, const void* LU,
                               const int32_t* piv, const void* linv, void* x, void* acc,
                               const int32_t* d_skip, int precision, const fhw_grp& grp = fhw_grp());
// part: 2 * batch * ceil(maxN/64) doubles of scratch; count: batch ints, zero
// before the first call (each call leaves them zero); per incidence of grp
// at strides spart, scount (x, g, r, norms, done/sweeps: sx, sg, sr, snorm, sflag)
// pending (optional): incremented once per matrix left above tol by this sweep
hipError_t launch_residual_t(hipStream_t s, const fhw_batch_dev& b, int32_t maxN, const void* A64,
                             const void* x, const void* g, void* r, double* part, int32_t* count,
                             double* norms, double tol, int32_t* done, int32_t* sweeps, int sweep,
                             int32_t* pending = nullptr, const fhw_grp& grp = fhw_grp());
hipError_t launch_convert_c128_c64(hipStream_t s, const void* src, void* dst, int64_t n);
// status words of nf (incidence, system) pairs in caller-provided device
// memory: cleared (and *notdone = 0) before the solves; after them resid[j] =
// ||r|| / ||g|| (-1 when refine == 0), sweeps_out[j] (refine_max for a pair
// that never met the tolerance, 0 when refine == 0), *notdone += such pairs
hipError_t launch_status_clear(hipStream_t s, int32_t* done, int32_t* sweeps, int32_t* notdone, int64_t nf);
hipError_t launch_status_finish(hipStream_t s, const int32_t* done, const int32_t* sweeps, const double* norms,
                                int64_t nf, int refine, int refine_max, double* resid, int32_t* sweeps_out,
                                int32_t* notdone);

// --- field.hip --------------------------------------------------------------
struct fhw_field_item {
    const double* geom;
    int64_t psi_off;
    int32_t N;
    double kappa;
    double eta;   // coupling of the system (the combined potential's single-layer weight)
};
hipError_t launch_field(hipStream_t s, const fhw_field_item* d_items, int32_t F, const void* psi,
                        const double* obs, int32_t N_r, double zero_value, void* V);
hipError_t launch_hankel01(hipStream_t s, const double* z, int64_t n, void* h);
// V[r][0] = zero_value, V[r][1 + j] = field of item j: complex128 [N_r][n_items + 1]
// the field of n_blk density blocks by the combined potential (block q at
// psi + q psi_bstride; every item at the same N) into V + q V_bstride, each as
// launch_field writes it with V(r, 0) = zero_value, or with list = true as
// launch_field_list writes it (the F items an explicit list)
hipError_t launch_field_blocks(hipStream_t s, const fhw_field_item* d_items, int32_t F, const void* psi,
                               int64_t psi_bstride, int32_t n_blk, const double* obs, int32_t N_r,
                               double zero_value, void* V, int64_t V_bstride, bool list = false);   // combined potential
// (combined: the combined potential instead of the single layer)
hipError_t launch_field_list(hipStream_t s, const fhw_field_item* d_items, int32_t n_items, const void* psi,
                             const double* obs, int32_t N_r, double zero_value, void* V, bool combined = false);

// --- lowfreq.hip --------------------------------------------------------------
// largest number of smooth-grid frequencies the continuation kernel takes;
// continuation points; Taylor terms of the small-argument moments
int lf_max_points(void);
int lf_fc_points(void);
int lf_taylor_terms(void);
// per (window, point): Fourier coefficients of the continued smooth part
// (cfs [K][N_r][n + FC_C]) and the graded subintervals' Chebyshev data
// (cheb [K][N_r][M][3][nc + 1]); B [K][n_om] at om = smooth grid then the
// M nc + 1 graded nodes; V [N_r][2F]; Vs [N_r][M nc + 1]
// With B == NULL each window has its own fields, window q's at V + q v_qstride
// and Vs + q vs_qstride (general boundary data), and no spectrum factor.
hipError_t launch_lf_coeffs(hipStream_t s, const void* B, const double* om, int n_om, const void* V, const void* Vs,
                            int N_r, int F, int jc, int n, int M, int nc, double tau0, int K, void* cfs, void* cheb,
                            int64_t v_qstride = 0, int64_t vs_qstride = 0);
// u [N_r][N_t] = sum over the K windows of (1/pi) Re (I_+ + I_0); mu [M + 1]
// graded mesh; taylor [nc + 1][40] moments of x^p against T_k
hipError_t launch_lf_synth(hipStream_t s, const void* cfs, const void* cheb, const int64_t* klist, int K,
                           const double* mu, const double* taylor, const double* times, int N_t, int N_r, int n,
                           int M, int nc, double h, double omega_c, double H, double tau0, double* u);

// --- synth.hip --------------------------------------------------------------
hipError_t launch_window_spectra(hipStream_t s, const double* f, int64_t n, double t0, double dt,
                                 double H, int64_t k_first, const int64_t* d_klist, int32_t count,
                                 double W, int32_t F, void* B);
// the same at the n_om frequencies d_om (device), B [count][n_om]
hipError_t launch_window_spectra_at(hipStream_t s, const double* f, int64_t n, double t0, double dt, double H,
                                    const int64_t* d_klist, int32_t count, const double* d_om, int32_t n_om,
                                    void* B);
// c: complex128 [count][N_r][2F]; or, with c == NULL, real parts only into c_re.
// bnd (optional, tracking): [count][N_r] sums of |Re c_m|, their maximum into
// *gmax (as the bits of a double; zero before the call); windows whose
// spectrum max wmax[q] (written here, [count]) is at most tol * (*gwmax)
// (zero before the call) get no coefficients and bound 0.  With B == NULL
// every window has its own field, window q's at V + q v_qstride, and the
// coefficients are those of V e^{-i omega tau0} (no tracking then).
hipError_t launch_fourier_coeffs(hipStream_t s, const void* B, int32_t count, const void* V,
                                 int32_t N_r, double W, int32_t F, double tau0, void* c, double* c_re,
                                 double* bnd = nullptr, unsigned long long* gmax = nullptr,
                                 double* wmax = nullptr, unsigned long long* gwmax = nullptr, double tol = 0.0,
                                 int64_t v_qstride = 0);
// Right-hand sides B of the combined-potential equation from sampled
// Dirichlet data b [n_t][N] (device, real) for windows k_first .. k_first +
// n_win - 1 (window q at g + q sg) and the n_sys items (omega = kappa c)
hipError_t launch_boundary_rhs(hipStream_t s, const double* b, int64_t n_t, int32_t N, double t0, double dt,
                               double H, int64_t k_first, int32_t n_win, double c, const fhw_assemble_item* d_items,
                               int32_t n_sys, int64_t sg, void* g);
// Fast scaled convolution on a uniform time grid (frft.hip).  A chunk is a
// run of n consecutive grid times from index n0 inside one window's active
// range; xs is the kernel argument W (t_{n0} - s_k - tau0) / pi of its first.
struct fhw_frft_chunk {
    int32_t slot;
    int32_t n0;
    int32_t n;
    int32_t pad;
    double xs;
};
// largest power-of-two convolution length Q (<= 8192) whose complex128 buffer
// fits in lds_bytes
int frft_max_q(int lds_bytes);
// the chirp spectrum Hs[Q] and the chirps cin[L], cout[NC] for (L, NC, Q, beta)
hipError_t launch_frft_setup(hipStream_t s, int L, int NC, int Q, double beta, void* Hs, void* cin, void* cout);
// u[r][n0 + i] += scale d(xs + beta i), i < n, for every chunk and point r;
// chunks of one launch must cover disjoint time ranges.  bnd != NULL
// (tracking): window slot sl is skipped at point r when
// bnd[sl N_r + r] <= tol * (*gmax)
hipError_t launch_frft(hipStream_t s, const double* c_re, const fhw_frft_chunk* d_chunks, int32_t n_chunks,
                       int32_t N_r, int32_t F, int32_t L, int32_t Q, double beta, double scale, const void* Hs,
                       const void* cin, const void* cout, double* u, int64_t N_t,
                       const double* bnd = nullptr, const unsigned long long* gmax = nullptr, double tol = 0.0);
// bnd != NULL: skip window slot sl at point r when bnd[sl N_r + r] <= tol * (*gmax)
hipError_t launch_synth(hipStream_t s, const void* c, const int32_t* d_slot, int64_t k_min,
                        int64_t k_max, int32_t n_slots, int32_t N_r, const double* times,
                        int32_t N_t, double W, int32_t F, double H, double tau0, double* u,
                        const double* bnd = nullptr, const unsigned long long* gmax = nullptr,
                        double tol = 0.0);
