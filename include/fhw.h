/*
 * fhw.h -- C ABI of the MI355X (gfx950) hot path of the frequency/time hybrid
 * wave-equation solver of Anderson, Bruno & Lyon, "High-order, dispersionless
 * Fast-Hybrid wave equation solver, Part I" (arXiv 1807.02718).
 *
 * The path, in the paper's order (Sec. 5, steps F1-F5 and T0-T6):
 *   fhw_plan             frequency grid, discretization sizes, boundary nodes,
 *                        Kress weights (Sec. 2.3, Sec. 4.1.1)
 *   fhw_solve_densities  assemble + factor + solve the direct combined-field
 *                        equation (eq. CFIE_direct) at every frequency (step F3)
 *   fhw_solve_incidences the same for several incident fields per factorization
 *   fhw_solve_cached     further incident fields on factors left resident
 *   fhw_plan_systems,    a batch of requests (any curve, frequency and N per
 *   fhw_factor,          system) factored together, then solved request by
 *   fhw_solve_range      request on the resident factors
 *   fhw_eval_field       layer potential U = int psi G (eqs. freq_domain_repr,
 *                        Ukslow_repr; step F5)
 *   fhw_synthesize       windowed, recentred signal spectra (eq. Bkslow_eqn,
 *                        steps F1-F2), Fourier coefficients (eq. fourier_approx,
 *                        T1a), sinc scaled-convolution synthesis and the sum
 *                        over windows (eqs. approx, discConv, ukW, final_u;
 *                        T2, T5)
 *   fhw_synthesize_uniform  the same on a uniform time grid, each window's
 *                        sum by the fast scaled convolution (Sec. 4.1.2, eq.
 *                        approx_conv_sum)
 *   fhw_run              the three calls above in one
 * plus stage entry points for the same steps on caller buffers.
 *
 * Conventions shared by every call
 *  - Return value: FHW_OK (0) or a negative FHW_E_* code; fhw_last_error()
 *    gives a message.  No call aborts the process.
 *  - Pointers are DEVICE pointers owned by the caller unless marked [host].
 *    The library never frees caller memory.
 *  - Work is enqueued on the HIP stream given to fhw_create and is
 *    asynchronous unless stated; calls that return host values synchronize
 *    that stream.  One context per stream; a context is not thread-safe.
 *  - Complex numbers are interleaved (re, im) pairs: double2 for FP64
 *    ("complex128"), float2 for FP32 ("complex64").
 *  - Matrices are column-major (entry (r, c) at c*N + r), packed, one after
 *    another at caller-given element offsets (ragged batches).
 *  - Frequencies: omega_j = j W / F, j = 1..F; wavenumber kappa = omega / c;
 *    coupling eta = max(kappa, 1).  The DFT grid is omega_l = (l - F) W / F,
 *    l = 0..2F-1, on [-W, W).
 *  - Boundary nodes: t_i = 2 pi i / N, i = 0..N-1 on a counter-clockwise
 *    curve; normals point out of the scatterer.
 */
#ifndef FHW_H
#define FHW_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FHW_OK 0
#define FHW_E_INVALID (-1)  /* bad argument, clockwise/degenerate curve, NaN input */
#define FHW_E_NOMEM (-2)    /* device memory or HBM budget exhausted */
#define FHW_E_HIP (-3)      /* HIP runtime error */
#define FHW_E_SINGULAR (-4) /* exactly zero pivot met in an LU factorization */
#define FHW_E_NOCONV (-5)   /* iterative refinement did not reach its tolerance */
#define FHW_E_STATE (-6)    /* call out of order (e.g. solve before plan) */
#define FHW_E_BUSY (-7)     /* serving: the queue is full, the request was not admitted */

#define FHW_FP64 0          /* complex128 LU and solves */
#define FHW_FP32_REFINE 1   /* complex64 LU on MFMA + FP64-residual refinement */

/* Boundary integral equation of a plan (fhw_problem.formulation). */
#define FHW_FORM_DIRECT 0   /* the direct combined-field equation (eq.
                               CFIE_direct): data of an incident wave (plane
                               waves, point sources); density = normal
                               derivative of the total field, field = single
                               layer (eq. freq_domain_repr) */
#define FHW_FORM_COMBINED 1 /* exterior Dirichlet problem for arbitrary data B:
                               u = int [dG/dnu_y - i eta G] phi dsigma_y with
                               (1/2) phi + K phi - i eta S phi = B (K the
                               double layer; Colton & Kress Sec. 3.2), for the
                               windowed data of general incident fields (eq.
                               bkdef2), which are not the trace of a wave */

typedef struct fhw_ctx fhw_ctx;

/* Scatterer boundary as a real trigonometric polynomial in s in [0, 2 pi):
 *   x1(s) = sum_{d=0}^{degree} cx[d] cos(d s) + sx[d] sin(d s), x2 likewise
 * with cy, sy.  [host] arrays of degree+1 doubles, counter-clockwise. */
typedef struct {
    int32_t degree;
    const double *cx, *sx, *cy, *sy;
} fhw_curve;

/* Frequency-domain problem (Sec. 2.1, Remark rem:pwe, Sec. 5 F3). */
typedef struct {
    double W;            /* band limit (> 0); solve frequencies j W / F        */
    int32_t F;           /* number of solve frequencies (>= 1)                 */
    double c;            /* wave speed (> 0); kappa = omega / c                */
    int32_t N_fixed;     /* > 0: this even N at every frequency; 0: rule below */
    double ppw;          /* points per wavelength over the curve length        */
    int32_t n_min, n_mult, n_cap;   /* N = clamp(ceil(ppw L kappa/(2 pi n_mult)) n_mult) */
    int32_t precision;   /* FHW_FP64 or FHW_FP32_REFINE                        */
    double refine_tol;   /* relative residual target ||g-A psi||/||g|| (FP32)  */
    int32_t refine_max;  /* maximum refinement sweeps (FP32 path)              */
    double direction[2]; /* plane-wave direction p (unit vector)               */
    int32_t j_first;     /* 0: frequencies j W / F, j = 1..F (the DFT grid of
                            fhw_eval_field / fhw_synthesize); > 0: the band
                            (j_first + j) W / F, j = 1..F, for frequency-domain
                            work only (solves; field and synthesis refuse it) */
    /* 2D low-frequency decomposition (Sec. 4.2; fhw_eval_field_lowfreq,
     * fhw_synthesize_lowfreq).  lf_M > 0 adds the graded frequencies: the
     * mesh mu_j = omega_c (j / lf_M)^lf_q, j = 0..lf_M (eq. gradedmesh),
     * omega_c = lf_jc W / F, and on each [mu_j, mu_{j+1}] the lf_N + 1
     * Clenshaw-Curtis points; the distinct ones in (0, omega_c), lf_M lf_N - 1
     * of them in ascending order, become systems F .. F + lf_M lf_N - 2 of the
     * plan (omega_c itself is system lf_jc - 1).  One curve, j_first = 0;
     * 1 <= lf_jc, F - lf_jc + 1 >= 20 (the continuation's matching points),
     * 1 <= lf_N <= 32, lf_q > 0.  lf_M = 0: none (the smooth-F path only). */
    int32_t lf_M, lf_N, lf_jc;
    double lf_q;
    /* FHW_FORM_DIRECT (0) or FHW_FORM_COMBINED.  A combined plan (one curve,
     * j_first = 0, the same N at every frequency; graded low-frequency
     * systems allowed) serves only fhw_solve_general and the window calls;
     * the direct calls (fhw_solve_densities, fhw_solve_incidences,
     * fhw_solve_cached, fhw_solve_range*, fhw_eval_field*, fhw_run) refuse
     * it with FHW_E_STATE, and the window calls refuse a direct plan. */
    int32_t formulation;
} fhw_problem;

/* Create a context bound to a HIP stream (hipStream_t passed as void*, NULL =
 * default stream).  hbm_budget_bytes caps the device workspace (0 = 90% of the
 * free device memory); solves are chunked over frequencies to fit it. */
int fhw_create(fhw_ctx** ctx, void* hip_stream, size_t hbm_budget_bytes);
int fhw_destroy(fhw_ctx* ctx);
const char* fhw_last_error(const fhw_ctx* ctx);
int fhw_version(void);

/* Plan a problem: frequencies, discretization sizes N_j, boundary nodes and
 * Kress weights per distinct N (Sec. 2.3), density layout, and the device
 * workspace (allocated here; later calls of the plan allocate nothing).
 * Outputs [host], optional (NULL to skip): N_out[F], psi_off_out[F+1]
 * (element offsets of psi_j in the ragged density buffer).
 * Errors: FHW_E_INVALID for a clockwise or degenerate curve, odd or
 * non-positive N, F < 1; FHW_E_NOMEM if one frequency does not fit the budget. */
int fhw_plan(fhw_ctx* ctx, const fhw_curve* curve, const fhw_problem* prob,
             int32_t* N_out, int64_t* psi_off_out);

/* Plan several scatterers with one problem (same frequencies, N rule,
 * precision): the frequency solves of all curves form one batch, so ragged
 * sizes across curves share every factorization launch.  System s = k F + j
 * is frequency j of curve k (curve-major); N_out [host] has n_curves F
 * entries and psi_off_out n_curves F + 1.  Every call below then covers all
 * systems (psi, resid and sweeps indexed by system); fields are per curve
 * (fhw_eval_field_curve).  Errors as fhw_plan, for any of the curves. */
int fhw_plan_curves(fhw_ctx* ctx, const fhw_curve* curves, int32_t n_curves, const fhw_problem* prob,
                    int32_t* N_out, int64_t* psi_off_out);

/* Step F3: densities psi_p(., omega_j) of eq. CFIE_direct with boundary data
 * exp(i kappa p.x), for all planned frequencies.
 * psi: complex128, psi_off[F] elements (ragged, offsets from fhw_plan).
 * resid [host, optional]: relative residuals per frequency (FP32 path: after
 * refinement; FP64 path: filled only when compute_resid != 0, else -1).
 * sweeps [host, optional]: refinement sweeps used per frequency.
 * Synchronizes the stream.  FHW_E_SINGULAR on an exactly zero pivot,
 * FHW_E_NOCONV if refinement misses refine_tol within refine_max sweeps. */
int fhw_solve_densities(fhw_ctx* ctx, void* psi, double* resid, int32_t* sweeps,
                        int32_t compute_resid);

/* Incident fields for fhw_solve_incidences (Sec. 2.1: any incident field
 * regular inside the scatterer; its boundary values B enter eq. CFIE_direct
 * through dB/dnu - i eta B). */
#define FHW_INC_PLANE 0     /* v = unit direction p: B = exp(i kappa p.x)          */
#define FHW_INC_POINT 1     /* v = source r0 outside the closed curve:
                               B = (i/4) H0(kappa |x - r0|); its field at omega = 0
                               is taken as 0 (eval_field zero_value = 0)          */
typedef struct {
    int32_t kind;
    double v[2];
} fhw_incidence;

/* Step F3 for several incident fields: each frequency is assembled and
 * factored once and its factors serve every incidence (the LU reuse of
 * Sec. 2.3 / Sec. 7 applied to many right-hand sides).
 * inc [host]: n_inc incidences (n_inc >= 1).
 * psi: complex128 [n_inc][psi_off[F]], incidence q's densities at
 * psi + q psi_off[F] in the ragged layout of fhw_plan (so that each block
 * can be passed to fhw_eval_field).
 * resid, sweeps [host, optional]: [n_inc][F], as in fhw_solve_densities.
 * The plan's own direction is not used.  Synchronizes the stream.
 * Errors: FHW_E_INVALID for an unknown kind, a direction that is not a unit
 * vector (to 1e-12), a source point on or inside the curve, or non-finite
 * values; FHW_E_SINGULAR / FHW_E_NOCONV as in fhw_solve_densities. */
int fhw_solve_incidences(fhw_ctx* ctx, const fhw_incidence* inc, int32_t n_inc, void* psi,
                         double* resid, int32_t* sweeps, int32_t compute_resid);

/* As fhw_solve_incidences, but with the factors left resident by the last
 * solve call on this plan: no assembly and no factorization, only the
 * triangular solves (and, in FP32_REFINE, the FP64-residual refinement
 * against the resident FP64 matrix).  Factors stay resident when the whole
 * plan fits one workspace chunk and the last solve did not compute FP64
 * residuals (those re-assemble A over the FP64 factors).
 * Errors: FHW_E_STATE when no factors are resident; otherwise as
 * fhw_solve_incidences. */
int fhw_solve_cached(fhw_ctx* ctx, const fhw_incidence* inc, int32_t n_inc, void* psi,
                     double* resid, int32_t* sweeps);

/* One frequency-domain system of a request: scatterer `curve` (index into the
 * plan's curves), frequency omega > 0 (kappa = omega / c) and an even N,
 * 4 <= N <= 4096 nodes. */
typedef struct {
    int32_t curve;
    double omega;
    int32_t N;
} fhw_system;

/* Plan an explicit list of systems (Sec. 2.3 discretization of eq.
 * CFIE_direct for each), for instance the frequencies of several requests of
 * different scatterers, bands and sizes, so that their factorizations share
 * every launch.  prob supplies c, precision, refine_tol, refine_max and the
 * plane-wave direction (W, F, the N rule and j_first are not used).  Such a
 * plan serves the solves only (fhw_eval_field, fhw_synthesize and the
 * DFT-grid stage calls refuse it with FHW_E_STATE).  psi_off_out [host,
 * optional]: n_systems + 1 offsets.  Errors: FHW_E_INVALID for a curve index
 * out of range, omega <= 0 or a bad N; otherwise as fhw_plan_curves. */
int fhw_plan_systems(fhw_ctx* ctx, const fhw_curve* curves, int32_t n_curves, const fhw_system* systems,
                     int32_t n_systems, const fhw_problem* prob, int64_t* psi_off_out);

/* Assemble and factor every system of the plan and leave the factors
 * resident (step F3 without a right-hand side), for fhw_solve_range and
 * fhw_solve_cached.  Synchronizes.  FHW_E_NOMEM if the plan needs more than
 * one workspace chunk; FHW_E_SINGULAR on an exactly zero pivot. */
int fhw_factor(fhw_ctx* ctx);

/* Solve systems s0 .. s0 + count - 1 on the resident factors for n_inc
 * incidences (as fhw_solve_cached, restricted to the range: one request of a
 * batched plan).  psi: complex128 [n_inc][E] with E = psi_off[s0 + count] -
 * psi_off[s0] (the range's densities, packed).  resid, sweeps [host,
 * optional]: [n_inc][count].  Synchronizes.  Errors: FHW_E_STATE without
 * resident factors; FHW_E_INVALID for a range outside the plan or bad
 * incidences; FHW_E_NOCONV as in fhw_solve_densities. */
int fhw_solve_range(fhw_ctx* ctx, int32_t s0, int32_t count, const fhw_incidence* inc, int32_t n_inc, void* psi,
                    double* resid, int32_t* sweeps);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * solves and results as fhw_solve_range, with its per-call status words (the
 * refinement's convergence flags, sweep counts and residual norms, and the
 * reported residuals) in a fixed device array of FHW_NOALLOC_SCRATCH_BYTES
 * inside the library instead of memory the library allocates.  The call
 * itself allocates nothing: no hipMalloc, hipFree or other allocating
 * routine; the factors, the plan's workspace and psi are as for
 * fhw_solve_range.  Limit: n_inc * count <= FHW_NOALLOC_MAX_PAIRS.  Every
 * call on one GPU uses that GPU's single array (each GPU the library runs on
 * holds it until the process ends), so such calls that overlap on one GPU,
 * from any context or thread, race; calls one after another do not (the
 * array is cleared at the start of each call).  The stage timers do not
 * record this call.  Synchronizes.  Errors: FHW_E_INVALID when n_inc * count
 * exceeds the limit; FHW_E_HIP if the array's device address could not be
 * looked up when the context was created; otherwise as fhw_solve_range. */
#define FHW_NOALLOC_SCRATCH_BYTES (1 << 20)
#define FHW_NOALLOC_MAX_PAIRS 16384
int fhw_solve_range_noalloc(fhw_ctx* ctx, int32_t s0, int32_t count, const fhw_incidence* inc, int32_t n_inc,
                            void* psi, double* resid, int32_t* sweeps);

/* ---------------- serving (continuous batching of frequency solves) ------- */

/* A solve request: frequencies omega[0 .. n_freq-1] (> 0) of one scatterer at N
 * nodes, n_inc incident fields (as fhw_solve_incidences).  psi: device
 * complex128 [n_inc][n_freq N] (incidence q, frequency j at q n_freq N + j N),
 * caller-owned, written when the request completes; resid, sweeps [host,
 * optional]: [n_inc][n_freq], written on completion.  The library copies
 * omegas and inc at submission; psi, resid and sweeps must stay valid until
 * the request is reported finished. */
typedef struct {
    int32_t curve;           /* index into the server's curves            */
    int32_t n_freq;
    const double* omegas;    /* [host] n_freq frequencies                  */
    int32_t N;               /* even, 4 <= N <= 4096                       */
    int32_t n_inc;
    const fhw_incidence* inc;/* [host] n_inc incidences                    */
    void* psi;
    double* resid;
    int32_t* sweeps;
} fhw_request;

typedef struct fhw_server fhw_server;

/* A server for requests on a fixed set of scatterers (Sec. 2.3 solves of eq.
 * CFIE_direct; the factorizations of a round stay resident for every
 * right-hand side of its requests, the LU reuse of Appendix A).  n_slots
 * worker slots on the current device, each a host thread with its own
 * context, HIP stream (non-blocking, default priority) and hbm_budget_bytes /
 * n_slots of workspace (0 = 85% of the free memory in all).  A free slot
 * takes every waiting request in arrival order while their matrices fit its
 * share, plans all their systems at once (fhw_plan_systems), factors them in
 * shared launches (fhw_factor) and solves each request on the resident
 * factors (fhw_solve_range), which completes it; a slot keeps its last
 * round's factors resident and serves a later round whose systems are all
 * among them without planning or factoring again.  Requests that arrive while
 * slots are busy wait for the next free slot; the slots' rounds overlap on
 * the device.  prob supplies c, precision, refine_tol, refine_max (the other
 * fields are not used).  queue_limit_bytes (0 = the whole budget): a request
 * submitted while the waiting requests hold more workspace bytes than this is
 * refused with FHW_E_BUSY.  curves [host] are copied. */
int fhw_server_create(fhw_server** server, const fhw_curve* curves, int32_t n_curves, const fhw_problem* prob,
                      int32_t n_slots, size_t hbm_budget_bytes, size_t queue_limit_bytes);
/* Queue a request; *ticket identifies it.  FHW_E_BUSY: not admitted (queue
 * full); FHW_E_NOMEM: larger than one slot's workspace; FHW_E_INVALID: bad
 * request.  Thread-safe. */
int fhw_server_submit(fhw_server* server, const fhw_request* req, int64_t* ticket);
/* Status of a request: *status = 1 while pending, else its result code
 * (FHW_OK or the solve's error).  wait != 0 blocks until it is finished.  A
 * finished ticket is reported once and then forgotten (FHW_E_INVALID after).
 * Thread-safe. */
int fhw_server_poll(fhw_server* server, int64_t ticket, int32_t wait, int32_t* status);
/* counts [host] int64[6]: rounds, requests finished, requests refused, systems
 * factored, requests waiting, requests served from a slot's resident factors
 * (no plan or factorization: every system of their round, (curve, omega, N)
 * at the server's precision, was among the factors the slot kept from its
 * previous round); busy_s [host, optional]: the slots' summed round time in
 * seconds.  A round's rounds, systems and cache counts are in before any of
 * its requests is reported finished; its busy time is added when the round
 * ends. */
int fhw_server_stats(fhw_server* server, int64_t* counts, double* busy_s);
/* Finishes the waiting requests, stops the slots and frees everything. */
int fhw_server_destroy(fhw_server* server);

/* Step F5 (eqs. freq_domain_repr, Ukslow_repr): V(r, omega_l) on the full DFT
 * grid, V[r][l], complex128 [N_r][2F]; V(r,-omega) = conj V(r,omega) and
 * V(r, 0) = zero_value (1 for plane-wave data: the low-frequency limit).
 * obs: [host] doubles [N_r][2], points off the boundary. */
int fhw_eval_field(fhw_ctx* ctx, const void* psi, const double* obs, int32_t N_r,
                   double zero_value, void* V);

/* As fhw_eval_field for curve k of a plan made by fhw_plan_curves (psi is the
 * whole density buffer of the plan); fhw_eval_field is curve 0. */
int fhw_eval_field_curve(fhw_ctx* ctx, int32_t curve, const void* psi, const double* obs,
                         int32_t N_r, double zero_value, void* V);

/* The field at the graded low-frequency nodes of a plan made with lf_M > 0
 * (Sec. 4.2): V_sing complex128 [N_r][lf_M lf_N + 1] (device), column g the
 * g-th node in ascending order: g = 0 is omega = 0 (value zero_value: 1 for
 * plane-wave data, the low-frequency limit), g = lf_M lf_N is omega_c.
 * obs [host] as in fhw_eval_field.  Errors: FHW_E_STATE for a plan without
 * the graded frequencies; FHW_E_INVALID for bad arguments. */
int fhw_eval_field_lowfreq(fhw_ctx* ctx, const void* psi, const double* obs, int32_t N_r, double zero_value,
                           void* V_sing);

/* Incident signal f sampled at t0 + n dt, n = 0..n-1 (device doubles); the
 * incident field is f(t - p.r/c) and the boundary signal is a = -f.  The
 * signal must vanish, with its derivatives, at both ends of the range. */
typedef struct {
    double t0, dt;
    int64_t n;
    const double* f;
} fhw_signal;

/* Partition of unity (Sec. 3.1): s_k = 1.5 H (k - 1), half-width H; tau0 is an
 * extra recentring shift (0 = the paper's choice).  track_tol > 0 turns on
 * active-partition tracking (Sec. 3.2, remark on tracking).  Window k is left
 * out everywhere when max_l (|Re B_k| + |Im B_k|) of its signal spectrum is
 * at most track_tol times the largest over the windows (its contribution is
 * then at most (W/pi) 2F max_l |B_k| max_l |V(r, .)|; no coefficients are
 * computed for it), and at observation point r when sum_m |Re c_{k,m}(r)| is
 * at most track_tol times the largest such sum over the remaining (k, r)
 * (|sinc| <= 1: the change is at most W/pi times that sum).  0 = every
 * window of the fixed rule |t - s_k - tau0| <= pi F / W. */
typedef struct {
    double H, tau0;
    double track_tol;
} fhw_windows;

/* Steps F1-F2 and T0-T6: scattered field u[r][t] (device doubles [N_r][N_t])
 * from V (device complex128 [N_r][2F], as written by fhw_eval_field) at the
 * [host] times[N_t].  Active windows: |t - s_k - tau0| <= pi F / W.
 * Errors: FHW_E_INVALID if 2F is not a power of two or inputs are non-finite. */
int fhw_synthesize(fhw_ctx* ctx, const fhw_signal* sig, const fhw_windows* win,
                   const void* V, int32_t N_r, const double* times, int32_t N_t,
                   double* u);

/* 2D time samples with the low-frequency decomposition (Sec. 4.2, eq.
 * fourier_sing_decomp; steps T1b, T2b-T2d, T5), for a plan with lf_M > 0.
 * For every window k whose support meets the signal's range (all of them at
 * every time: in 2D the low-frequency part of u_k decays only algebraically)
 * and t' = t - s_k - tau0, F_k(w) = B_k^slow(w) V(r, w) e^{-i w tau0}:
 *   u(r, t) = sum_k (1/pi) Re [ I_+ + I_0 ],
 *   I_+ = int_{omega_c}^{W} F_k e^{-i w t'} dw: F_k on the solve grid of
 *         [omega_c, W] extended by its FC(Gram) continuation (10 matching
 *         points, 25 continuation points: Remark Fourier-FC) and integrated
 *         term by term (eq. approx with period P != 2A);
 *   I_0 = int_0^{omega_c} F_k e^{-i w t'} dw by the composite
 *         Filon-Clenshaw-Curtis rule on the graded mesh (eq.
 *         gradedmeshIntRule), exact moments.
 * V: complex128 [N_r][2F] as written by fhw_eval_field; V_sing: [N_r][lf_M
 * lf_N + 1] as written by fhw_eval_field_lowfreq; times [host]; u: device
 * doubles [N_r][N_t], overwritten.  win->track_tol must be 0.
 * Errors: FHW_E_STATE without the graded frequencies; FHW_E_INVALID for bad
 * arguments or a smooth grid beyond the kernel's LDS (F - lf_jc + 1 too
 * large for the continuation and its coefficients in 64 KiB). */
int fhw_synthesize_lowfreq(fhw_ctx* ctx, const fhw_signal* sig, const fhw_windows* win, const void* V,
                           const void* V_sing, int32_t N_r, const double* times, int32_t N_t, double* u);

/* Sec. 4.1.2 (FFT accelerated evaluation of scaled discrete convolutions, eqs.
 * conv_sum and approx_conv_sum): as fhw_synthesize, on the uniform grid
 * t_n = t_first + n t_step, n < N_t, with each window's sum over m replaced
 * by its L-periodic approximation
 *   sum_m Re c_{k,m} sinc(x - m) ~= (1/L) sum_{p=-L/2}^{L/2-1} C_p e^{2 pi i p x / L},
 *   C_p = sum_m Re c_{k,m} e^{-2 pi i m p / L},   x = W (t_n - s_k - tau0) / pi,
 * evaluated by an L-point FFT and a chirp-z (Bluestein) convolution per
 * window, point and run of grid times.  The error against fhw_synthesize is
 * O(L^-2), carried by the spectrum's content near +-W; it vanishes to
 * roundoff where the spectrum is negligible there.  Same windows, active
 * sets and tracking rules (win->track_tol) as fhw_synthesize.
 *   u       device doubles [N_r][N_t], overwritten.
 *   L       0 = max(4F, 8); else a power of two with max(4F, 8) <= L <= 4096
 *           (the chirp-z convolution of length <= 8192 lives in LDS).
 * Errors: FHW_E_INVALID for a bad L, t_step <= 0, non-finite inputs, track_tol
 * < 0, N_r > 65535 or 2F not a power of two; FHW_E_STATE as fhw_synthesize. */
int fhw_synthesize_uniform(fhw_ctx* ctx, const fhw_signal* sig, const fhw_windows* win,
                           const void* V, int32_t N_r, double t_first, double t_step,
                           int32_t N_t, int32_t L, double* u);

/* The whole hot path in one call for a plan of one curve (fhw_plan) with its
 * plane-wave direction: fhw_solve_densities (step F3), fhw_eval_field with
 * V(r, 0) = 1 (step F5) and fhw_synthesize (F1-F2, T0-T6), in that order on
 * the context's stream, with the same kernels and results as the three calls.
 * psi: complex128 [psi_off[F]]; V: complex128 [N_r][2F]; u: doubles [N_r][N_t]
 * (all device, caller-owned; psi and V are written as by the separate calls).
 * obs, times, resid, sweeps [host] as in those calls.  Synchronizes.
 * Errors: FHW_E_STATE without a plan; FHW_E_INVALID for a plan of several
 * curves or bad arguments; otherwise the first failing step's code. */
int fhw_run(fhw_ctx* ctx, const fhw_signal* sig, const fhw_windows* win, const double* obs, int32_t N_r,
            const double* times, int32_t N_t, void* psi, void* V, double* u, double* resid,
            int32_t* sweeps);

/* Tracking statistics of the last fhw_synthesize on this context: pairs =
 * (window, point) pairs of the fixed rule, active = those kept (= pairs when
 * tracking was off).  [host] outputs.  FHW_E_STATE before any synthesis. */
int fhw_synth_active_pairs(fhw_ctx* ctx, int64_t* pairs, int64_t* active);

/* ---------------- general incident fields (eq. bkdef2) -------------------- */

/* Sampled Dirichlet data of a general incident field on the plan's nodes
 * (Sec. 3.2, eq. bkdef2: the boundary data of the scattered field is b =
 * -u_inc): b(x_i, t_n) at t_n = t0 + n dt, n < n_t, for the N Nystrom nodes
 * x_i of fhw_geometry(ctx, N, ...).  b: device doubles [n_t][N], time-major
 * (one time's nodes contiguous), caller-owned, read during
 * fhw_solve_general only. */
typedef struct {
    const double* b;
    int32_t N;
    int64_t n_t;
    double t0, dt;
} fhw_boundary;

/* The windows k = k_first .. k_first + n_win - 1 of the partition of unity
 * (Sec. 3.1: s_k = 1.5 H (k - 1), support [s_k - H, s_k + H]) whose support
 * meets [t_lo, t_hi].  [host] outputs.  FHW_E_INVALID for t_hi < t_lo, H <= 0
 * or non-finite arguments.  Needs no context. */
int fhw_window_range(double t_lo, double t_hi, double H, int64_t* k_first, int32_t* n_win);

/* Step F3 for general boundary data (Sec. 3.2, eq. bkdef2, with eq.
 * Bkslow_eqn applied node by node): u_k is the solution whose Dirichlet data
 * is the windowed b_k = w_k b.  For each window k = k_first + q, q < n_win,
 * and every system of the plan (solve frequencies, and the graded
 * low-frequency ones if planned), the recentred transform
 *   B_k(x_i, omega) = dt sum_n w(t_n - s_k) b(x_i, t_n) e^{i omega (t_n - s_k)}
 * (the rectangle rule, exact to roundoff for data resolved by the samples
 * since the windowed integrand vanishes with all derivatives at the
 * support's ends) is the right-hand side of the combined-potential equation
 * (FHW_FORM_COMBINED), solved on the resident factors (fhw_factor first).
 *   psi     device complex128 [n_win][psi_off[S]] (S systems): the densities
 *           phi of window k_first + q at q psi_off[S].
 *   resid, sweeps [host, optional]: [n_win][S] as fhw_solve_incidences.
 * Synchronizes.  Errors: FHW_E_STATE without resident factors or for a plan
 * that is not FHW_FORM_COMBINED; FHW_E_INVALID for null buffers, n_win < 1,
 * bnd->N not the plan's N, n_t < 2, dt <= 0, non-finite t0 or H <= 0;
 * FHW_E_NOCONV as fhw_solve_densities. */
int fhw_solve_general(fhw_ctx* ctx, const fhw_boundary* bnd, double H, int64_t k_first, int32_t n_win,
                      void* psi, double* resid, int32_t* sweeps);

/* Step F5 for the n_win density blocks of fhw_solve_general: each window's
 * field by the combined potential, V_k(r, omega) = (2 pi / N) sum_j |x'_j|
 * [(i kappa/4) H1(kappa rho) nu_j . (r - x_j)/rho + (eta/4) H0(kappa rho)]
 * phi_j, rho = |r - x_j| (trapezoidal rule; r away from the curve), at the
 * solve frequencies.  V: device complex128 [n_win][N_r][2F], block q as
 * fhw_eval_field lays out its field, with V(r, 0) = 0 (the zero-frequency
 * limit of a window's field, the bounded harmonic extension of its data, is
 * not computed).  obs [host] doubles [N_r][2].  Synchronizes.  Errors as
 * fhw_eval_field, and FHW_E_STATE for a plan fhw_solve_general does not take. */
int fhw_eval_field_windows(fhw_ctx* ctx, const void* psi, int32_t n_win, const double* obs, int32_t N_r,
                           void* V);

/* The same at the graded low-frequency nodes of a plan with lf_M > 0:
 * V_sing device complex128 [n_win][N_r][lf_M lf_N + 1], block q as
 * fhw_eval_field_lowfreq lays it out (ascending nodes, V(r, 0) = 0 first).
 * Errors: FHW_E_STATE without graded nodes; otherwise as above. */
int fhw_eval_field_windows_lowfreq(fhw_ctx* ctx, const void* psi, int32_t n_win, const double* obs, int32_t N_r,
                                   void* V_sing);

/* Steps T1a-T6 with each window's own field (general boundary data): u(r, t)
 * = sum over the windows k = k_first + q, q < n_win, active at t (|t - s_k -
 * tau0| <= pi F / W) of
 *   Re (W/pi) sum_m c_{k,m}(r) sinc(W (t - s_k - tau0)/pi - m),
 * c_{k,m}(r) the Fourier coefficients on [-W, W) of V_k(r, omega) e^{-i
 * omega tau0} (eqs. fourier_approx, approx, ukW, final_u; the windowed
 * boundary data already inside V_k, so there is no spectrum factor).
 * V: device complex128 [n_win][N_r][2F] (fhw_eval_field_windows); times
 * [host] N_t; u: device doubles [N_r][N_t], overwritten.  win->H and tau0 as
 * for fhw_solve_general; win->track_tol must be 0.  Synchronizes.
 * Errors: FHW_E_INVALID for bad arguments, non-finite times or 2F not a
 * power of two up to 8192; FHW_E_STATE as fhw_eval_field_windows. */
int fhw_synthesize_windows(fhw_ctx* ctx, const fhw_windows* win, int64_t k_first, int32_t n_win,
                           const void* V, int32_t N_r, const double* times, int32_t N_t, double* u);

/* fhw_synthesize_lowfreq with each window's own field (Sec. 4.2 for general
 * boundary data): for every window k = k_first + q, q < n_win, at every time
 * and t' = t - s_k - tau0, F_k(w) = V_k(r, w) e^{-i w tau0}, u(r, t) = sum_k
 * (1/pi) Re [I_+ + I_0] with I_+ from the FC(Gram) continuation of F_k on
 * the solve grid of [omega_c, W] and I_0 by the graded Filon-Clenshaw-Curtis
 * rule.  V: [n_win][N_r][2F] (fhw_eval_field_windows), V_sing: [n_win][N_r]
 * [lf_M lf_N + 1] (fhw_eval_field_windows_lowfreq); times [host]; u device
 * doubles [N_r][N_t], overwritten.  win->track_tol must be 0.  Errors as
 * fhw_synthesize_lowfreq and fhw_synthesize_windows. */
int fhw_synthesize_windows_lowfreq(fhw_ctx* ctx, const fhw_windows* win, int64_t k_first, int32_t n_win,
                                   const void* V, const void* V_sing, int32_t N_r, const double* times,
                                   int32_t N_t, double* u);

/* ---------------- stage entry points (same kernels, caller buffers) -------- */

/* Boundary nodes of the planned curve at N points (Sec. 2.3 Nystrom nodes):
 * geom doubles [9][N] = x1, x2, x1', x2', x1'', x2'', |x'|, nu1, nu2. */
int fhw_geometry(fhw_ctx* ctx, int32_t N, double* geom);

/* Kress weights R_l (l = 0..N-1) of the log-kernel product rule and the table
 * log(4 sin^2(l pi / N)) (entry 0 = 0), doubles [N] each (Sec. 2.3). */
int fhw_kress_weights(fhw_ctx* ctx, int32_t N, double* R, double* logtab);

/* Nystrom matrix and plane-wave RHS of eq. CFIE_direct for planned frequencies
 * j0 .. j0+count-1 (0-based): A complex128 at A_off[q] (N_j^2 elements each,
 * column-major), g complex128 at g_off[q] (N_j elements).  A_off, g_off [host].
 * For a plan of the combined formulation, A is that formulation's matrix. */
int fhw_assemble(fhw_ctx* ctx, int32_t j0, int32_t count, void* A, const int64_t* A_off,
                 void* g, const int64_t* g_off);

/* In-place batched LU with partial pivoting (max |re|+|im|, first index on
 * ties) of `batch` column-major square matrices: N[q], A_off[q], piv_off[q]
 * [host]; A complex128 (precision FHW_FP64) or complex64 (FHW_FP32_REFINE);
 * piv int32 (global row swapped with row i, applied in order).  Rows of
 * earlier column panels are not permuted by later pivots (the solve below
 * replays the pivots panel by panel).  linv: device workspace of
 * sum_q 4096*ceil(N[q]/64) elements of the same complex type, linv_off[q]
 * [host]; block p of matrix q (64x64 column-major at linv_off[q] + 4096 p)
 * receives the inverse of the unit-lower diagonal block p below its diagonal
 * and the inverse of the upper diagonal block on and above it.
 * Returns FHW_E_SINGULAR if any exactly zero pivot was met. */
int fhw_lu_factor(fhw_ctx* ctx, int32_t batch, const int32_t* N, const int64_t* A_off,
                  void* A, const int64_t* piv_off, int32_t* piv, const int64_t* linv_off,
                  void* linv, int32_t precision);

/* x = A^{-1} b from fhw_lu_factor output, in place on b (complex128,
 * b_off[q] [host]).  Factors may be complex64 (precision FHW_FP32_REFINE);
 * vectors are always complex128. */
int fhw_lu_solve(fhw_ctx* ctx, int32_t batch, const int32_t* N, const int64_t* A_off,
                 const void* LU, const int64_t* piv_off, const int32_t* piv,
                 const int64_t* linv_off, const void* linv, const int64_t* b_off,
                 void* b, int32_t precision);

/* Window spectra B_k^slow(omega_l) (eq. Bkslow_eqn) for windows k = k_first +
 * q, q = 0..count-1, on the planned DFT grid: B complex128 [count][2F]. */
int fhw_window_spectra(fhw_ctx* ctx, const fhw_signal* sig, const fhw_windows* win,
                       int64_t k_first, int32_t count, void* B);

/* Fourier coefficients c_{k,m}(r), m = -F..F-1 (eq. fourier_approx; T1a) of
 * B_k(omega) V(r, omega) exp(-i omega tau0) on [-W, W): c complex128
 * [count][N_r][2F] (index m + F) from B [count][2F] and V [N_r][2F]. */
int fhw_fourier_coefficients(fhw_ctx* ctx, const void* B, int32_t count, const void* V,
                             int32_t N_r, double tau0, void* c);

/* ---------------- diagnostics ------------------------------------------------ */

/* Stage timers: with profiling on, every kernel launch of the context is
 * bracketed by HIP events on the context's stream.  fhw_profile(ctx, 1) turns
 * it on and clears the counters, fhw_profile(ctx, 0) turns it off.
 * fhw_profile_read synchronizes the stream, writes the summed milliseconds and
 * the launch count per stage into [host] ms[FHW_N_STAGES] and
 * launches[FHW_N_STAGES], and clears the counters. */
#define FHW_STAGE_GEOMETRY 0
#define FHW_STAGE_KRESS 1
#define FHW_STAGE_ASSEMBLE 2
#define FHW_STAGE_LU_PANEL 3
#define FHW_STAGE_LU_DIAGINV 4
#define FHW_STAGE_LU_SWAP 5
#define FHW_STAGE_LU_TRSM 6
#define FHW_STAGE_LU_UPDATE 7
#define FHW_STAGE_SOLVE 8
#define FHW_STAGE_RESIDUAL 9
#define FHW_STAGE_FIELD 10
#define FHW_STAGE_SPECTRA 11
#define FHW_STAGE_COEFFS 12
#define FHW_STAGE_SYNTH 13
#define FHW_N_STAGES 14
int fhw_profile(fhw_ctx* ctx, int32_t enable);
int fhw_profile_read(fhw_ctx* ctx, double* ms, int64_t* launches);

/* Hankel functions H0^(1)(z), H1^(1)(z) at z[n] > 0 (device doubles) into
 * h complex128 [n][2] (diagnostic of the in-register Bessel evaluation). */
int fhw_hankel01(fhw_ctx* ctx, const double* z, int64_t n, void* h);

#ifdef __cplusplus
}
#endif
#endif /* FHW_H */
