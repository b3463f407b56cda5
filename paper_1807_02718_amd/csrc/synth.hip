// Frequency-to-time synthesis with windowing and recentring (Sec. 3, Sec. 4.1):
//   B_k^slow(omega_l) = int w(t) a(t + s_k) e^{i omega_l t} dt         (eq. Bkslow_eqn)
//   c_{k,m}(r): Fourier coefficients on [-W, W) of
//               B_k^slow(omega) V(r, omega) e^{-i omega tau0}         (eq. fourier_approx, T1a)
//   u(r, t) = Re sum_{k active} (W/pi) sum_m c_{k,m}(r) sinc(W (t - s_k - tau0)/pi - m)
//                                                  (eqs. approx, discConv, ukW, final_u; T2, T5)
#include "fhw_device.h"
#include "fhw_internal.h"
#include "lds_fft.h"

#define SYN_THREADS 256
#define SYN_MMAX 8192   // largest 2F: the LDS buffer and the 64 x 64 twiddle tables
#define WS_CHUNK 2048

// Partition-of-unity window (eq. window_func) with eta(u) = exp(2 e^{-1/u}/(u-1)).
__device__ __forceinline__ double fhw_eta(double u) {
    if (u <= 0.0) return 1.0;
    if (u >= 1.0) return 0.0;
    return exp(2.0 * exp(-1.0 / u) / (u - 1.0));
}
__device__ __forceinline__ double fhw_window(double t, double H) {
    const double h2 = 0.5 * H;
    if (t >= -H && t <= -h2) return 1.0 - fhw_eta((t + H) / h2);
    if (t > -h2 && t < h2) return 1.0;
    if (t >= h2 && t <= H) return fhw_eta((t - h2) / h2);
    return 0.0;
}

// grid (count, ceil(2F / 32)): a workgroup takes 32 grid frequencies omega_l
// and splits the window's samples over 8 phases (sample i to phase i mod 8),
// so that a window's transform spreads over many workgroups; the 8 partial
// sums of a frequency are added in phase order.
#define WS_FREQ 32
#define WS_PH (SYN_THREADS / WS_FREQ)
// With om_list != NULL the frequencies are om_list[0 .. n_om - 1] instead of
// the DFT grid (B row length n_om).
__global__ __launch_bounds__(SYN_THREADS) void k_window_spectra(const double* __restrict__ f, int64_t n, double t0,
                                                                double dt, double H, int64_t k_first,
                                                                const int64_t* __restrict__ klist, double W, int F,
                                                                const double* __restrict__ om_list, int n_om,
                                                                zd* __restrict__ B) {
    __shared__ double wa[WS_CHUNK];
    __shared__ double tau[WS_CHUNK];
    __shared__ double red[2][WS_PH][WS_FREQ];
    const int q = blockIdx.x;
    const int64_t k = klist ? klist[q] : (k_first + q);
    const double sk = 1.5 * H * ((double)k - 1.0);
    const int M = om_list ? n_om : 2 * F;
    const int fl = threadIdx.x % WS_FREQ, ph = threadIdx.x / WS_FREQ;
    const int l = blockIdx.y * WS_FREQ + fl;
    const double dw = W / (double)F;
    const double om = om_list ? (l < M ? om_list[l] : 0.0) : -W + dw * (double)l;
    int64_t n_lo = (int64_t)floor((sk - H - t0) / dt) - 1;
    int64_t n_hi = (int64_t)ceil((sk + H - t0) / dt) + 1;
    if (n_lo < 0) n_lo = 0;
    if (n_hi > n - 1) n_hi = n - 1;
    double ar = 0.0, ai = 0.0;
    for (int64_t c0 = n_lo; c0 <= n_hi; c0 += WS_CHUNK) {
        const int cnt = (int)min<int64_t>(WS_CHUNK, n_hi - c0 + 1);
        __syncthreads();
        for (int i = threadIdx.x; i < cnt; i += SYN_THREADS) {
            const int64_t nn = c0 + i;
            const double tn = t0 + dt * (double)nn;
            const double tt = tn - sk;
            tau[i] = tt;
            wa[i] = fhw_window(tt, H) * (-f[nn]);
        }
        __syncthreads();
        if (l < M) {
            for (int i = ph; i < cnt; i += WS_PH) {
                const double w = wa[i];
                if (w != 0.0) {
                    double s, c;
                    sincos(om * tau[i], &s, &c);
                    ar = fma(w, c, ar);
                    ai = fma(w, s, ai);
                }
            }
        }
    }
    red[0][ph][fl] = ar;
    red[1][ph][fl] = ai;
    __syncthreads();
    if (ph == 0 && l < M) {
        double sr = 0.0, si = 0.0;
#pragma unroll
        for (int p = 0; p < WS_PH; ++p) {
            sr += red[0][p][fl];
            si += red[1][p][fl];
        }
        B[(int64_t)q * M + l] = cmk(dt * sr, dt * si);
    }
}

// Right-hand sides of the combined-potential equation for general boundary
// data (eq. bkdef2): window k = k_first + q, system j (items[j]: omega =
// kappa c, offset g_off), node i:
//   B = dt sum_n w(t_n - s_k) b(x_i, t_n) e^{i omega (t_n - s_k)}
// written at g + q sg + g_off + i.  b: samples [n_t][N] (time-major, so one
// time's nodes are contiguous).  Grid (n_win, ceil(n_sys / BW_SYS),
// ceil(N / (BW_NPT SYN_THREADS))): a thread takes BW_NPT nodes (node + p
// SYN_THREADS) and BW_SYS systems; the factors w e^{i omega tau} of a run of
// samples are staged in LDS, so each sample is read once per BW_SYS systems
// and each staged factor serves BW_NPT nodes.
#ifndef FHW_BW_NPT
#define FHW_BW_NPT 4     // nodes per thread (1: 4.0 ms, 2: 3.2 ms against 2.9 ms per general call)
#endif
#define BW_SYS 8
#define BW_NPT FHW_BW_NPT
#define BW_CHUNK 256
__global__ __launch_bounds__(SYN_THREADS) void k_boundary_rhs(const double* __restrict__ b, int64_t n_t, int N,
                                                              double t0, double dt, double H, int64_t k_first,
                                                              double c, const fhw_assemble_item* __restrict__ items,
                                                              int n_sys, int64_t sg, zd* __restrict__ g) {
    __shared__ zd E[BW_SYS][BW_CHUNK];
    const int q = blockIdx.x;
    const int j0 = blockIdx.y * BW_SYS;
    const int ns = min(BW_SYS, n_sys - j0);
    const int node0 = blockIdx.z * (BW_NPT * SYN_THREADS) + threadIdx.x;
    const double sk = 1.5 * H * ((double)(k_first + q) - 1.0);
    // samples whose window weight can be nonzero, [sk - H, sk + H]
    int64_t n_lo = (int64_t)floor((sk - H - t0) / dt);
    int64_t n_hi = (int64_t)ceil((sk + H - t0) / dt);
    if (n_lo < 0) n_lo = 0;
    if (n_hi > n_t - 1) n_hi = n_t - 1;
    zd aB[BW_NPT][BW_SYS];
#pragma unroll
    for (int p = 0; p < BW_NPT; ++p)
#pragma unroll
        for (int u = 0; u < BW_SYS; ++u) aB[p][u] = cmk(0.0, 0.0);
    for (int64_t c0 = n_lo; c0 <= n_hi; c0 += BW_CHUNK) {
        const int cnt = (int)min<int64_t>(BW_CHUNK, n_hi - c0 + 1);
        __syncthreads();
        // one sample per thread: its window weight once, the group's phases
        for (int i = threadIdx.x; i < cnt; i += SYN_THREADS) {
            const double tau = t0 + dt * (double)(c0 + i) - sk;
            const double w = fhw_window(tau, H);
#pragma unroll
            for (int u = 0; u < BW_SYS; ++u) {
                zd v = cmk(0.0, 0.0);
                if (u < ns && w != 0.0) {
                    double sn, cs;
                    sincos(items[j0 + u].kappa * c * tau, &sn, &cs);
                    v = cmk(w * cs, w * sn);
                }
                E[u][i] = v;
            }
        }
        __syncthreads();
        if (node0 < N) {
            // the thread's nodes past N read node0's samples (never written)
            const double* bp[BW_NPT];
#pragma unroll
            for (int p = 0; p < BW_NPT; ++p) {
                const int nd = node0 + p * SYN_THREADS;
                bp[p] = b + c0 * (int64_t)N + (nd < N ? nd : node0);
            }
            int i = 0;
            // four samples' loads per node in flight before their products
            for (; i + 4 <= cnt; i += 4) {
                double bv[BW_NPT][4];
#pragma unroll
                for (int p = 0; p < BW_NPT; ++p)
#pragma unroll
                    for (int k = 0; k < 4; ++k) bv[p][k] = bp[p][(int64_t)(i + k) * N];
#pragma unroll
                for (int k = 0; k < 4; ++k) {
#pragma unroll
                    for (int u = 0; u < BW_SYS; ++u) {
                        const zd e = E[u][i + k];
#pragma unroll
                        for (int p = 0; p < BW_NPT; ++p)
                            aB[p][u] = cmk(fma(bv[p][k], e.re, aB[p][u].re), fma(bv[p][k], e.im, aB[p][u].im));
                    }
                }
            }
            for (; i < cnt; ++i) {
                double bv[BW_NPT];
#pragma unroll
                for (int p = 0; p < BW_NPT; ++p) bv[p] = bp[p][(int64_t)i * N];
#pragma unroll
                for (int u = 0; u < BW_SYS; ++u) {
                    const zd e = E[u][i];
#pragma unroll
                    for (int p = 0; p < BW_NPT; ++p)
                        aB[p][u] = cmk(fma(bv[p], e.re, aB[p][u].re), fma(bv[p], e.im, aB[p][u].im));
                }
            }
        }
    }
#pragma unroll
    for (int p = 0; p < BW_NPT; ++p) {
        const int nd = node0 + p * SYN_THREADS;
        if (nd >= N) continue;
#pragma unroll
        for (int u = 0; u < BW_SYS; ++u) {
            if (u < ns) {
                const fhw_assemble_item it = items[j0 + u];
                g[(int64_t)q * sg + it.g_off + nd] = cmk(dt * aB[p][u].re, dt * aB[p][u].im);
            }
        }
    }
}

// Tracking, window level: wmax[q] = max_l (|Re B_q| + |Im B_q|) over the DFT
// grid, and the largest over the windows into *gwmax (double bits, zero before).
__global__ __launch_bounds__(SYN_THREADS) void k_window_max(const zd* __restrict__ B, int M,
                                                            double* __restrict__ wmax,
                                                            unsigned long long* __restrict__ gwmax) {
    __shared__ double red[SYN_THREADS / 64];
    const int q = blockIdx.x;
    const zd* Bq = B + (int64_t)q * M;
    double m = 0.0;
    for (int l = threadIdx.x; l < M; l += SYN_THREADS) m = fmax(m, fabs(Bq[l].re) + fabs(Bq[l].im));
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) m = fmax(m, __shfl_xor(m, off, 64));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < SYN_THREADS / 64; ++w) t = fmax(t, red[w]);
        wmax[q] = t;
        atomicMax(gwmax, (unsigned long long)__double_as_longlong(t));
    }
}

// One workgroup per (point r, window slot q): LDS radix-2^3 FFT of length M = 2F
// of G_l = B_q(omega_l) V(r, omega_l) e^{-i omega_l tau0};
// c_m = (-1)^m X[m mod M] / M stored at index m + F: complex128 into c, or,
// when c_re is given instead, only the real parts (all the synthesis needs:
// its sinc weights are real and the field is the real part of the sum).
// With bnd given (tracking): also bnd[q N_r + r] = sum_m |Re c_m| in a fixed
// order, and the largest such bound into *gmax (the bits of a non-negative
// double order as an unsigned integer; *gmax starts at 0).
__global__ __launch_bounds__(SYN_THREADS) void k_fourier_coeffs(const zd* __restrict__ B, const zd* __restrict__ V,
                                                                int64_t v_qstride, int N_r, double W, int F,
                                                                int logM, double tau0,
                                                                zd* __restrict__ c, double* __restrict__ c_re,
                                                                double* __restrict__ bnd,
                                                                unsigned long long* __restrict__ gmax,
                                                                const double* __restrict__ wmax,
                                                                const unsigned long long* __restrict__ gwmax,
                                                                double tol) {
    extern __shared__ zd X[];
    const int r = blockIdx.x;
    const int q = blockIdx.y;
    if (bnd && wmax[q] <= tol * __longlong_as_double((long long)*gwmax)) {
        // a silent window: no coefficients, bound 0 (the synthesis skips it)
        if (threadIdx.x == 0) bnd[(int64_t)q * N_r + r] = 0.0;
        return;
    }
    const int M = 2 * F;
    const double dw = W / (double)F;
    const zd* Bq = B ? B + (int64_t)q * M : nullptr;   // NULL: each window has its own V
    const zd* Vr = V + (int64_t)q * v_qstride + (int64_t)r * M;
    __shared__ zd thi[64], tlo[64];
    fft_tables(thi, tlo, M);
    for (int l = threadIdx.x; l < M; l += SYN_THREADS) {
        const double om = -W + dw * (double)l;
        double s, cs;
        sincos(-om * tau0, &s, &cs);
        const zd g = cmul(Bq ? cmul(Bq[l], Vr[l]) : Vr[l], cmk(cs, s));
        const int rev = (int)(__brev((unsigned)l) >> (32 - logM));
        X[rev] = g;
    }
    __syncthreads();
    lds_fft<SYN_THREADS, SYN_MMAX>(X, logM, thi, tlo, logM);
    const int64_t base = ((int64_t)q * N_r + r) * M;
    const double inv = 1.0 / (double)M;
    double babs = 0.0;
    for (int idx = threadIdx.x; idx < M; idx += SYN_THREADS) {
        const int m = idx - F;
        const zd x = X[(idx + F) % M];
        const double sg = (m & 1) ? -inv : inv;
        if (c_re) c_re[base + idx] = sg * x.re;
        else c[base + idx] = cmk(sg * x.re, sg * x.im);
        babs += fabs(x.re) * inv;
    }
    if (bnd) {
        __shared__ double red[SYN_THREADS / 64];
        babs = wave_sum(babs);
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = babs;
        __syncthreads();
        if (threadIdx.x == 0) {
            double t = 0.0;
            for (int w = 0; w < SYN_THREADS / 64; ++w) t += red[w];
            bnd[(int64_t)q * N_r + r] = t;
            atomicMax(gmax, (unsigned long long)__double_as_longlong(t));
        }
    }
}

// u(r, t) = (W/pi) sum_{k active} sum_m Re c_{k,m}(r) sinc(x - m), x = W (t - s_k
// - tau0)/pi, active: |t - s_k - tau0| <= pi F / W.  With sinc(x - m) =
// (-1)^m sin(pi x) / (pi (x - m)) the sum over m is sin(pi x)/pi times
// sum_m (-1)^m Re c_m / (x - m); an integer x leaves the single term m = x.
// One wave per (point r, block of ST consecutive time indices): each lane
// reads its coefficients of a window once and serves all ST times; fixed-
// order reductions.
#define ST 8

// 1/y: the hardware reciprocal estimate (relative error below 2^-24, measured
// over 2^20 arguments) refined by one Newton-Raphson step, which squares it:
// within about 3e-15 of 1/y, the size of the rounding of the 2F-term sum it
// feeds and far below the synthesis's truncation error (a second step cost
// 15% of the kernel: 1.54 vs 1.30 ms per headline step).
__device__ __forceinline__ double synth_recip(double y) {
    const double r = __builtin_amdgcn_rcp(y);
    return fma(r, fma(-y, r, 1.0), r);
}

// Tracking (bnd != NULL): window slot sl is skipped at point r when
// bnd[sl N_r + r] <= tol * gmax; its whole contribution is bounded by
// (W/pi) bnd (|sinc| <= 1).
__global__ __launch_bounds__(SYN_THREADS, 4) void k_synth(const double* __restrict__ cre, const int* __restrict__ slot,
                                                       int64_t k_min, int64_t k_max, int N_r,
                                                       const double* __restrict__ times, int N_t, double W, int F,
                                                       double H, double tau0, double* __restrict__ u,
                                                       const double* __restrict__ bnd,
                                                       const unsigned long long* __restrict__ gmax, double tol) {
    const int nblk = (N_t + ST - 1) / ST;
    const int64_t wave = (int64_t)blockIdx.x * (SYN_THREADS / 64) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (wave >= (int64_t)N_r * nblk) return;
    const int r = (int)(wave / nblk);
    const int it0 = (int)(wave - (int64_t)r * nblk) * ST;
    const int M = 2 * F;
    const double P = FHW_PI / (W / (double)F);
    const double span = 1.5 * H;
    double tq[ST];
    int64_t ka = INT64_MAX, kb = INT64_MIN;
#pragma unroll
    for (int q = 0; q < ST; ++q) {
        tq[q] = (it0 + q < N_t) ? times[it0 + q] : times[it0];
        ka = min(ka, (int64_t)floor((tq[q] - tau0 - P) / span) + 1 - 1);
        kb = max(kb, (int64_t)ceil((tq[q] - tau0 + P) / span) + 1 + 1);
    }
    ka = max(ka, k_min);
    kb = min(kb, k_max);
    const double cut = bnd ? tol * __longlong_as_double((long long)*gmax) : -1.0;
    double tot[ST];
#pragma unroll
    for (int q = 0; q < ST; ++q) tot[q] = 0.0;
    for (int64_t k = ka; k <= kb; ++k) {
        const int sl = slot[k - k_min];
        if (sl < 0) continue;
        if (bnd && bnd[(int64_t)sl * N_r + r] <= cut) continue;   // inactive here
        const double sk = 1.5 * H * ((double)k - 1.0);
        // a time that does not use this window's sum (inactive, or at an
        // integer x) takes x = 1/2: its terms stay finite and its weight is 0,
        // so the sum over m needs no per-term guard
        double xq[ST], scale[ST], part[ST];
        bool anyk = false;
#pragma unroll
        for (int q = 0; q < ST; ++q) {
            const bool act = (it0 + q < N_t) && fabs(tq[q] - sk - tau0) <= P;
            const double x = W * (tq[q] - sk - tau0) / FHW_PI;
            const bool integral = act && x == floor(x);
            const bool use = act && !integral;
            scale[q] = use ? sinpi(x) / FHW_PI : 0.0;
            xq[q] = use ? x : 0.5;
            part[q] = 0.0;
            anyk |= act;
            if (integral && lane == 0) {
                // sinc(x - m) = 1 at m = x, 0 at every other m
                const int idx = (int)x + F;
                if (idx >= 0 && idx < M) tot[q] += cre[((int64_t)sl * N_r + r) * M + idx];
            }
        }
        if (!anyk) continue;
        const double* ck = cre + ((int64_t)sl * N_r + r) * M;
        for (int idx = lane; idx < M; idx += 64) {
            const int m = idx - F;
            const double a = (m & 1) ? -ck[idx] : ck[idx];
#pragma unroll
            for (int q = 0; q < ST; ++q) part[q] = fma(a, synth_recip(xq[q] - (double)m), part[q]);
        }
#pragma unroll
        for (int q = 0; q < ST; ++q) tot[q] = fma(scale[q], part[q], tot[q]);
    }
#pragma unroll
    for (int q = 0; q < ST; ++q) {
        const double v = wave_sum(tot[q]);
        if (lane == 0 && it0 + q < N_t) u[(int64_t)r * N_t + it0 + q] = (W / FHW_PI) * v;
    }
}

hipError_t launch_window_spectra(hipStream_t s, const double* f, int64_t n, double t0, double dt, double H,
                                 int64_t k_first, const int64_t* d_klist, int32_t count, double W, int32_t F,
                                 void* B) {
    if (count <= 0) return hipSuccess;
    dim3 grid(count, (2 * F + WS_FREQ - 1) / WS_FREQ);
    hipLaunchKernelGGL(k_window_spectra, grid, dim3(SYN_THREADS), 0, s, f, n, t0, dt, H, k_first, d_klist, W, F,
                       (const double*)nullptr, 0, (zd*)B);
    return hipGetLastError();
}

hipError_t launch_boundary_rhs(hipStream_t s, const double* b, int64_t n_t, int32_t N, double t0, double dt,
                               double H, int64_t k_first, int32_t n_win, double c, const fhw_assemble_item* d_items,
                               int32_t n_sys, int64_t sg, void* g) {
    if (n_win <= 0 || n_sys <= 0 || N <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_boundary_rhs, dim3(n_win, (n_sys + BW_SYS - 1) / BW_SYS,
                                            (N + BW_NPT * SYN_THREADS - 1) / (BW_NPT * SYN_THREADS)),
                       dim3(SYN_THREADS), 0, s, b, n_t, N, t0, dt, H, k_first, c, d_items, n_sys, sg, (zd*)g);
    return hipGetLastError();
}

hipError_t launch_window_spectra_at(hipStream_t s, const double* f, int64_t n, double t0, double dt, double H,
                                    const int64_t* d_klist, int32_t count, const double* d_om, int32_t n_om,
                                    void* B) {
    if (count <= 0 || n_om <= 0) return hipSuccess;
    dim3 grid(count, (n_om + WS_FREQ - 1) / WS_FREQ);
    hipLaunchKernelGGL(k_window_spectra, grid, dim3(SYN_THREADS), 0, s, f, n, t0, dt, H, (int64_t)0, d_klist, 1.0, 1,
                       d_om, n_om, (zd*)B);
    return hipGetLastError();
}

hipError_t launch_fourier_coeffs(hipStream_t s, const void* B, int32_t count, const void* V, int32_t N_r, double W,
                                 int32_t F, double tau0, void* c, double* c_re, double* bnd,
                                 unsigned long long* gmax, double* wmax, unsigned long long* gwmax, double tol,
                                 int64_t v_qstride) {
    if (count <= 0 || N_r <= 0) return hipSuccess;
    if (!B && bnd) return hipErrorInvalidValue;   // tracking needs the window spectra
    const int M = 2 * F;
    if (M > SYN_MMAX || (M & (M - 1))) return hipErrorInvalidValue;
    int logM = 0;
    while ((1 << logM) < M) ++logM;
    size_t lds = (size_t)M * sizeof(zd);
    static std::atomic<uint64_t> attr{0};
    fhw_once_on_device(attr, [&] {
        // transforms up to 2F = 8192 (128 KiB) beside the static LDS
        (void)hipFuncSetAttribute((const void*)k_fourier_coeffs, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  SYN_MMAX * (int)sizeof(zd));
    });
    if (bnd) {
        hipLaunchKernelGGL(k_window_max, dim3(count), dim3(SYN_THREADS), 0, s, (const zd*)B, M, wmax, gwmax);
    }
    hipLaunchKernelGGL(k_fourier_coeffs, dim3(N_r, count), dim3(SYN_THREADS), lds, s, (const zd*)B, (const zd*)V,
                       v_qstride, N_r, W, F, logM, tau0, (zd*)c, c_re, bnd, gmax, (const double*)wmax,
                       (const unsigned long long*)gwmax, tol);
    return hipGetLastError();
}

hipError_t launch_synth(hipStream_t s, const void* c, const int32_t* d_slot, int64_t k_min, int64_t k_max,
                        int32_t n_slots, int32_t N_r, const double* times, int32_t N_t, double W, int32_t F, double H,
                        double tau0, double* u, const double* bnd, const unsigned long long* gmax, double tol) {
    (void)n_slots;
    const int64_t waves = (int64_t)N_r * ((N_t + ST - 1) / ST);
    if (waves <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_synth, dim3((unsigned)((waves + 3) / 4)), dim3(SYN_THREADS), 0, s, (const double*)c, d_slot,
                       k_min, k_max, N_r, times, N_t, W, F, H, tau0, u, bnd, gmax, tol);
    return hipGetLastError();
}
