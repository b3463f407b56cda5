// Time samples in 2D with the low-frequency decomposition (Sec. 4.2, eq.
// fourier_sing_decomp; steps T1b, T2b-T2d, T5).  Per window k and point r,
// with F(w) = B_k^slow(w) V(r, w) e^{-i w tau0} and t' = t - s_k - tau0,
//   u_k(r, t) = (1/pi) Re [ I_+(t') + I_0(t') ]
//   I_+ = int_{omega_c}^{W} F e^{-i w t'} dw: F on the solve grid of
//         [omega_c, W] is extended by its FC(Gram) continuation (Remark
//         Fourier-FC) to one period of L = n + C points; the trigonometric
//         interpolant of period P = L h is integrated term by term over
//         [omega_c, W] (eq. approx with P != 2A);
//   I_0 = int_0^{omega_c} F e^{-i w t'} dw by the Filon-Clenshaw-Curtis rule
//         on each subinterval of the graded mesh (eqs. gradedmesh,
//         gradedmeshIntRule): the degree-n interpolant at the subinterval's
//         Clenshaw-Curtis points, times the oscillatory kernel, integrated
//         exactly.
// The negative frequencies are the complex conjugates (real signals), hence
// (1/2 pi) 2 Re.  Every window with signal content is summed at every time.
#include "fc_tables.h"
#include "fhw_device.h"
#include "fhw_internal.h"

#define LF_THREADS 256

// Coefficients of one (window, point): the L Fourier coefficients c_m (m =
// -L/2 .. L/2-1) of the continued smooth part, and per graded subinterval the
// Chebyshev coefficients alpha_k of the interpolant and the derivatives
// p^(j)(+1), p^(j)(-1) (j = 0..n) of p = sum_k alpha_k T_k.
// B: spectra [K][n_om] at om (smooth grid, then the M n + 1 graded nodes);
// V: [N_r][2F] on the DFT grid; Vs: [N_r][M n + 1] at the graded nodes.
__global__ __launch_bounds__(LF_THREADS) void k_lf_coeffs(const zd* __restrict__ B, const double* __restrict__ om,
                                                         int n_om, const zd* __restrict__ V, const zd* __restrict__ Vs,
                                                         int64_t v_qstride, int64_t vs_qstride, int N_r, int F,
                                                         int jc, int n, int M, int nc, double tau0,
                                                         zd* __restrict__ cfs, zd* __restrict__ cheb) {
    extern __shared__ zd lds[];
    const int L = n + FC_C;
    zd* g = lds;          // [L] samples and continuation
    zd* tw = lds + L;     // [L] e^{-2 pi i j / L}
    __shared__ zd aR[FC_D], aL[FC_D];
    const int q = blockIdx.x / N_r, r = blockIdx.x - q * N_r;
    const zd* Bq = B ? B + (int64_t)q * n_om : nullptr;   // NULL: each window has its own field
    const zd* Vr = V + (int64_t)q * v_qstride + (int64_t)r * 2 * F;
    Vs += (int64_t)q * vs_qstride;
    const int tid = threadIdx.x;
    for (int i = tid; i < n; i += LF_THREADS) {
        const int l = F + jc + i;   // grid index of omega = (jc + i) W / F; +W is stored as conj at l = 0
        const zd v = l < 2 * F ? Vr[l] : cconj(Vr[0]);
        double s, c;
        sincos(om[i] * tau0, &s, &c);
        g[i] = cmul(Bq ? cmul(Bq[i], v) : v, cmk(c, -s));
    }
    for (int j = tid; j < L; j += LF_THREADS) {
        double s, c;
        sincospi(-2.0 * (double)j / (double)L, &s, &c);
        tw[j] = cmk(c, s);
    }
    __syncthreads();
    // Gram projections of the last d samples and of the first d, reversed
    if (tid < 2 * FC_D) {
        const int k = tid % FC_D;
        zd a = cmk(0.0, 0.0);
        if (tid < FC_D) {
            for (int j = 0; j < FC_D; ++j) a = cfma(a, cmk(FC_Q[j][k], 0.0), g[n - FC_D + j]);
            aR[k] = a;
        } else {
            for (int j = 0; j < FC_D; ++j) a = cfma(a, cmk(FC_Q[j][k], 0.0), g[FC_D - 1 - j]);
            aL[k] = a;
        }
    }
    __syncthreads();
    // continuation: blend to zero of the right end plus the mirrored blend
    // from zero of the left end
    if (tid < FC_C) {
        zd vr = cmk(0.0, 0.0), vl = cmk(0.0, 0.0);
        for (int k = 0; k < FC_D; ++k) {
            vr = cfma(vr, cmk(FC_A[tid][k], 0.0), aR[k]);
            vl = cfma(vl, cmk(FC_A[FC_C - 1 - tid][k], 0.0), aL[k]);
        }
        g[n + tid] = cadd(vr, vl);
    }
    __syncthreads();
    // c_m = (1/L) sum_j g_j e^{-2 pi i m j / L}, exact twiddle indices
    zd* cq = cfs + (int64_t)blockIdx.x * L;
    for (int mi = tid; mi < L; mi += LF_THREADS) {
        const int m = mi - L / 2;
        const int64_t mm = ((int64_t)m % L + L) % L;
        zd acc = cmk(0.0, 0.0);
        int64_t idx = 0;
        for (int j = 0; j < L; ++j) {
            acc = cfma(acc, g[j], tw[idx]);
            idx += mm;
            if (idx >= L) idx -= L;
        }
        cq[mi] = cmk(acc.re / (double)L, acc.im / (double)L);
    }
    // Filon-Clenshaw-Curtis data per subinterval (one thread each)
    for (int j = tid; j < M; j += LF_THREADS) {
        zd G[33];
        for (int i = 0; i <= nc; ++i) {
            // Clenshaw-Curtis point i (x_i = cos(pi i / nc)) is graded node j nc + nc - i
            const int gidx = j * nc + nc - i;
            double s, c;
            sincos(om[n + gidx] * tau0, &s, &c);
            const zd vs = Vs[(int64_t)r * (M * nc + 1) + gidx];
            G[i] = cmul(Bq ? cmul(Bq[n + gidx], vs) : vs, cmk(c, -s));
        }
        zd* out = cheb + ((int64_t)blockIdx.x * M + j) * 3 * (nc + 1);
        for (int k = 0; k <= nc; ++k) {
            zd a = cmk(0.0, 0.0);
            for (int i = 0; i <= nc; ++i) {
                double w = cospi((double)((i * k) % (2 * nc)) / (double)nc);
                if (i == 0 || i == nc) w *= 0.5;
                a = cadd(a, cmk(w * G[i].re, w * G[i].im));
            }
            double sc = 2.0 / (double)nc;
            if (k == 0 || k == nc) sc *= 0.5;
            out[k] = cmk(sc * a.re, sc * a.im);
        }
        // p^(d)(+-1) = sum_k alpha_k T_k^(d)(+-1), T_k^(d)(1) = prod_{l<d} (k^2 - l^2)/(2l + 1),
        // T_k^(d)(-1) = (-1)^(k+d) T_k^(d)(1)
        for (int d = 0; d <= nc; ++d) {
            zd pp = cmk(0.0, 0.0), pm = cmk(0.0, 0.0);
            for (int k = d; k <= nc; ++k) {
                double t = 1.0;
                for (int l = 0; l < d; ++l) t *= (double)(k * k - l * l) / (double)(2 * l + 1);
                const double sg = ((k + d) & 1) ? -1.0 : 1.0;
                pp = cadd(pp, cmk(t * out[k].re, t * out[k].im));
                pm = cadd(pm, cmk(sg * t * out[k].re, sg * t * out[k].im));
            }
            out[nc + 1 + d] = pp;
            out[2 * (nc + 1) + d] = pm;
        }
    }
}

// u[r][t] for every time of one point: a workgroup per (point, run of 256
// times), a thread per time; the window's coefficients are staged in LDS.
// taylor[k][p] = int_{-1}^{1} T_k(x) x^p dx (p < LF_TAYLOR) for the moments
// at |kappa| < LF_KAPPA_SWITCH; above it, integration by parts.
#define LF_TAYLOR 40
#define LF_KAPPA_SWITCH 6.0
__global__ __launch_bounds__(LF_THREADS) void k_lf_synth(const zd* __restrict__ cfs, const zd* __restrict__ cheb,
                                                        const int64_t* __restrict__ klist, int K,
                                                        const double* __restrict__ mu, const double* __restrict__ taylor,
                                                        const double* __restrict__ times, int N_t, int N_r, int n,
                                                        int M, int nc, double h, double omega_c, double H,
                                                        double tau0, double* __restrict__ u) {
    extern __shared__ zd lds[];
    const int L = n + FC_C;
    zd* cs = lds;                 // [L] coefficients of the window
    zd* tw2 = lds + L;            // [L] e^{i pi m (n - 1) / L}
    zd* ch = lds + 2 * L;         // [M][3][nc + 1]
    const int r = blockIdx.y;
    const int ti = blockIdx.x * LF_THREADS + threadIdx.x;
    const double t = ti < N_t ? times[ti] : 0.0;
    const double D = (double)(n - 1) * h;
    for (int mi = threadIdx.x; mi < L; mi += LF_THREADS) {
        const int64_t m = mi - L / 2;
        const int64_t a = ((m * (int64_t)(n - 1)) % (2 * (int64_t)L) + 2 * (int64_t)L) % (2 * (int64_t)L);
        double s, c;
        sincospi((double)a / (double)L, &s, &c);
        tw2[mi] = cmk(c, s);
    }
    double acc = 0.0;
    const int nch = M * 3 * (nc + 1);
    for (int q = 0; q < K; ++q) {
        __syncthreads();
        const zd* cq = cfs + ((int64_t)q * N_r + r) * L;
        for (int mi = threadIdx.x; mi < L; mi += LF_THREADS) cs[mi] = cq[mi];
        const zd* chq = cheb + ((int64_t)q * N_r + r) * nch;
        for (int i = threadIdx.x; i < nch; i += LF_THREADS) ch[i] = chq[i];
        __syncthreads();
        const double sk = 1.5 * H * ((double)klist[q] - 1.0);
        const double tp = t - sk - tau0;
        // I_+: sum_m c_m e^{i x_m} D sinc(x_m), x_m = pi m (n-1)/L - t' D / 2
        double s, c;
        sincos(-0.5 * tp * D, &s, &c);
        const zd z = cmk(c, s);
        const double half = 0.5 * tp * D;
        zd ip = cmk(0.0, 0.0);
        for (int mi = 0; mi < L; ++mi) {
            const double xm = FHW_PI * (double)(mi - L / 2) * (double)(n - 1) / (double)L - half;
            const zd e = cmul(tw2[mi], z);
            double sn;
            if (fabs(xm) >= 0.25) {
                sn = e.im / xm;
            } else {
                sn = xm == 0.0 ? 1.0 : sin(xm) / xm;
            }
            ip = cfma(ip, cs[mi], cmk(D * sn * e.re, D * sn * e.im));
        }
        double so, co;
        sincos(omega_c * tp, &so, &co);
        ip = cmul(ip, cmk(co, -so));
        // I_0: per subinterval rho e^{-i delta t'} int_{-1}^{1} p(x) e^{-i kappa x} dx
        zd i0 = cmk(0.0, 0.0);
        for (int j = 0; j < M; ++j) {
            const double rho = 0.5 * (mu[j + 1] - mu[j]), delta = 0.5 * (mu[j + 1] + mu[j]);
            const double kap = rho * tp;
            const zd* al = ch + j * 3 * (nc + 1);
            zd val = cmk(0.0, 0.0);
            if (fabs(kap) < LF_KAPPA_SWITCH) {
                // m_k = sum_p (-i kappa)^p / p! int T_k x^p
                for (int k = 0; k <= nc; ++k) {
                    zd mk = cmk(0.0, 0.0);
                    zd pw = cmk(1.0, 0.0);   // (-i kappa)^p / p!
                    for (int p = 0; p < LF_TAYLOR; ++p) {
                        const double tk = taylor[k * LF_TAYLOR + p];
                        mk = cadd(mk, cmk(tk * pw.re, tk * pw.im));
                        pw = cmul(pw, cmk(0.0, -kap / (double)(p + 1)));
                    }
                    val = cfma(val, al[k], mk);
                }
            } else {
                // sum_d (-1)^d / s^(d+1) (p^(d)(1) e^{s} - p^(d)(-1) e^{-s}), s = -i kappa
                double sk2, ck2;
                sincos(kap, &sk2, &ck2);
                const zd ep = cmk(ck2, -sk2), em = cmk(ck2, sk2);
                const zd inv_s = cmk(0.0, 1.0 / kap);   // 1 / (-i kappa)
                zd fac = inv_s;
                for (int d = 0; d <= nc; ++d) {
                    const zd term = csub(cmul(al[nc + 1 + d], ep), cmul(al[2 * (nc + 1) + d], em));
                    const zd tf = (d & 1) ? cmk(-fac.re, -fac.im) : fac;
                    val = cfma(val, tf, term);
                    fac = cmul(fac, inv_s);
                }
            }
            double sd, cd;
            sincos(delta * tp, &sd, &cd);
            i0 = cfma(i0, cmk(rho * cd, -rho * sd), val);
        }
        acc += (ip.re + i0.re) / FHW_PI;
    }
    if (ti < N_t) u[(int64_t)r * N_t + ti] = acc;
}

int lf_max_points(void) { return 2048 - FC_C; }
int lf_fc_points(void) { return FC_C; }
int lf_taylor_terms(void) { return LF_TAYLOR; }

hipError_t launch_lf_coeffs(hipStream_t s, const void* B, const double* om, int n_om, const void* V, const void* Vs,
                            int N_r, int F, int jc, int n, int M, int nc, double tau0, int K, void* cfs, void* cheb,
                            int64_t v_qstride, int64_t vs_qstride) {
    if (n < FC_D || n + FC_C > 2048 || nc < 1 || nc > 32 || K < 1 || N_r < 1) return hipErrorInvalidValue;
    const size_t lds = (size_t)2 * (n + FC_C) * sizeof(zd);
    static std::atomic<uint64_t> attr{0};
    fhw_once_on_device(attr, [&] {
        (void)hipFuncSetAttribute((const void*)k_lf_coeffs, hipFuncAttributeMaxDynamicSharedMemorySize, 65536);
    });
    hipLaunchKernelGGL(k_lf_coeffs, dim3((unsigned)(K * N_r)), dim3(LF_THREADS), lds, s, (const zd*)B, om, n_om,
                       (const zd*)V, (const zd*)Vs, v_qstride, vs_qstride, N_r, F, jc, n, M, nc, tau0, (zd*)cfs,
                       (zd*)cheb);
    return hipGetLastError();
}

hipError_t launch_lf_synth(hipStream_t s, const void* cfs, const void* cheb, const int64_t* klist, int K,
                           const double* mu, const double* taylor, const double* times, int N_t, int N_r, int n,
                           int M, int nc, double h, double omega_c, double H, double tau0, double* u) {
    if (N_t < 1 || N_r < 1 || N_r > 65535) return hipErrorInvalidValue;
    const size_t lds = ((size_t)2 * (n + FC_C) + (size_t)M * 3 * (nc + 1)) * sizeof(zd);
    if (lds > 65536) return hipErrorInvalidValue;
    static std::atomic<uint64_t> attr{0};
    fhw_once_on_device(attr, [&] {
        (void)hipFuncSetAttribute((const void*)k_lf_synth, hipFuncAttributeMaxDynamicSharedMemorySize, 65536);
    });
    hipLaunchKernelGGL(k_lf_synth, dim3((unsigned)((N_t + LF_THREADS - 1) / LF_THREADS), (unsigned)N_r),
                       dim3(LF_THREADS), lds, s, (const zd*)cfs, (const zd*)cheb, klist, K, mu, taylor, times, N_t,
                       N_r, n, M, nc, h, omega_c, H, tau0, u);
    return hipGetLastError();
}
