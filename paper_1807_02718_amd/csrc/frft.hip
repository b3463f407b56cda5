// Fast scaled convolution for time samples on a uniform grid (Sec. 4.1.2, FFT
// accelerated evaluation of scaled discrete convolutions, eqs. conv_sum and
// approx_conv_sum; the fractional DFT of Bailey & Swarztrauber, evaluated in
// Bluestein's chirp-z form).
//
// For window k, point r and a chunk of consecutive grid times whose kernel
// arguments are x_i = xs + beta i (beta = W dt / pi), with a_m = Re c_{k,m}(r),
// m = -F..F-1, the sum d(x) = sum_m a_m sinc(x - m) is replaced by
//   d(x) ~= (1/L) sum_{p=-L/2}^{L/2-1} C_p B_p e^{2 pi i p x / L},
//   C_p = sum_m a_m e^{-2 pi i m p / L}   (gamma = 1).
// The coefficients span the whole period of the band, so the kernel samples
// sinc(q) at the integers form the unit impulse and B_p = 1.  With
// 2 i p = i^2 + p^2 - (i - p)^2 the sum over p for all i of a chunk is one
// linear convolution,
//   d(xs + beta i) = e^{i pi beta i^2 / L} sum_{P=0}^{L-1} z_P h(i - P),
//   z_P = C_p e^{2 pi i p xs / L} e^{i pi beta p^2 / L} / L,   p = P - L/2,
//   h(j) = e^{-i pi beta (j + L/2)^2 / L},   j = -(L-1) .. NC-1,
// taken as a circular convolution of length Q >= NC + L - 1 in LDS.
#include "fhw_device.h"
#include "fhw_internal.h"
#include "lds_fft.h"

#define FRFT_THREADS 1024
#define FRFT_QMAX 8192
#define FRFT_PER (FRFT_QMAX / FRFT_THREADS)

__device__ __forceinline__ int frft_brev(int i, int logn) { return (int)(__brev((unsigned)i) >> (32 - logn)); }

// e^{i pi v s} for an exactly representable s: the rounding error of v s is
// recovered with an fma and the product reduced modulo 2 (exactly) before
// sincospi, so large arguments keep full absolute accuracy.
__device__ __forceinline__ zd frft_expipi(double v, double s) {
    const double t = v * s;
    const double e = fma(v, s, -t);
    const double rdc = t - 2.0 * floor(0.5 * t);
    double sn, cs;
    sincospi(rdc + e, &sn, &cs);
    return cmk(cs, sn);
}

// Spectrum of the chirp h (laid out circularly over Q), divided by Q so that
// the inverse transform of the product needs no further scaling; and the
// chirps shared by every chunk and point: cin[P] = e^{i pi beta p^2 / L} / L,
// p = P - L/2, P < L, and cout[i] = e^{i pi beta i^2 / L}, i < NC.
__global__ __launch_bounds__(FRFT_THREADS) void k_frft_chirp(int L, int NC, int Q, int logQ, double beta,
                                                             zd* __restrict__ Hs,
                                                             zd* __restrict__ cin, zd* __restrict__ cout) {
    extern __shared__ zd X[];
    const double il = 1.0 / (double)L;
    for (int P = threadIdx.x; P < L; P += FRFT_THREADS) {
        const double p = (double)(P - L / 2);
        const zd w = frft_expipi(beta, p * p * il);
        cin[P] = cmk(w.re * il, w.im * il);
    }
    for (int i = threadIdx.x; i < NC; i += FRFT_THREADS) cout[i] = frft_expipi(beta, (double)i * (double)i * il);
    __shared__ zd thi[64], tlo[64];
    fft_tables(thi, tlo, Q);
    for (int pos = threadIdx.x; pos < Q; pos += FRFT_THREADS) {
        zd v = cmk(0.0, 0.0);
        int j = 0;
        bool used = false;
        if (pos < NC) { j = pos; used = true; }
        else if (pos >= Q - (L - 1)) { j = pos - Q; used = true; }
        if (used) {
            const double jj = (double)(j + L / 2);
            v = frft_expipi(-beta, jj * jj / (double)L);
        }
        X[frft_brev(pos, logQ)] = v;
    }
    __syncthreads();
    lds_fft<FRFT_THREADS, FRFT_QMAX>(X, logQ, thi, tlo, logQ);
    const double iq = 1.0 / (double)Q;
    for (int k = threadIdx.x; k < Q; k += FRFT_THREADS) Hs[k] = cmk(X[k].re * iq, X[k].im * iq);
}

// One workgroup per (chunk, point r): adds scale * d(x_i) into u[r][n0 + i],
// i < n.  The chunks of one launch cover disjoint time ranges.
__global__ __launch_bounds__(FRFT_THREADS) void k_frft(const double* __restrict__ cre,
                                                       const fhw_frft_chunk* __restrict__ chunks, int N_r, int F,
                                                       int L, int logL, int Q, int logQ, double beta, double scale,
                                                       const zd* __restrict__ Hs, const zd* __restrict__ cin, const zd* __restrict__ cout,
                                                       double* __restrict__ u, int64_t N_t,
                                                       const double* __restrict__ bnd,
                                                       const unsigned long long* __restrict__ gmax, double tol) {
    extern __shared__ zd X[];
    __shared__ zd thi[64], tlo[64];
    const fhw_frft_chunk ch = chunks[blockIdx.x];
    const int r = blockIdx.y;
    // tracking: the whole workgroup leaves before its first barrier
    if (bnd && bnd[(int64_t)ch.slot * N_r + r] <= tol * __longlong_as_double((long long)*gmax)) return;
    fft_tables(thi, tlo, Q);
    const int M = 2 * F;
    const double* a = cre + ((int64_t)ch.slot * N_r + r) * M;
    // a_m at index m mod L, zero elsewhere, in bit-reversed order
    for (int idx = threadIdx.x; idx < L; idx += FRFT_THREADS) {
        const int m = idx < L / 2 ? idx : idx - L;
        const double v = (m >= -F && m < F) ? a[m + F] : 0.0;
        X[frft_brev(idx, logL)] = cmk(v, 0.0);
    }
    __syncthreads();
    // C_p = FFT(a) lands at K = p mod L in the final pass; z_P, P = p + L/2,
    // goes straight to the convolution buffer's bit-reversed slot.  A thread's
    // outputs K = t + e L/8 have p = t + d L/8 with d = e (e < 4) or e - 8,
    // so the phase ramp e^{2 pi i p xs / L} is r0 st^d, st = e^{i pi xs / 4}.
    const double il = 1.0 / (double)L;
    const int sh = logL - 3;
    const zd r0 = frft_expipi(ch.xs, 2.0 * (double)threadIdx.x * il);
    const zd st = frft_expipi(ch.xs, 0.25);
    zd pw[8];
    pw[0] = r0;
#pragma unroll
    for (int e = 1; e < 4; ++e) pw[e] = cmul(pw[e - 1], st);
    pw[7] = cmul(r0, cconj(st));
#pragma unroll
    for (int e = 6; e >= 4; --e) pw[e] = cmul(pw[e + 1], cconj(st));
    lds_fft_epi<FRFT_THREADS, FRFT_QMAX, true>(
        X, logL, thi, tlo, logQ,
        [&](int K, zd c) {
            const int P = (K + L / 2) & (L - 1);
            return cmul(cmul(c, pw[(K - (int)threadIdx.x) >> sh]), cin[P]);
        },
        [&](int K, zd z) { X[frft_brev((K + L / 2) & (L - 1), logQ)] = z; });
    for (int P = L + threadIdx.x; P < Q; P += FRFT_THREADS) X[frft_brev(P, logQ)] = cmk(0.0, 0.0);
    __syncthreads();
    // forward transform; its outputs times the chirp spectrum, conjugated,
    // go to bit-reversed slots for the inverse as conj(FFT(conj))
    lds_fft_epi<FRFT_THREADS, FRFT_QMAX, true>(
        X, logQ, thi, tlo, logQ, [&](int K, zd v) { return cconj(cmul(v, Hs[K])); },
        [&](int K, zd w) { X[frft_brev(K, logQ)] = w; });
    __syncthreads();
    // inverse transform; output i = conj(X_i) times the output chirp
    double* ur = u + (int64_t)r * N_t + ch.n0;
    lds_fft_epi<FRFT_THREADS, FRFT_QMAX, false>(
        X, logQ, thi, tlo, logQ, [&](int K, zd v) { return v; },
        [&](int K, zd v) {
            if (K < ch.n) {
                const zd w = cout[K];
                ur[K] += scale * (w.re * v.re + w.im * v.im);
            }
        });
}

int frft_max_q(int lds_bytes) {
    int q = FRFT_QMAX;
    while (q > 2 && (size_t)q * sizeof(zd) > (size_t)lds_bytes) q >>= 1;
    return q;
}

static int ilog2(int v) {
    int l = 0;
    while ((1 << l) < v) ++l;
    return l;
}

hipError_t launch_frft_setup(hipStream_t s, int L, int NC, int Q, double beta, void* Hs, void* cin, void* cout) {
    if (Q > FRFT_QMAX || Q < 2 || (Q & (Q - 1)) || L > Q || NC < 1 || NC + L - 1 > Q) return hipErrorInvalidValue;
    static std::atomic<uint64_t> attr{0};
    fhw_once_on_device(attr, [&] {
        const int dyn = FRFT_QMAX * (int)sizeof(zd);
        (void)hipFuncSetAttribute((const void*)k_frft_chirp, hipFuncAttributeMaxDynamicSharedMemorySize, dyn);
        (void)hipFuncSetAttribute((const void*)k_frft, hipFuncAttributeMaxDynamicSharedMemorySize, dyn);
    });
    hipLaunchKernelGGL(k_frft_chirp, dim3(1), dim3(FRFT_THREADS), (size_t)Q * sizeof(zd), s, L, NC, Q, ilog2(Q), beta,
                       (zd*)Hs, (zd*)cin, (zd*)cout);
    return hipGetLastError();
}

hipError_t launch_frft(hipStream_t s, const double* c_re, const fhw_frft_chunk* d_chunks, int32_t n_chunks,
                       int32_t N_r, int32_t F, int32_t L, int32_t Q, double beta, double scale, const void* Hs,
                       const void* cin, const void* cout, double* u, int64_t N_t,
                       const double* bnd, const unsigned long long* gmax, double tol) {
    if (n_chunks <= 0 || N_r <= 0) return hipSuccess;
    if (N_r > 65535 || Q > FRFT_QMAX || L > Q || L < 8 || 2 * F > L) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_frft, dim3(n_chunks, N_r), dim3(FRFT_THREADS), (size_t)Q * sizeof(zd), s, c_re, d_chunks,
                       N_r, F, L, ilog2(L), Q, ilog2(Q), beta, scale, (const zd*)Hs, (const zd*)cin,
                       (const zd*)cout, u, N_t, bnd, gmax, tol);
    return hipGetLastError();
}
