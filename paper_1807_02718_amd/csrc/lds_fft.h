// LDS radix-2^3 FFT shared by the Fourier-coefficient and fast
// scaled-convolution kernels.
#pragma once
#include "fhw_device.h"

// Twiddle e^{-2 pi i j / Q}, j < Q/2 <= 4096, as the product of two LDS
// table entries: thi[a] = e^{-2 pi i 64 a / Q}, tlo[b] = e^{-2 pi i b / Q}.
__device__ __forceinline__ zd fft_tw(const zd* thi, const zd* tlo, int j) { return cmul(thi[j >> 6], tlo[j & 63]); }

// The two 64-entry tables for a transform length Q, by sincospi (the caller
// synchronizes before use).
__device__ __forceinline__ void fft_tables(zd* thi, zd* tlo, int Q) {
    if (threadIdx.x < 64) {
        const int t = threadIdx.x;
        double sn, cs;
        sincospi(-2.0 * (double)t / (double)Q, &sn, &cs);
        tlo[t] = t < Q / 2 ? cmk(cs, sn) : cmk(1.0, 0.0);
        sincospi(-2.0 * (double)(64 * t) / (double)Q, &sn, &cs);
        thi[t] = 64 * t < Q / 2 ? cmk(cs, sn) : cmk(1.0, 0.0);
    }
}

// One radix-2 DIT stage of half-length h on two values in registers.
__device__ __forceinline__ void fft_bfly(zd& a, zd& b, zd w) {
    const zd t = cmul(b, w);
    b = csub(a, t);
    a = cadd(a, t);
}

// One radix-2^3 group: the stages of half-lengths h, 2h and 4h on x[e] =
// X[i0 + e h], e < 8, with pos = i0 mod h, for the stage index lg of the
// first (half-length h = 2^(lg-1)).
__device__ __forceinline__ void fft_radix8(zd (&x)[8], const zd* thi, const zd* tlo, int pos, int lg, int logQ) {
    // one table twiddle w8 = W_{8h}^pos; the others from it:
    // W_{4h}^pos = w8^2, W_{2h}^pos = w8^4, W_{4h}^{pos+h} = -i W_{4h}^pos,
    // W_{8h}^{pos+h} = W_8 w8, W_{8h}^{pos+2h} = -i w8, W_{8h}^{pos+3h} = -i W_{8h}^{pos+h}
    const zd w8 = fft_tw(thi, tlo, pos << (logQ - lg - 2));
    const zd w4 = cmul(w8, w8);
    const zd w2 = cmul(w4, w4);
#pragma unroll
    for (int e = 0; e < 8; e += 2) fft_bfly(x[e], x[e + 1], w2);
    const zd w4b = cmk(w4.im, -w4.re);
    fft_bfly(x[0], x[2], w4);
    fft_bfly(x[4], x[6], w4);
    fft_bfly(x[1], x[3], w4b);
    fft_bfly(x[5], x[7], w4b);
    const zd w8b = cmul(w8, cmk(FHW_INV_SQRT2, -FHW_INV_SQRT2));
    fft_bfly(x[0], x[4], w8);
    fft_bfly(x[1], x[5], w8b);
    fft_bfly(x[2], x[6], cmk(w8.im, -w8.re));
    fft_bfly(x[3], x[7], cmk(w8b.im, -w8b.re));
}

// The passes of the FFT below, all of them (last = true) or all but the
// final radix-2^3 pass (last = false, logS >= 3).
template <int TH, int SMAX>
__device__ void lds_fft_passes(zd* X, int logS, const zd* thi, const zd* tlo, int logQ, bool last) {
    const int S = 1 << logS;
    int lg = 1;
    const int lead = logS % 3;
    if (lead == 1) {
#pragma unroll
        for (int k = 0; k < (SMAX / 2 + TH - 1) / TH; ++k) {
            const int t = threadIdx.x + k * TH;
            if (t < (S >> 1)) {
                zd a = X[2 * t], b = X[2 * t + 1];
                fft_bfly(a, b, cmk(1.0, 0.0));
                X[2 * t] = a;
                X[2 * t + 1] = b;
            }
        }
        __syncthreads();
        lg = 2;
    } else if (lead == 2) {
#pragma unroll
        for (int k = 0; k < (SMAX / 4 + TH - 1) / TH; ++k) {
            const int t = threadIdx.x + k * TH;
            if (t < (S >> 2)) {
                // stages of half-lengths 1 and 2 on x[4t .. 4t+3]
                zd x0 = X[4 * t], x1 = X[4 * t + 1], x2 = X[4 * t + 2], x3 = X[4 * t + 3];
                fft_bfly(x0, x1, cmk(1.0, 0.0));
                fft_bfly(x2, x3, cmk(1.0, 0.0));
                fft_bfly(x0, x2, cmk(1.0, 0.0));
                fft_bfly(x1, x3, fft_tw(thi, tlo, 1 << (logQ - 2)));
                X[4 * t] = x0;
                X[4 * t + 1] = x1;
                X[4 * t + 2] = x2;
                X[4 * t + 3] = x3;
            }
        }
        __syncthreads();
        lg = 3;
    }
    const int lg_end = last ? logS : logS - 3;
    for (; lg + 2 <= lg_end; lg += 3) {
        const int h = 1 << (lg - 1);
#pragma unroll
        for (int k = 0; k < (SMAX / 8 + TH - 1) / TH; ++k) {
            const int t = threadIdx.x + k * TH;
            if (t < (S >> 3)) {
                const int pos = t & (h - 1);
                const int i0 = ((t >> (lg - 1)) << (lg + 2)) + pos;
                zd x[8];
#pragma unroll
                for (int e = 0; e < 8; ++e) x[e] = X[i0 + e * h];
                fft_radix8(x, thi, tlo, pos, lg, logQ);
#pragma unroll
                for (int e = 0; e < 8; ++e) X[i0 + e * h] = x[e];
            }
        }
        __syncthreads();
    }
}

// In-place decimation-in-time FFT of length S = 2^logS (S <= Q, S <= SMAX)
// by a workgroup of TH threads, of LDS data stored in bit-reversed order:
// X_k = sum_j x_j e^{-2 pi i j k / S}.  The radix-2 stages go three at a
// time (radix 2^3, fft_radix8); one or two leading stages go two at a time
// or alone so that the rest divides by three.  Ends with a barrier.
template <int TH, int SMAX>
__device__ void lds_fft(zd* X, int logS, const zd* thi, const zd* tlo, int logQ) {
    lds_fft_passes<TH, SMAX>(X, logS, thi, tlo, logQ, true);
}

// The same transform with the final radix-2^3 pass kept in registers: for
// every output k, v = pre(k, X_k) before a barrier (when SYNC), then
// post(k, v) after it, in place of the store of X_k (the output is not
// written back).  With SYNC, post may write LDS that other threads read in
// the final pass.  Needs logS >= 3 and S / 8 <= TH (one group per thread).
template <int TH, int SMAX, bool SYNC, class Pre, class Post>
__device__ void lds_fft_epi(zd* X, int logS, const zd* thi, const zd* tlo, int logQ, Pre pre, Post post) {
    static_assert(SMAX / 8 <= TH, "one radix-2^3 group per thread in the final pass");
    lds_fft_passes<TH, SMAX>(X, logS, thi, tlo, logQ, false);
    const int S = 1 << logS;
    const int lg = logS - 2;
    const int h = S >> 3;
    const int t = threadIdx.x;
    const bool act = t < h;
    zd y[8];
    if (act) {
        zd x[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) x[e] = X[t + e * h];
        fft_radix8(x, thi, tlo, t, lg, logQ);
#pragma unroll
        for (int e = 0; e < 8; ++e) y[e] = pre(t + e * h, x[e]);
    }
    if (SYNC) __syncthreads();
    if (act) {
#pragma unroll
        for (int e = 0; e < 8; ++e) post(t + e * h, y[e]);
    }
}


