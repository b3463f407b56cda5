// Triangular solves with the batched LU factors and FP64-residual iterative
// refinement (step F3; the mixed-precision variant keeps the complex64 factors
// and corrects with residuals g - A psi computed from the FP64 matrix).
#include "fhw_device.h"
#include "fhw_internal.h"

#define NB FHW_LU_NB
#define SOLVE_THREADS 256

// row swaps of one panel (LAPACK order: row k0+jj with row piv[k0+jj])
__device__ __forceinline__ void replay_pivots(zd* xs, const int* piv, int k0, int nb) {
    for (int jj = 0; jj < nb; ++jj) {
        const int r2 = piv[k0 + jj];
        if (r2 != k0 + jj) {
            const zd t = xs[k0 + jj];
            xs[k0 + jj] = xs[r2];
            xs[r2] = t;
        }
    }
}

// One workgroup per matrix; x (complex128, length N) lives in LDS.  Factors
// are column-major (entry (r, c) at c*N + r); linv blocks hold the inverses
// of the diagonal blocks (column-major 64x64).
// Forward: per panel, replay the panel's swaps, multiply by the inverse of
// the unit-lower diagonal block, subtract L21 * y from the rows below (one
// thread per row, coalesced down the columns); pivot order as the paired
// factorization left it (below).
// Backward: per panel from the last, subtract U12 * x from the block's rows
// (one lane per row, waves over columns), multiply by the inverse of U11.
template <typename T>
__global__ __launch_bounds__(SOLVE_THREADS) void k_lu_solve(const int* __restrict__ Ns,
                                                            const int64_t* __restrict__ a_off,
                                                            const int64_t* __restrict__ piv_off,
                                                            const int64_t* __restrict__ linv_off,
                                                            const int64_t* __restrict__ v_off,
                                                            const cpx<T>* __restrict__ LUbase,
                                                            const int* __restrict__ pivbase,
                                                            const cpx<T>* __restrict__ linvbase, zd* __restrict__ v,
                                                            zd* __restrict__ acc, const int* __restrict__ skip) {
    extern __shared__ zd xs[];
    __shared__ zd rhs[NB];
    __shared__ zd part[SOLVE_THREADS / 64][NB];
    const int b = blockIdx.x;
    if (skip && skip[b]) return;
    const int N = Ns[b];
    const cpx<T>* LU = LUbase + a_off[b];
    const int* piv = pivbase + piv_off[b];
    const cpx<T>* Lb = linvbase + linv_off[b];
    zd* vb = v + v_off[b];
    const int tid = threadIdx.x;
    const int lane = tid & 63, wid = tid >> 6;
    for (int i = tid; i < N; i += SOLVE_THREADS) xs[i] = vb[i];
    const int np = (N + NB - 1) / NB;
    __syncthreads();
    // ---- forward.  Panels were factored in pairs (2q, 2q+1) and panel 2q's
    // L rows below the pair's first panel carry the pivots of panel 2q+1, so
    // those pivots are replayed before panel 2q's update of the rows below.
    for (int p = 0; p < np; ++p) {
        const int k0 = p * NB;
        const int nb = min(NB, N - k0);
        if (tid == 0 && (p & 1) == 0) replay_pivots(xs, piv, k0, nb);
        __syncthreads();
        const cpx<T>* D = Lb + (int64_t)p * NB * NB;
        zd y = cmk(0.0, 0.0);
        if (tid < nb) {
            y = xs[k0 + tid];
            for (int c = 0; c < tid; ++c) {
                const cpx<T> l = D[c * NB + tid];
                y = cfma(y, cmk((double)l.re, (double)l.im), xs[k0 + c]);
            }
        }
        __syncthreads();
        if (tid < nb) xs[k0 + tid] = y;
        __syncthreads();
        if ((p & 1) == 0 && p + 1 < np) {
            if (tid == 0) replay_pivots(xs, piv, k0 + NB, min(NB, N - k0 - NB));
            __syncthreads();
        }
        for (int i = k0 + nb + tid; i < N; i += SOLVE_THREADS) {
            const cpx<T>* Li = LU + (int64_t)k0 * N + i;
            // eight independent partial sums: eight loads in flight per thread
            zd s8[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) s8[u] = cmk(0.0, 0.0);
            int c = 0;
            for (; c + 8 <= nb; c += 8) {
                cpx<T> l8[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) l8[u] = Li[(int64_t)(c + u) * N];
#pragma unroll
                for (int u = 0; u < 8; ++u) s8[u] = cfma(s8[u], cmk((double)l8[u].re, (double)l8[u].im), xs[k0 + c + u]);
            }
            for (; c < nb; ++c) {
                const cpx<T> l = Li[(int64_t)c * N];
                s8[0] = cfma(s8[0], cmk((double)l.re, (double)l.im), xs[k0 + c]);
            }
            zd s = s8[0];
#pragma unroll
            for (int u = 1; u < 8; ++u) s = cadd(s, s8[u]);
            xs[i] = csub(xs[i], s);
        }
        __syncthreads();
    }
    // ---- backward
    for (int p = np - 1; p >= 0; --p) {
        const int k0 = p * NB;
        const int nb = min(NB, N - k0);
        const int c0 = k0 + nb;
        zd s = cmk(0.0, 0.0);
        if (lane < nb) {
            const cpx<T>* Ur = LU + k0 + lane;
            constexpr int NW = SOLVE_THREADS / 64;
            // four independent partial sums per lane: four loads in flight
            zd s4[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) s4[u] = cmk(0.0, 0.0);
            int c = c0 + wid;
            for (; c + 3 * NW < N; c += 4 * NW) {
                cpx<T> u4[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) u4[u] = Ur[(int64_t)(c + u * NW) * N];
#pragma unroll
                for (int u = 0; u < 4; ++u) s4[u] = cfma(s4[u], cmk((double)u4[u].re, (double)u4[u].im), xs[c + u * NW]);
            }
            for (; c < N; c += NW) {
                const cpx<T> u = Ur[(int64_t)c * N];
                s4[0] = cfma(s4[0], cmk((double)u.re, (double)u.im), xs[c]);
            }
            s = cadd(cadd(s4[0], s4[1]), cadd(s4[2], s4[3]));
        }
        part[wid][lane] = s;
        __syncthreads();
        if (tid < nb) {
            zd t = xs[k0 + tid];
#pragma unroll
            for (int q = 0; q < SOLVE_THREADS / 64; ++q) t = csub(t, part[q][tid]);
            rhs[tid] = t;
        }
        __syncthreads();
        const cpx<T>* D = Lb + (int64_t)p * NB * NB;
        zd y = cmk(0.0, 0.0);
        if (tid < nb) {
            for (int c = tid; c < nb; ++c) {
                const cpx<T> u = D[c * NB + tid];
                y = cfma(y, cmk((double)u.re, (double)u.im), rhs[c]);
            }
        }
        __syncthreads();
        if (tid < nb) xs[k0 + tid] = y;
        __syncthreads();
    }
    if (acc) {
        zd* ab = acc + v_off[b];
        for (int i = tid; i < N; i += SOLVE_THREADS) ab[i] = cadd(ab[i], xs[i]);
    } else {
        for (int i = tid; i < N; i += SOLVE_THREADS) vb[i] = xs[i];
    }
}

// r = g - A x with the FP64 column-major matrix; norms[2b] = ||r||_2,
// norms[2b+1] = ||g||_2.  Marks done[b] (and sweeps[b] = sweep) once
// ||r|| <= tol ||g||.  Matrices already done are skipped.  One thread per row,
// four rows at a time, coalesced down the columns; fixed-order reductions.
__global__ __launch_bounds__(SOLVE_THREADS) void k_residual(const int* __restrict__ Ns,
                                                            const int64_t* __restrict__ a_off,
                                                            const int64_t* __restrict__ v_off,
                                                            const zd* __restrict__ Abase, const zd* __restrict__ x,
                                                            const zd* __restrict__ g, zd* __restrict__ r,
                                                            double* __restrict__ norms, double tol,
                                                            int* __restrict__ done, int* __restrict__ sweeps,
                                                            int sweep) {
    extern __shared__ zd xs[];
    __shared__ double part[2][SOLVE_THREADS / 64];
    const int b = blockIdx.x;
    if (done && done[b]) return;
    const int N = Ns[b];
    const zd* A = Abase + a_off[b];
    const zd* xb = x + v_off[b];
    const zd* gb = g + v_off[b];
    zd* rb = r + v_off[b];
    const int tid = threadIdx.x;
    const int lane = tid & 63, wid = tid >> 6;
    for (int i = tid; i < N; i += SOLVE_THREADS) xs[i] = xb[i];
    __syncthreads();
    double rr = 0.0, gg = 0.0;
    constexpr int RB = 4;
    for (int i0 = 0; i0 < N; i0 += RB * SOLVE_THREADS) {
        zd s[RB];
#pragma unroll
        for (int q = 0; q < RB; ++q) s[q] = cmk(0.0, 0.0);
        for (int c = 0; c < N; ++c) {
            const zd xc = xs[c];
            const zd* Ac = A + (int64_t)c * N + i0 + tid;
#pragma unroll
            for (int q = 0; q < RB; ++q)
                if (i0 + tid + q * SOLVE_THREADS < N) s[q] = cfma(s[q], Ac[q * SOLVE_THREADS], xc);
        }
#pragma unroll
        for (int q = 0; q < RB; ++q) {
            const int i = i0 + tid + q * SOLVE_THREADS;
            if (i < N) {
                const zd gi = gb[i];
                const zd ri = csub(gi, s[q]);
                rb[i] = ri;
                rr += ri.re * ri.re + ri.im * ri.im;
                gg += gi.re * gi.re + gi.im * gi.im;
            }
        }
    }
    rr = wave_sum(rr);
    gg = wave_sum(gg);
    if (lane == 0) { part[0][wid] = rr; part[1][wid] = gg; }
    __syncthreads();
    if (tid == 0) {
        double R2 = 0.0, G2 = 0.0;
        for (int q = 0; q < SOLVE_THREADS / 64; ++q) { R2 += part[0][q]; G2 += part[1][q]; }
        norms[2 * b] = sqrt(R2);
        norms[2 * b + 1] = sqrt(G2);
        if (done && R2 <= tol * tol * G2) {
            done[b] = 1;
            if (sweeps) sweeps[b] = sweep;
        }
    }
}

__global__ void k_c128_to_c64(const zd* __restrict__ src, zf* __restrict__ dst, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) dst[i] = cmk((float)src[i].re, (float)src[i].im);
}

hipError_t launch_lu_solve(hipStream_t s, const fhw_batch_dev& b, int32_t maxN, const void* LU, const int32_t* piv,
                           const void* linv, void* x, const int32_t* d_skip, int precision) {
    return launch_lu_solve_acc(s, b, maxN, LU, piv, linv, x, nullptr, d_skip, precision);
}

hipError_t launch_lu_solve_acc(hipStream_t s, const fhw_batch_dev& b, int32_t maxN, const void* LU,
                               const int32_t* piv, const void* linv, void* x, void* acc, const int32_t* d_skip,
                               int precision) {
    size_t lds = (size_t)maxN * sizeof(zd);
    if (precision == FHW_FP64)
        hipLaunchKernelGGL((k_lu_solve<double>), dim3(b.batch), dim3(SOLVE_THREADS), lds, s, b.N, b.a_off, b.piv_off,
                           b.linv_off, b.v_off, (const zd*)LU, piv, (const zd*)linv, (zd*)x, (zd*)acc, d_skip);
    else
        hipLaunchKernelGGL((k_lu_solve<float>), dim3(b.batch), dim3(SOLVE_THREADS), lds, s, b.N, b.a_off, b.piv_off,
                           b.linv_off, b.v_off, (const zf*)LU, piv, (const zf*)linv, (zd*)x, (zd*)acc, d_skip);
    return hipGetLastError();
}

hipError_t launch_residual_t(hipStream_t s, const fhw_batch_dev& b, int32_t maxN, const void* A64, const void* x,
                             const void* g, void* r, double* norms, double tol, int32_t* done, int32_t* sweeps,
                             int sweep) {
    size_t lds = (size_t)maxN * sizeof(zd);
    hipLaunchKernelGGL(k_residual, dim3(b.batch), dim3(SOLVE_THREADS), lds, s, b.N, b.a_off, b.v_off, (const zd*)A64,
                       (const zd*)x, (const zd*)g, (zd*)r, norms, tol, done, sweeps, sweep);
    return hipGetLastError();
}

hipError_t launch_convert_c128_c64(hipStream_t s, const void* src, void* dst, int64_t n) {
    int blocks = (int)std::min<int64_t>((n + 255) / 256, 65536);
    hipLaunchKernelGGL(k_c128_to_c64, dim3(blocks), dim3(256), 0, s, (const zd*)src, (zf*)dst, n);
    return hipGetLastError();
}
