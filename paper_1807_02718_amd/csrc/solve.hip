// Triangular solves with the batched LU factors and FP64-residual iterative
// refinement (step F3; the mixed-precision variant keeps the complex64 factors
// and corrects with residuals g - A psi computed from the FP64 matrix).
#include "fhw_device.h"
#include "fhw_internal.h"

#define NB FHW_LU_NB
#define SOLVE_THREADS 256

// One workgroup per matrix; x (complex128, length N) lives in LDS.
// Forward: per panel, replay the panel's swaps, multiply by the inverse of
// the unit-lower diagonal block, subtract L21 * y from the rows below.
// Backward: per panel from the last, subtract U12 * x from the block's rows,
// multiply by the inverse of U11.
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
    // ---- forward
    for (int p = 0; p < np; ++p) {
        const int k0 = p * NB;
        const int nb = min(NB, N - k0);
        if (tid == 0) {
            for (int jj = 0; jj < nb; ++jj) {
                const int r2 = piv[k0 + jj];
                if (r2 != k0 + jj) {
                    zd t = xs[k0 + jj];
                    xs[k0 + jj] = xs[r2];
                    xs[r2] = t;
                }
            }
        }
        __syncthreads();
        const cpx<T>* D = Lb + (int64_t)p * NB * NB;
        zd y = cmk(0.0, 0.0);
        if (tid < nb) {
            y = xs[k0 + tid];
            for (int c = 0; c < tid; ++c) {
                cpx<T> l = D[tid * NB + c];
                y = cfma(y, cmk((double)l.re, (double)l.im), xs[k0 + c]);
            }
        }
        __syncthreads();
        if (tid < nb) xs[k0 + tid] = y;
        __syncthreads();
        // rows below: 8 lanes per row, each lane 8 consecutive columns
        const int grp = tid >> 3, sub = tid & 7;
        for (int i0 = k0 + nb; i0 < N; i0 += SOLVE_THREADS / 8) {
            const int i = i0 + grp;
            zd s = cmk(0.0, 0.0);
            if (i < N) {
                const cpx<T>* Lrow = LU + (int64_t)i * N + k0;
#pragma unroll
                for (int q = 0; q < 8; ++q) {
                    const int c = sub * 8 + q;
                    if (c < nb) {
                        cpx<T> l = Lrow[c];
                        s = cfma(s, cmk((double)l.re, (double)l.im), xs[k0 + c]);
                    }
                }
            }
#pragma unroll
            for (int off = 1; off < 8; off <<= 1) {
                s.re += __shfl_xor(s.re, off, 64);
                s.im += __shfl_xor(s.im, off, 64);
            }
            if (i < N && sub == 0) xs[i] = csub(xs[i], s);
        }
        __syncthreads();
    }
    // ---- backward
    __shared__ zd rhs[NB];
    for (int p = np - 1; p >= 0; --p) {
        const int k0 = p * NB;
        const int nb = min(NB, N - k0);
        const int c0 = k0 + nb;
        // rhs_r = x[k0+r] - sum_{c >= c0} U[k0+r][c] x[c]; one wave per row
        for (int r = wid; r < nb; r += SOLVE_THREADS / 64) {
            const cpx<T>* Urow = LU + (int64_t)(k0 + r) * N;
            zd s = cmk(0.0, 0.0);
            for (int c = c0 + lane; c < N; c += 64) {
                cpx<T> u = Urow[c];
                s = cfma(s, cmk((double)u.re, (double)u.im), xs[c]);
            }
            s.re = wave_sum(s.re);
            s.im = wave_sum(s.im);
            if (lane == 0) rhs[r] = csub(xs[k0 + r], s);
        }
        __syncthreads();
        const cpx<T>* D = Lb + (int64_t)p * NB * NB;
        zd y = cmk(0.0, 0.0);
        if (tid < nb) {
            for (int c = tid; c < nb; ++c) {
                cpx<T> u = D[tid * NB + c];
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

// r = g - A x with the FP64 matrix; norms[2b] = ||r||_2, norms[2b+1] = ||g||_2.
// Marks done[b] (and sweeps[b] = sweep) once ||r|| <= tol ||g||.  Matrices
// already done are skipped.  Fixed-order reductions (deterministic).
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
    for (int i = wid; i < N; i += SOLVE_THREADS / 64) {
        const zd* Arow = A + (int64_t)i * N;
        zd s = cmk(0.0, 0.0);
        for (int c = lane; c < N; c += 64) s = cfma(s, Arow[c], xs[c]);
        s.re = wave_sum(s.re);
        s.im = wave_sum(s.im);
        const zd gi = gb[i];
        const zd ri = csub(gi, s);
        if (lane == 0) rb[i] = ri;
        rr += ri.re * ri.re + ri.im * ri.im;
        gg += gi.re * gi.re + gi.im * gi.im;
    }
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
