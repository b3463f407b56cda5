// Batched dense complex LU with partial pivoting on gfx950 (step F3: one
// Nystrom system per frequency), FP64 or FP32, ragged batches of row-major
// packed matrices.
//
// Right-looking, blocked by NB = 64 columns.  Per panel k0:
//   k_lu_panel   one 1024-thread workgroup per matrix factors the (N-k0) x 64
//                panel in sub-panels of W columns held in registers (pivot
//                search = wave shuffles + one LDS round, first index on ties),
//                applies the sub-panel swaps and updates inside the panel, and
//                writes the inverses of the 64x64 unit-lower and upper
//                diagonal blocks (used by the trailing TRSM and by the solves).
//   k_lu_swap    applies the 64 row swaps to the trailing columns.
//   k_lu_gemm    U12 = L11^{-1} A12 (in place) and A22 -= L21 U12, 64x64 tiles,
//                complex product as 4 real MFMA 16x16x4 products per k-step.
// Earlier panels' L columns are not permuted by later pivots; the solves
// replay the pivots panel by panel.
#include "fhw_device.h"
#include "fhw_internal.h"

#define NB FHW_LU_NB
#define PANEL_THREADS 1024

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

// linv block layout per matrix: panel p at linv_off + p*NB*NB, row-major 64x64:
// strictly lower part = inverse of the unit-lower L11, upper part incl. the
// diagonal = inverse of U11.

template <typename T>
__device__ __forceinline__ bool piv_better(T v, int i, T bv, int bi) {
    return (v > bv) || (v == bv && i < bi);
}

template <typename T, int R, int W>
__global__ __launch_bounds__(PANEL_THREADS) void k_lu_panel(int k0, const int* __restrict__ Ns,
                                                            const int64_t* __restrict__ a_off,
                                                            const int64_t* __restrict__ piv_off,
                                                            const int64_t* __restrict__ linv_off,
                                                            cpx<T>* __restrict__ Abase, int* __restrict__ piv,
                                                            cpx<T>* __restrict__ linv, int* __restrict__ status) {
    const int b = blockIdx.x;
    const int N = Ns[b];
    if (k0 >= N) return;
    const int nb = min(NB, N - k0);
    cpx<T>* A = Abase + a_off[b];
    const int tid = threadIdx.x;
    const int lane = tid & 63, wid = tid >> 6;

    __shared__ cpx<T> prow[W];
    __shared__ cpx<T> rowk[W];
    __shared__ T redv[PANEL_THREADS / 64];
    __shared__ int redi[PANEL_THREADS / 64];
    __shared__ int s_piv[NB];
    __shared__ cpx<T> L11s[W][W];
    __shared__ cpx<T> Ublk[W][NB];
    __shared__ int s_sing;
    if (tid == 0) s_sing = 0;

    cpx<T> a[R][W];

    for (int s = 0; s < nb; s += W) {
        const int w = min(W, nb - s);
        const int kc = k0 + s;
        // rows kc + tid + i*PANEL_THREADS belong to this thread
#pragma unroll
        for (int i = 0; i < R; ++i) {
            const int row = kc + tid + i * PANEL_THREADS;
#pragma unroll
            for (int q = 0; q < W; ++q)
                a[i][q] = (row < N && q < w) ? A[(int64_t)row * N + kc + q] : cmk((T)0, (T)0);
        }
#pragma unroll
        for (int j = 0; j < W; ++j) {
            if (j < w) {
                const int col = kc + j;
                T bv = (T)-1;
                int bi = 0x7fffffff;
#pragma unroll
                for (int i = 0; i < R; ++i) {
                    const int row = kc + tid + i * PANEL_THREADS;
                    if (row >= col && row < N) {
                        T v = cabs1(a[i][j]);
                        if (piv_better(v, row, bv, bi)) { bv = v; bi = row; }
                    }
                }
#pragma unroll
                for (int off = 32; off >= 1; off >>= 1) {
                    T ov = __shfl_xor(bv, off, 64);
                    int oi = __shfl_xor(bi, off, 64);
                    if (piv_better(ov, oi, bv, bi)) { bv = ov; bi = oi; }
                }
                if (lane == 0) { redv[wid] = bv; redi[wid] = bi; }
                __syncthreads();
                bv = redv[0]; bi = redi[0];
#pragma unroll
                for (int q = 1; q < PANEL_THREADS / 64; ++q)
                    if (piv_better(redv[q], redi[q], bv, bi)) { bv = redv[q]; bi = redi[q]; }
                // no candidate (NaN column) or zero column: keep the row, flag it
                const bool zero = !(bv > (T)0) || bi >= N;
                const int p = (bi >= N) ? col : bi;
                const int tp = (p - kc) % PANEL_THREADS, ip = (p - kc) / PANEL_THREADS;
                const int tc = (col - kc) % PANEL_THREADS, ic = (col - kc) / PANEL_THREADS;
                if (tid == tp) {
#pragma unroll
                    for (int i = 0; i < R; ++i)
                        if (i == ip) {
#pragma unroll
                            for (int q = 0; q < W; ++q) prow[q] = a[i][q];
                        }
                }
                if (tid == tc) {
#pragma unroll
                    for (int i = 0; i < R; ++i)
                        if (i == ic) {
#pragma unroll
                            for (int q = 0; q < W; ++q) rowk[q] = a[i][q];
                        }
                }
                if (tid == 0) {
                    s_piv[s + j] = p;
                    if (zero) s_sing = 1;
                }
                __syncthreads();
                if (tid == tc) {
#pragma unroll
                    for (int i = 0; i < R; ++i)
                        if (i == ic) {
#pragma unroll
                            for (int q = 0; q < W; ++q) a[i][q] = prow[q];
                        }
                }
                if (tid == tp && p != col) {
#pragma unroll
                    for (int i = 0; i < R; ++i)
                        if (i == ip) {
#pragma unroll
                            for (int q = 0; q < W; ++q) a[i][q] = rowk[q];
                        }
                }
                const cpx<T> pinv = zero ? cmk((T)0, (T)0) : crcp(prow[j]);
#pragma unroll
                for (int i = 0; i < R; ++i) {
                    const int row = kc + tid + i * PANEL_THREADS;
                    if (row > col && row < N) {
                        const cpx<T> l = cmul(a[i][j], pinv);
                        a[i][j] = l;
#pragma unroll
                        for (int q = j + 1; q < W; ++q) a[i][q] = cfms(a[i][q], l, prow[q]);
                    }
                }
                __syncthreads();
            }
        }
        // write the factored sub-panel back
#pragma unroll
        for (int i = 0; i < R; ++i) {
            const int row = kc + tid + i * PANEL_THREADS;
            if (row < N) {
#pragma unroll
                for (int q = 0; q < W; ++q)
                    if (q < w) A[(int64_t)row * N + kc + q] = a[i][q];
            }
        }
        // this sub-panel's swaps on the other columns of the outer panel
        if (tid < nb) {
            const int c = k0 + tid;
            if (c < kc || c >= kc + w) {
                for (int jj = 0; jj < w; ++jj) {
                    const int r1 = kc + jj, r2 = s_piv[s + jj];
                    if (r1 != r2) {
                        cpx<T> t1 = A[(int64_t)r1 * N + c];
                        cpx<T> t2 = A[(int64_t)r2 * N + c];
                        A[(int64_t)r1 * N + c] = t2;
                        A[(int64_t)r2 * N + c] = t1;
                    }
                }
            }
        }
        const int ncols = nb - s - w;
        if (ncols > 0) {
            if (tid < w) {
#pragma unroll
                for (int q = 0; q < W; ++q) L11s[tid][q] = a[0][q];
            }
            __syncthreads();
            // U block rows kc..kc+w-1, columns kc+w .. k0+nb-1: unit-lower solve
            if (tid < ncols) {
                const int c = kc + w + tid;
                for (int rr = 0; rr < w; ++rr) {
                    cpx<T> v = A[(int64_t)(kc + rr) * N + c];
                    for (int q = 0; q < rr; ++q) v = cfms(v, L11s[rr][q], Ublk[q][tid]);
                    Ublk[rr][tid] = v;
                    A[(int64_t)(kc + rr) * N + c] = v;
                }
            }
            __syncthreads();
            // rows below the sub-panel, columns kc+w .. k0+nb-1
#pragma unroll
            for (int i = 0; i < R; ++i) {
                const int row = kc + tid + i * PANEL_THREADS;
                if (row >= kc + w && row < N) {
                    cpx<T>* Arow = A + (int64_t)row * N + kc + w;
                    for (int c = 0; c < ncols; ++c) {
                        cpx<T> v = Arow[c];
#pragma unroll
                        for (int q = 0; q < W; ++q)
                            if (q < w) v = cfms(v, a[i][q], Ublk[q][c]);
                        Arow[c] = v;
                    }
                }
            }
        }
        __syncthreads();
    }
    if (tid < nb) piv[piv_off[b] + k0 + tid] = s_piv[tid];
    if (tid == 0 && s_sing) atomicOr(status, 1);
    __syncthreads();

    // inverses of the diagonal blocks: thread c < nb owns column c of Linv,
    // thread NB + c owns column c of Uinv.  Values are written to the linv
    // block and re-read by the same thread only.
    cpx<T>* Lb = linv + linv_off[b] + (int64_t)(k0 / NB) * NB * NB;
    const cpx<T>* D = A + (int64_t)k0 * N + k0;
    if (tid < nb) {
        const int c = tid;
        for (int r = c + 1; r < nb; ++r) {
            // x_c = 1 implicitly
            cpx<T> v = csub(cmk((T)0, (T)0), D[(int64_t)r * N + c]);
            for (int q = c + 1; q < r; ++q) v = cfms(v, D[(int64_t)r * N + q], Lb[q * NB + c]);
            Lb[r * NB + c] = v;
        }
    } else if (tid >= NB && tid < NB + nb) {
        const int c = tid - NB;
        // Uinv column c: x_c = 1/U_cc, x_r = -(sum_{q=r+1}^{c} U_rq x_q)/U_rr, r < c
        Lb[c * NB + c] = crcp(D[(int64_t)c * N + c]);
        for (int r = c - 1; r >= 0; --r) {
            cpx<T> v = cmk((T)0, (T)0);
            for (int q = r + 1; q <= c; ++q) v = cfms(v, D[(int64_t)r * N + q], Lb[q * NB + c]);
            Lb[r * NB + c] = cmul(v, crcp(D[(int64_t)r * N + r]));
        }
    }
}

// Row swaps of panel k0 on columns [k0+nb, N): one thread per column, swaps in
// order (grid.y blocks of 256 columns).
template <typename T>
__global__ __launch_bounds__(256) void k_lu_swap(int k0, const int* __restrict__ Ns,
                                                 const int64_t* __restrict__ a_off,
                                                 const int64_t* __restrict__ piv_off,
                                                 cpx<T>* __restrict__ Abase, const int* __restrict__ piv) {
    const int b = blockIdx.x;
    const int N = Ns[b];
    if (k0 >= N) return;
    const int nb = min(NB, N - k0);
    const int c = k0 + nb + blockIdx.y * 256 + threadIdx.x;
    __shared__ int sp[NB];
    if (threadIdx.x < nb) sp[threadIdx.x] = piv[piv_off[b] + k0 + threadIdx.x];
    __syncthreads();
    if (c >= N) return;
    cpx<T>* A = Abase + a_off[b];
    for (int jj = 0; jj < nb; ++jj) {
        const int r1 = k0 + jj, r2 = sp[jj];
        if (r1 != r2) {
            cpx<T> t1 = A[(int64_t)r1 * N + c];
            cpx<T> t2 = A[(int64_t)r2 * N + c];
            A[(int64_t)r1 * N + c] = t2;
            A[(int64_t)r2 * N + c] = t1;
        }
    }
}

// ---------------------------------------------------------------------------
// Tiled complex GEMM on MFMA for the trailing update.
//   TRSM mode: C(64 x 64 tile of rows k0..k0+nb, cols k0+nb+64*tc) = Linv * C
//   SUB  mode: C(rows k0+nb+64*tr, cols k0+nb+64*tc) -= L21 * U12
// 4 waves; wave (wm, wn) owns a 32x32 quarter = 2x2 MFMA 16x16 blocks.
// ---------------------------------------------------------------------------
#define GT 64
#define GK 16
#define GPAD 1

template <typename T>
struct mfma_traits;
template <>
struct mfma_traits<double> {
    typedef v4d acc_t;
    static __device__ __forceinline__ acc_t mac(double a, double b, acc_t c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
};
template <>
struct mfma_traits<float> {
    typedef v4f acc_t;
    static __device__ __forceinline__ acc_t mac(float a, float b, acc_t c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
};

__device__ __forceinline__ int find_prefix(const int* __restrict__ prefix, int n, int blk) {
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (prefix[mid] <= blk) lo = mid; else hi = mid - 1;
    }
    return lo;
}

template <typename T, bool SUB>
__global__ __launch_bounds__(256) void k_lu_gemm(int k0, const int* __restrict__ prefix, int batch,
                                                 const int* __restrict__ Ns, const int64_t* __restrict__ a_off,
                                                 const int64_t* __restrict__ linv_off, cpx<T>* __restrict__ Abase,
                                                 const cpx<T>* __restrict__ linv) {
    typedef typename mfma_traits<T>::acc_t acc_t;
    const int b = find_prefix(prefix, batch, blockIdx.x);
    const int tile = blockIdx.x - prefix[b];
    const int N = Ns[b];
    const int nb = min(NB, N - k0);
    const int rest = N - k0 - nb;
    const int tcols = (rest + GT - 1) / GT;
    int tr, tc;
    if (SUB) { tr = tile / tcols; tc = tile - tr * tcols; } else { tr = 0; tc = tile; }
    cpx<T>* A = Abase + a_off[b];
    const int col0 = k0 + nb + tc * GT;
    const int row0 = SUB ? (k0 + nb + tr * GT) : k0;
    const int nrows = SUB ? min(GT, N - row0) : nb;
    const int ncols = min(GT, N - col0);
    // A operand: SUB -> A[row0 + i][k0 + k] (ld N); TRSM -> Linv[i][k] (ld NB)
    const cpx<T>* Aop = SUB ? (A + (int64_t)row0 * N + k0)
                            : (linv + linv_off[b] + (int64_t)(k0 / NB) * NB * NB);
    const int lda = SUB ? N : NB;
    const cpx<T>* Bop = A + (int64_t)k0 * N + col0;   // rows k0.. (U12 / A12), ld N

    __shared__ cpx<T> As[GK][GT + GPAD];
    __shared__ cpx<T> Bs[GK][GT];

    const int tid = threadIdx.x;
    const int lane = tid & 63, wid = tid >> 6;
    const int wm = wid >> 1, wn = wid & 1;
    acc_t accr[2][2], acci[2][2];
#pragma unroll
    for (int mi = 0; mi < 2; ++mi)
#pragma unroll
        for (int ni = 0; ni < 2; ++ni) {
            accr[mi][ni] = (acc_t)(0);
            acci[mi][ni] = (acc_t)(0);
        }

    for (int kb = 0; kb < nb; kb += GK) {
        // A chunk: 64 rows x 16 k; thread -> (row = tid/16 + 16*pass, k = tid%16)
#pragma unroll
        for (int pass = 0; pass < 4; ++pass) {
            const int i = (tid >> 4) + 16 * pass;
            const int k = tid & 15;
            const bool ok = (i < nrows) && (kb + k < nb);
            // TRSM: Linv is lower-unit + upper(Uinv) packed; use only the unit-lower part
            cpx<T> v = cmk((T)0, (T)0);
            if (ok) {
                if (SUB) {
                    v = Aop[(int64_t)i * lda + kb + k];
                } else {
                    const int kk = kb + k;
                    if (kk < i) v = Aop[i * lda + kk];
                    else if (kk == i) v = cmk((T)1, (T)0);
                }
            }
            As[k][i] = v;
        }
        // B chunk: 16 k x 64 cols; thread -> (k = tid/64 + 4*pass, col = tid%64)
#pragma unroll
        for (int pass = 0; pass < 4; ++pass) {
            const int k = (tid >> 6) + 4 * pass;
            const int j = tid & 63;
            const bool ok = (kb + k < nb) && (j < ncols);
            Bs[k][j] = ok ? Bop[(int64_t)(kb + k) * N + j] : cmk((T)0, (T)0);
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < GK; kk += 4) {
            const int kr = kk + (lane >> 4);
            cpx<T> af[2], bf[2];
#pragma unroll
            for (int mi = 0; mi < 2; ++mi) af[mi] = As[kr][wm * 32 + mi * 16 + (lane & 15)];
#pragma unroll
            for (int ni = 0; ni < 2; ++ni) bf[ni] = Bs[kr][wn * 32 + ni * 16 + (lane & 15)];
#pragma unroll
            for (int mi = 0; mi < 2; ++mi) {
                const T nai = -af[mi].im;
#pragma unroll
                for (int ni = 0; ni < 2; ++ni) {
                    accr[mi][ni] = mfma_traits<T>::mac(af[mi].re, bf[ni].re, accr[mi][ni]);
                    accr[mi][ni] = mfma_traits<T>::mac(nai, bf[ni].im, accr[mi][ni]);
                    acci[mi][ni] = mfma_traits<T>::mac(af[mi].re, bf[ni].im, acci[mi][ni]);
                    acci[mi][ni] = mfma_traits<T>::mac(af[mi].im, bf[ni].re, acci[mi][ni]);
                }
            }
        }
        __syncthreads();
    }
    // epilogue: lane holds D[4*(lane/16) + v][lane%16] of each 16x16 block
    cpx<T>* C = A + (int64_t)row0 * N + col0;
#pragma unroll
    for (int mi = 0; mi < 2; ++mi)
#pragma unroll
        for (int ni = 0; ni < 2; ++ni)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int i = wm * 32 + mi * 16 + 4 * (lane >> 4) + v;
                const int j = wn * 32 + ni * 16 + (lane & 15);
                if (i < nrows && j < ncols) {
                    cpx<T>* p = C + (int64_t)i * N + j;
                    if (SUB) {
                        cpx<T> o = *p;
                        *p = cmk(o.re - accr[mi][ni][v], o.im - acci[mi][ni][v]);
                    } else {
                        *p = cmk(accr[mi][ni][v], acci[mi][ni][v]);
                    }
                }
            }
}

// ---------------------------------------------------------------------------
// Host side: schedule and launches
// ---------------------------------------------------------------------------
void lu_build_schedule(const int32_t* N, int32_t batch, fhw_lu_sched& sch) {
    int32_t maxN = 0;
    for (int q = 0; q < batch; ++q) maxN = std::max(maxN, N[q]);
    sch.nsteps = (maxN + NB - 1) / NB;
    sch.R.clear(); sch.W.clear(); sch.gemm_trsm_off.clear(); sch.gemm_upd_off.clear();
    sch.gemm_trsm_tiles.clear(); sch.gemm_upd_tiles.clear(); sch.swap_blocks.clear(); sch.prefix.clear();
    for (int p = 0; p < sch.nsteps; ++p) {
        const int k0 = p * NB;
        int rows = 0;
        for (int q = 0; q < batch; ++q) rows = std::max(rows, N[q] - k0);
        int R = (rows + PANEL_THREADS - 1) / PANEL_THREADS;
        R = R <= 1 ? 1 : (R <= 2 ? 2 : 4);
        sch.R.push_back(R);
        sch.W.push_back(R == 1 ? 16 : (R == 2 ? 8 : 4));
        int maxrest = 0;
        // TRSM prefix
        sch.gemm_trsm_off.push_back((int64_t)sch.prefix.size());
        int acc = 0;
        for (int q = 0; q < batch; ++q) {
            sch.prefix.push_back(acc);
            int rest = N[q] - k0 - NB;
            if (rest > 0) { acc += (rest + GT - 1) / GT; maxrest = std::max(maxrest, rest); }
        }
        sch.prefix.push_back(acc);
        sch.gemm_trsm_tiles.push_back(acc);
        // update prefix
        sch.gemm_upd_off.push_back((int64_t)sch.prefix.size());
        acc = 0;
        for (int q = 0; q < batch; ++q) {
            sch.prefix.push_back(acc);
            int rest = N[q] - k0 - NB;
            if (rest > 0) { int t = (rest + GT - 1) / GT; acc += t * t; }
        }
        sch.prefix.push_back(acc);
        sch.gemm_upd_tiles.push_back(acc);
        sch.swap_blocks.push_back(maxrest > 0 ? (maxrest + 255) / 256 : 0);
    }
}

template <typename T>
static hipError_t lu_factor_t(hipStream_t s, const fhw_batch_dev& bd, const fhw_lu_sched& sch,
                              const int32_t* d_prefix, cpx<T>* A, int32_t* piv, cpx<T>* linv, int32_t* st,
                              fhw_prof* prof) {
    for (int p = 0; p < sch.nsteps; ++p) {
        const int k0 = p * NB;
        const int R = sch.R[p];
        prof_begin(prof, FHW_STAGE_LU_PANEL, s);
        if (R == 1)
            hipLaunchKernelGGL((k_lu_panel<T, 1, 16>), dim3(bd.batch), dim3(PANEL_THREADS), 0, s, k0, bd.N,
                               bd.a_off, bd.piv_off, bd.linv_off, A, piv, linv, st);
        else if (R == 2)
            hipLaunchKernelGGL((k_lu_panel<T, 2, 8>), dim3(bd.batch), dim3(PANEL_THREADS), 0, s, k0, bd.N,
                               bd.a_off, bd.piv_off, bd.linv_off, A, piv, linv, st);
        else
            hipLaunchKernelGGL((k_lu_panel<T, 4, 4>), dim3(bd.batch), dim3(PANEL_THREADS), 0, s, k0, bd.N,
                               bd.a_off, bd.piv_off, bd.linv_off, A, piv, linv, st);
        prof_end(prof, s);
        if (sch.swap_blocks[p] > 0) {
            prof_begin(prof, FHW_STAGE_LU_SWAP, s);
            hipLaunchKernelGGL((k_lu_swap<T>), dim3(bd.batch, sch.swap_blocks[p]), dim3(256), 0, s, k0, bd.N,
                               bd.a_off, bd.piv_off, A, piv);
            prof_end(prof, s);
        }
        if (sch.gemm_trsm_tiles[p] > 0) {
            prof_begin(prof, FHW_STAGE_LU_TRSM, s);
            hipLaunchKernelGGL((k_lu_gemm<T, false>), dim3(sch.gemm_trsm_tiles[p]), dim3(256), 0, s, k0,
                               d_prefix + sch.gemm_trsm_off[p], bd.batch, bd.N, bd.a_off, bd.linv_off, A,
                               (const cpx<T>*)linv);
            prof_end(prof, s);
        }
        if (sch.gemm_upd_tiles[p] > 0) {
            prof_begin(prof, FHW_STAGE_LU_UPDATE, s);
            hipLaunchKernelGGL((k_lu_gemm<T, true>), dim3(sch.gemm_upd_tiles[p]), dim3(256), 0, s, k0,
                               d_prefix + sch.gemm_upd_off[p], bd.batch, bd.N, bd.a_off, bd.linv_off, A,
                               (const cpx<T>*)linv);
            prof_end(prof, s);
        }
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_lu_factor(hipStream_t s, const fhw_batch_dev& b, const fhw_lu_sched& sch,
                            const int32_t* d_prefix, void* A, int32_t* piv, void* linv, int32_t* d_status,
                            int precision, fhw_prof* prof) {
    if (precision == FHW_FP64)
        return lu_factor_t<double>(s, b, sch, d_prefix, (zd*)A, piv, (zd*)linv, d_status, prof);
    return lu_factor_t<float>(s, b, sch, d_prefix, (zf*)A, piv, (zf*)linv, d_status, prof);
}
