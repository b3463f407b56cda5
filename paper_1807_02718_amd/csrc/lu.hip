// Batched dense complex LU with partial pivoting on gfx950 (step F3: one
// Nystrom system per frequency), FP64 or FP32, ragged batches of
// column-major packed matrices (element (r, c) of matrix b at a_off[b] + c N + r).
//
// Right-looking, blocked by NB = 64 columns, panels in pairs (the schedule
// at lu_build_schedule).  Per panel k0:
//   k_lu_panel    one 256-thread workgroup per matrix (two to four per CU) factors
//                 the (N-k0) x 64 panel in sub-panels of W columns held in
//                 registers, rows owned by threads (coalesced in column-major),
//                 left-looking across sub-panels so each is read and written once.
//   k_lu_diaginv  inverses of the 64x64 unit-lower and upper diagonal blocks
//                 (used by the trailing TRSM and by the solves), in LDS.
//   k_lu_swap     the panel's row swaps on a column range (no work when the
//                 panel did not pivot, the usual case for these systems).
//   k_lu_gemm     U12 = L11^{-1} A12 (in place) and A22 -= L21 U12 on 64x64
//                 tiles with depth 64 or 128, the complex product as 3 real
//                 MFMA 16x16x4 products (Gauss's 3M form).
// A panel's L columns carry the pivots of its pair partner but not those of
// later pairs; the solves replay the pivots pair by pair.
#include <algorithm>

#include "fhw_device.h"
#include "fhw_internal.h"
#include "gemm_table.h"
#include "panel_table.h"

#define NB FHW_LU_NB
#define PANEL_THREADS 256
#define INV_THREADS 1024

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

// linv block layout per matrix: panel p at linv_off + p*NB*NB, column-major
// 64x64 (entry (r, c) at c*NB + r): strictly lower part = inverse of the
// unit-lower L11, upper part including the diagonal = inverse of U11.

template <typename T>
__device__ __forceinline__ bool piv_better(T v, int i, T bv, int bi) {
    return (v > bv) || (v == bv && i < bi);
}

// Panel factorization, left-looking over sub-panels of W columns.  Thread
// tid owns rows k0 + tid + i*PT of the panel.  Each sub-panel is read once,
// brought up to date with the factored sub-panels t < s one after the other
// (U_t = L_tt^{-1} X_t on its W diagonal rows, then X -= L_t U_t on the rows
// below, L_t streamed from memory), factored in registers (pivot search by
// wave shuffles and one LDS round, max |re|+|im|, first index on ties) and
// written back once: the panel's columns are never rewritten between
// sub-panels.  R rows per thread and W columns per sub-panel set the register
// budget, WPE the waves per SIMD.
// Column q of L_t for the thread's rows (zero for rows at or above lo).
template <typename T, int R, int PT>
__device__ __forceinline__ void lazy_load(cpx<T> (&l)[R], const cpx<T>* Lq, int tid, int lo, int m) {
#pragma unroll
    for (int i = 0; i < R; ++i) {
        const int rho = tid + i * PT;
        l[i] = (rho >= lo && rho < m) ? Lq[i * PT] : cmk((T)0, (T)0);
    }
}

// Rows at or below lo: x(row, :) -= l(row) * u(:).  l is zero outside rows
// [lo, m) (lazy_load), so every row takes the update unguarded: rows above
// lo (final U rows, or rows about to be replaced by U_t) and rows past m
// (never written back) are left as they are, up to the sign of a zero.  A
// guard per row would cost a select per updated value (the compiler
// if-converts it), half again the four FMAs of the complex update.
template <typename T, int R, int W>
__device__ __forceinline__ void lazy_update(T (&ar)[R][W], T (&ai)[R][W], const cpx<T> (&l)[R], const cpx<T>* u) {
#pragma unroll
    for (int c = 0; c < W; ++c) {
        const cpx<T> uc = u[c];
#pragma unroll
        for (int i = 0; i < R; ++i) {
            ar[i][c] = ar[i][c] - l[i].re * uc.re + l[i].im * uc.im;
            ai[i][c] = ai[i][c] - l[i].re * uc.im - l[i].im * uc.re;
        }
    }
}

template <typename T, int W, int PT>
struct panel_lds {
    cpx<T> X[W][W];             // rows t*W .. t*W+W-1 of the sub-panel (lazy step t)
    cpx<T> U[2][W][W];          // U_t, double-buffered across lazy steps
    cpx<T> Lkeep[NB / W][W][W]; // unit-lower diagonal blocks of the factored sub-panels
    cpx<T> prow[W];
    cpx<T> rowk[W];
    T redv[PT / 64];
    int redi[PT / 64];
    int s_piv[NB];
    int sing;
};

// PD: columns of L_t in flight during a lazy step (a rolling register
// buffer: column q + PD is requested as soon as column q has been applied);
// 0 selects the default (all W for FP32 with one row per thread, one column
// ahead for FP32 otherwise, none for FP64).
template <typename T, int R, int W, int WPE, int PT = PANEL_THREADS, int PD = 0>
__global__ __launch_bounds__(PT, WPE) void k_lu_panel(int k0, const int* __restrict__ Ns,
                                                      const int64_t* __restrict__ a_off,
                                                      const int64_t* __restrict__ piv_off,
                                                      cpx<T>* __restrict__ Abase, int* __restrict__ piv,
                                                      int* __restrict__ status, const int32_t* __restrict__ ids) {
    static_assert(NB % W == 0, "sub-panels tile the panel");
    __shared__ panel_lds<T, W, PT> S;
    const int b = ids ? ids[blockIdx.x] : (int)blockIdx.x;
    const int N = Ns[b];
    if (k0 >= N) return;
    const int m = N - k0;
    const int nb = min(NB, m);
    // P[c*N + r]: entry (k0 + r, k0 + c) of the matrix
    cpx<T>* P = Abase + a_off[b] + (int64_t)k0 * N + k0;
    const int tid = threadIdx.x;
    const int lane = tid & 63, wid = tid >> 6;
    const bool wave_live = __builtin_amdgcn_readfirstlane(wid) * 64 < m;   // row tid + i PT >= wid 64
    if (tid == 0) S.sing = 0;

    T ar[R][W], ai[R][W];
    for (int s = 0; s < nb; s += W) {
        const int w = min(W, nb - s);
        const int kc = k0 + s;
#pragma unroll
        for (int i = 0; i < R; ++i) {
            const int rho = tid + i * PT;
#pragma unroll
            for (int q = 0; q < W; ++q) {
                T vr = (T)0, vi = (T)0;
                if (rho < m && q < w) {
                    const cpx<T> v = P[(int64_t)(s + q) * N + rho];
                    vr = v.re;
                    vi = v.im;
                }
                ar[i][q] = vr;
                ai[i][q] = vi;
            }
        }
        // lazy updates by the factored sub-panels (all of full width W)
        for (int t = 0; t < s / W; ++t) {
            const int tb = t * W;
            const int buf = t & 1;
            // rows below block t: X -= L_t U_t.  L_t is final, so its loads go
            // out before U_t is formed: by default FP32 with one row per
            // thread all W columns, else FP32 one column ahead of the
            // arithmetic and FP64 the first column only (register budgets,
            // measured); PD > 0: PD columns in flight, in a rolling buffer
            const cpx<T>* Lt = P + (int64_t)tb * N + tid;
            constexpr bool F32 = sizeof(T) == 4;
            constexpr int PF = PD > 0 ? (PD < W ? PD : W) : ((F32 && R == 1) ? W : 1);
            cpx<T> l[PF][R];
#pragma unroll
            for (int q = 0; q < PF; ++q) lazy_load<T, R, PT>(l[q], Lt + (int64_t)q * N, tid, tb + W, m);
            if (wid == 0) {
                // rows tb .. tb+W-1 are rows i = 0 of lanes tb .. tb+W-1
                if (lane >= tb && lane < tb + W) {
#pragma unroll
                    for (int q = 0; q < W; ++q) S.X[lane - tb][q] = cmk(ar[0][q], ai[0][q]);
                }
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                if (lane < W) {
                    // column lane of U_t = L_tt^{-1} X_t (unit lower, forward substitution)
                    cpx<T> x[W];
#pragma unroll
                    for (int rr = 0; rr < W; ++rr) x[rr] = S.X[rr][lane];
#pragma unroll
                    for (int rr = 1; rr < W; ++rr) {
#pragma unroll
                        for (int q = 0; q < rr; ++q) x[rr] = cfms(x[rr], S.Lkeep[t][rr][q], x[q]);
                    }
#pragma unroll
                    for (int rr = 0; rr < W; ++rr) S.U[buf][rr][lane] = x[rr];
                }
            }
            __syncthreads();
            // a wave whose rows all lie past the panel's end skips the update
            // (a wave-uniform branch, no barrier inside)
            if (!wave_live) {
            } else if constexpr (PF == W) {
#pragma unroll
                for (int q = 0; q < W; ++q) lazy_update<T, R, W>(ar, ai, l[q], S.U[buf][q]);
            } else if constexpr (PD > 0) {
                // column q0 + k from slot k, which then takes column q0 + k + PF
#pragma unroll 1
                for (int q0 = 0; q0 < W; q0 += PF) {
#pragma unroll
                    for (int k = 0; k < PF; ++k) {
                        lazy_update<T, R, W>(ar, ai, l[k], S.U[buf][q0 + k]);
                        if (q0 + k + PF < W)
                            lazy_load<T, R, PT>(l[k], Lt + (int64_t)(q0 + k + PF) * N, tid, tb + W, m);
                    }
                }
            } else {
#pragma unroll 1
                for (int q = 0; q < W; ++q) {
                    if constexpr (F32) {
                        // column q + 1 (no rows, so zeros and no loads, after the last)
                        cpx<T> ln[R];
                        lazy_load<T, R, PT>(ln, Lt + (int64_t)(q + 1) * N, tid, q + 1 < W ? tb + W : m, m);
                        lazy_update<T, R, W>(ar, ai, l[0], S.U[buf][q]);
#pragma unroll
                        for (int i = 0; i < R; ++i) l[0][i] = ln[i];
                    } else {
                        if (q > 0) lazy_load<T, R, PT>(l[0], Lt + (int64_t)q * N, tid, tb + W, m);
                        lazy_update<T, R, W>(ar, ai, l[0], S.U[buf][q]);
                    }
                }
            }
            if (tid >= tb && tid < tb + W) {
#pragma unroll
                for (int c = 0; c < W; ++c) {
                    const cpx<T> u = S.U[buf][tid - tb][c];
                    ar[0][c] = u.re;
                    ai[0][c] = u.im;
                }
            }
        }
        // factor the sub-panel: rows kc .. N-1 of its columns
#pragma clang loop unroll(full)
        for (int j = 0; j < W; ++j) {
            if (j < w) {
                const int col = kc + j;
                T bv = (T)-1;
                int bi = 0x7fffffff;
#pragma unroll
                for (int i = 0; i < R; ++i) {
                    const int row = k0 + tid + i * PT;
                    if (row >= col && row < N) {
                        const T v = fabs(ar[i][j]) + fabs(ai[i][j]);
                        if (piv_better(v, row, bv, bi)) { bv = v; bi = row; }
                    }
                }
#pragma unroll
                for (int off = 32; off >= 1; off >>= 1) {
                    T ov = __shfl_xor(bv, off, 64);
                    int oi = __shfl_xor(bi, off, 64);
                    if (piv_better(ov, oi, bv, bi)) { bv = ov; bi = oi; }
                }
                if (lane == 0) { S.redv[wid] = bv; S.redi[wid] = bi; }
                __syncthreads();
                bv = S.redv[0]; bi = S.redi[0];
#pragma unroll
                for (int q = 1; q < PT / 64; ++q)
                    if (piv_better(S.redv[q], S.redi[q], bv, bi)) { bv = S.redv[q]; bi = S.redi[q]; }
                // no candidate (NaN column) or zero column: keep the row, flag it
                const bool zp = !(bv > (T)0) || bi >= N;
                const int p = (bi >= N) ? col : bi;
                const int tp = (p - k0) % PT, ip = (p - k0) / PT;
                const int tc = (col - k0) % PT, ic = (col - k0) / PT;
#pragma unroll
                for (int i = 0; i < R; ++i) {
                    if (tid == tp && i == ip) {
#pragma unroll
                        for (int q = 0; q < W; ++q) S.prow[q] = cmk(ar[i][q], ai[i][q]);
                    }
                    if (tid == tc && i == ic) {
#pragma unroll
                        for (int q = 0; q < W; ++q) S.rowk[q] = cmk(ar[i][q], ai[i][q]);
                    }
                }
                if (tid == 0) {
                    S.s_piv[s + j] = p;
                    if (zp) S.sing = 1;
                }
                __syncthreads();
#pragma unroll
                for (int i = 0; i < R; ++i) {
                    if (tid == tc && i == ic) {
#pragma unroll
                        for (int q = 0; q < W; ++q) { ar[i][q] = S.prow[q].re; ai[i][q] = S.prow[q].im; }
                    }
                    if (tid == tp && p != col && i == ip) {
#pragma unroll
                        for (int q = 0; q < W; ++q) { ar[i][q] = S.rowk[q].re; ai[i][q] = S.rowk[q].im; }
                    }
                }
                const cpx<T> pinv = zp ? cmk((T)0, (T)0) : crcp(S.prow[j]);
#pragma unroll
                for (int i = 0; i < R; ++i) {
                    const int row = k0 + tid + i * PT;
                    if (row > col && row < N) {
                        const T lr = ar[i][j] * pinv.re - ai[i][j] * pinv.im;
                        const T li = ar[i][j] * pinv.im + ai[i][j] * pinv.re;
                        ar[i][j] = lr;
                        ai[i][j] = li;
#pragma unroll
                        for (int q = j + 1; q < W; ++q) {
                            const cpx<T> u = S.prow[q];
                            ar[i][q] = ar[i][q] - lr * u.re + li * u.im;
                            ai[i][q] = ai[i][q] - lr * u.im - li * u.re;
                        }
                    }
                }
            }
        }
        // the sub-panel back (its U rows above and its factored rows), and its
        // unit-lower diagonal block kept for the later sub-panels
#pragma unroll
        for (int i = 0; i < R; ++i) {
            const int rho = tid + i * PT;
            if (rho < m) {
#pragma unroll
                for (int q = 0; q < W; ++q)
                    if (q < w) P[(int64_t)(s + q) * N + rho] = cmk(ar[i][q], ai[i][q]);
            }
        }
        if (s + w < nb && tid >= s && tid < s + W) {
#pragma unroll
            for (int q = 0; q < W; ++q) S.Lkeep[s / W][tid - s][q] = cmk(ar[0][q], ai[0][q]);
        }
        // this sub-panel's swaps, in order, on the other columns of the panel
        if (tid < nb && (tid < s || tid >= s + w)) {
            cpx<T>* Pc = P + (int64_t)tid * N - k0;   // indexed by absolute row
            for (int jj = 0; jj < w; ++jj) {
                const int r1 = kc + jj, r2 = S.s_piv[s + jj];
                if (r1 != r2) {
                    const cpx<T> t1 = Pc[r1];
                    Pc[r1] = Pc[r2];
                    Pc[r2] = t1;
                }
            }
        }
        __syncthreads();
    }
    if (tid < nb) piv[piv_off[b] + k0 + tid] = S.s_piv[tid];
    if (tid == 0 && S.sing) atomicOr(status, 1);
}

// Inverses of the unit-lower and upper parts of the factored diagonal block
// of panel k0 (one 1024-thread workgroup per matrix, block in LDS), blocked:
// the four 16x16 diagonal blocks by substitution (16 lanes per column, a
// 16-lane reduction per step), then 32x32 and 64x64 inverses from
//   inv([A 0; C B]) = [inv A, 0; -inv B C inv A, inv B]   (unit lower)
//   inv([A B; 0 D]) = [inv A, -inv A B inv D; 0, inv D]   (upper)
// with two triangular products per level, one output entry per thread.
// I holds the result: strict lower = inverse of the unit-lower part,
// upper with the diagonal = inverse of the upper part.
template <typename T>
struct inv_lds {
    cpx<T> D[NB][NB + 1];
    cpx<T> I[NB][NB + 1];
    cpx<T> Tm[NB / 2][NB / 2 + 1];
    cpx<T> rd[NB];   // reciprocals of the diagonal of U
};

template <typename T>
__global__ __launch_bounds__(INV_THREADS) void k_lu_diaginv(int k0, const int* __restrict__ Ns,
                                                           const int64_t* __restrict__ a_off,
                                                           const int64_t* __restrict__ linv_off,
                                                           const cpx<T>* __restrict__ Abase,
                                                           cpx<T>* __restrict__ linv) {
    extern __shared__ __align__(16) char smem_raw[];
    inv_lds<T>& S = *reinterpret_cast<inv_lds<T>*>(smem_raw);
    const int b = blockIdx.x;
    const int N = Ns[b];
    if (k0 >= N) return;
    const int nb = min(NB, N - k0);
    const cpx<T>* Db = Abase + a_off[b] + (int64_t)k0 * N + k0;
    const int tid = threadIdx.x;
    const cpx<T> zero = cmk((T)0, (T)0), one = cmk((T)1, (T)0);
    // the block, padded to 64 with the identity (whose inverse parts are the identity)
    for (int e = tid; e < NB * NB; e += INV_THREADS) {
        const int c = e / NB, r = e - c * NB;
        S.D[r][c] = (r < nb && c < nb) ? Db[(int64_t)c * N + r] : ((r == c) ? one : zero);
    }
    __syncthreads();
    if (tid < NB) S.rd[tid] = crcp(S.D[tid][tid]);
    __syncthreads();
    // ---- level 0: 16x16 diagonal blocks; thread = (block bb, column c, lane t)
    {
        const int bb = tid >> 8, c = (tid >> 4) & 15, t = tid & 15;
        const int o = 16 * bb;
        // unit lower: x_c = 1, x_r = -sum_{q=c}^{r-1} L_rq x_q
        cpx<T> x = (t == c) ? one : zero;
        for (int r = c + 1; r < 16; ++r) {
            cpx<T> acc = (t >= c && t < r) ? cmul(S.D[o + r][o + t], x) : zero;
#pragma unroll
            for (int off = 1; off < 16; off <<= 1) {
                acc.re += __shfl_xor(acc.re, off, 64);
                acc.im += __shfl_xor(acc.im, off, 64);
            }
            if (t == r) x = cmk(-acc.re, -acc.im);
        }
        if (t > c) S.I[o + t][o + c] = x;
        // upper: x_c = 1/U_cc, x_r = -(sum_{q=r+1}^{c} U_rq x_q) / U_rr, r < c
        x = (t == c) ? S.rd[o + c] : zero;
        for (int r = c - 1; r >= 0; --r) {
            cpx<T> acc = (t > r && t <= c) ? cmul(S.D[o + r][o + t], x) : zero;
#pragma unroll
            for (int off = 1; off < 16; off <<= 1) {
                acc.re += __shfl_xor(acc.re, off, 64);
                acc.im += __shfl_xor(acc.im, off, 64);
            }
            if (t == r) x = cmul(cmk(-acc.re, -acc.im), S.rd[o + r]);
        }
        if (t <= c) S.I[o + t][o + c] = x;
    }
    __syncthreads();
    // ---- levels 1 (m = 16, two pairs) and 2 (m = 32, one pair)
    for (int m = 16; m < NB; m <<= 1) {
        const int pairs = NB / (2 * m);
        const int outs = m * m;                 // per pair
        const int active = pairs * outs;        // 512 or 1024 threads
        const int pr = tid / outs, e = tid - pr * outs;
        const int r = e % m, j = e / m;
        const int o = pr * 2 * m;               // pair origin: A at (o, o), B at (o+m, o+m)
        const int tr = pr * m + r;              // this pair's rows of Tm (pairs * m <= 32)
        // unit lower, step 1: Tm = C inv(A), C = L[o+m.., o..]; inv(A) unit lower
        if (tid < active) {
            cpx<T> acc = S.D[o + m + r][o + j];
            for (int q = j + 1; q < m; ++q) acc = cfma(acc, S.D[o + m + r][o + q], S.I[o + q][o + j]);
            S.Tm[tr][j] = acc;
        }
        __syncthreads();
        // step 2: X = -inv(B) Tm, inv(B) unit lower
        cpx<T> xv = zero;
        if (tid < active) {
            cpx<T> acc = S.Tm[tr][j];
            for (int q = 0; q < r; ++q) acc = cfma(acc, S.I[o + m + r][o + m + q], S.Tm[pr * m + q][j]);
            xv = cmk(-acc.re, -acc.im);
        }
        __syncthreads();
        if (tid < active) S.I[o + m + r][o + j] = xv;
        // upper, step 1: Tm = B inv(D), B = U[o.., o+m..]; inv(D) upper with diagonal
        if (tid < active) {
            cpx<T> acc = zero;
            for (int q = 0; q <= j; ++q) acc = cfma(acc, S.D[o + r][o + m + q], S.I[o + m + q][o + m + j]);
            S.Tm[tr][j] = acc;
        }
        __syncthreads();
        // step 2: X = -inv(A) Tm, inv(A) upper with diagonal
        if (tid < active) {
            cpx<T> acc = zero;
            for (int q = r; q < m; ++q) acc = cfma(acc, S.I[o + r][o + q], S.Tm[pr * m + q][j]);
            xv = cmk(-acc.re, -acc.im);
        }
        __syncthreads();
        if (tid < active) S.I[o + r][o + m + j] = xv;
        __syncthreads();
    }
    cpx<T>* Lb = linv + linv_off[b] + (int64_t)(k0 / NB) * NB * NB;
    for (int e = tid; e < NB * NB; e += INV_THREADS) {
        const int cc = e / NB, r = e - cc * NB;
        Lb[e] = S.I[r][cc];
    }
}

// Row swaps of panel k0 on the columns [cbeg, cbeg + ccount) (ccount = 0: up
// to N), one thread per column, swaps in order (grid.y blocks of 256
// columns).  Returns at once when no pivot of the panel moved.
template <typename T>
__global__ __launch_bounds__(256) void k_lu_swap(int k0, int cbeg, int ccount, const int* __restrict__ Ns,
                                                 const int64_t* __restrict__ a_off,
                                                 const int64_t* __restrict__ piv_off,
                                                 cpx<T>* __restrict__ Abase, const int* __restrict__ piv) {
    const int b = blockIdx.x;
    const int N = Ns[b];
    if (k0 >= N) return;
    const int nb = min(NB, N - k0);
    __shared__ int sp[NB];
    __shared__ int any;
    if (threadIdx.x == 0) any = 0;
    __syncthreads();
    if (threadIdx.x < nb) {
        sp[threadIdx.x] = piv[piv_off[b] + k0 + threadIdx.x];
        if (sp[threadIdx.x] != k0 + (int)threadIdx.x) any = 1;
    }
    __syncthreads();
    if (!any) return;
    const int cend = ccount > 0 ? min(N, cbeg + ccount) : N;
    const int c = cbeg + blockIdx.y * 256 + threadIdx.x;
    if (c >= cend) return;
    cpx<T>* Ac = Abase + a_off[b] + (int64_t)c * N;
    for (int jj = 0; jj < nb; ++jj) {
        const int r1 = k0 + jj, r2 = sp[jj];
        if (r1 != r2) {
            const cpx<T> t1 = Ac[r1];
            Ac[r1] = Ac[r2];
            Ac[r2] = t1;
        }
    }
}

// ---------------------------------------------------------------------------
// Tiled complex GEMM on MFMA for the trailing update (column-major).
//   TRSM mode: C(rows k0..k0+nb, cols k0+coff+64*tc ..) = Linv * C (in place)
//   SUB  mode: C(rows k0+roff+64*tr.., cols k0+coff+64*tc..) -= L U with
//              L = columns k0..k0+K-1 and U = rows k0..k0+K-1 of the matrix
//              (K = 64: one panel; K = 128: a pair of panels)
// The MFMA computes the transposed tile, D(j, i) = sum_k U(k, j) L(i, k), so
// that the 16 consecutive lanes of a result row are 16 consecutive matrix rows
// (coalesced column-major stores).  4 waves; wave (wj, wi) owns a 32x32
// quarter = 2x2 MFMA 16x16 blocks.
// ---------------------------------------------------------------------------
#define GT 64
#define GPAD 1

// K-chunk staged through LDS and workgroups per CU (the launch-bounds hint)
// per precision, from the project's autotuner (gemm_table.h)
template <typename T>
struct gemm_cfg;
template <>
struct gemm_cfg<float> {
    static constexpr int GK = FHW_GEMM_GK_F32, OCC = FHW_GEMM_OCC_F32;
};
template <>
struct gemm_cfg<double> {
    static constexpr int GK = FHW_GEMM_GK_F64, OCC = FHW_GEMM_OCC_F64;
};
template <typename T>
constexpr int gk_v = gemm_cfg<T>::GK;

template <typename T>
struct mfma_traits;
// Both take A[i][k] from lane i + 16k and B[k][j] from lane j + 16k.  The
// 16x16 result lands differently: element v of lane l is row 4v + l/16 for
// the f64 form and row 4(l/16) + v for the f32 form; column l % 16 in both.
template <>
struct mfma_traits<double> {
    typedef v4d acc_t;
    static __device__ __forceinline__ acc_t mac(double a, double b, acc_t c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int lane, int v) { return 4 * v + (lane >> 4); }
};
template <>
struct mfma_traits<float> {
    typedef v4f acc_t;
    static __device__ __forceinline__ acc_t mac(float a, float b, acc_t c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int lane, int v) { return 4 * (lane >> 4) + v; }
};

__device__ __forceinline__ int find_prefix(const int* __restrict__ prefix, int n, int blk) {
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (prefix[mid] <= blk) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// Workgroups are dispatched to the 8 XCDs round-robin (workgroup w runs on
// XCD w mod 8), and each XCD has its own L2.  Renumber so that XCD x takes
// one contiguous range of tiles: the tiles of a matrix then share one L2 and
// its L and U panels are fetched from HBM about once.
__device__ __forceinline__ int xcd_tile(int w, int G) {
    constexpr int NX = 8;
    const int per = G / NX, rem = G % NX;
    const int x = w % NX, i = w / NX;
    return (x < rem) ? x * (per + 1) + i : rem * (per + 1) + (x - rem) * per + i;
}

// Stage one GK-deep chunk (GK = gk_v<T>) of the L and U operands in registers
// (real and imaginary parts apart): L (k = tid/64 + 4p, i = tid%64), U (j =
// tid/GK + (256/GK) p, k = tid%GK), p < GK/4.
template <typename T>
struct gemm_stage {
    T lr[gk_v<T> / 4], li[gk_v<T> / 4], ur[gk_v<T> / 4], ui[gk_v<T> / 4];
};

template <typename T, bool SUB>
__device__ __forceinline__ void gemm_load_chunk(gemm_stage<T>& g, int kb, int tid, int nrows, int ncols, int nb,
                                                const cpx<T>* __restrict__ Lop, int ldl,
                                                const cpx<T>* __restrict__ Uop, int N) {
#pragma unroll
    for (int pass = 0; pass < gk_v<T> / 4; ++pass) {
        const int k = (tid >> 6) + 4 * pass;
        const int i = tid & 63;
        const int kk = kb + k;
        T vr = (T)0, vi = (T)0;
        if (i < nrows && kk < nb) {
            if (SUB) {
                const cpx<T> v = Lop[(int64_t)kk * ldl + i];
                vr = v.re;
                vi = v.im;
            } else {
                // unit-lower part of the packed inverse block
                if (kk < i) {
                    const cpx<T> v = Lop[kk * ldl + i];
                    vr = v.re;
                    vi = v.im;
                } else if (kk == i) {
                    vr = (T)1;
                }
            }
        }
        g.lr[pass] = vr;
        g.li[pass] = vi;
    }
#pragma unroll
    for (int pass = 0; pass < gk_v<T> / 4; ++pass) {
        const int j = tid / gk_v<T> + (256 / gk_v<T>) * pass;
        const int k = tid % gk_v<T>;
        T vr = (T)0, vi = (T)0;
        if ((kb + k < nb) && (j < ncols)) {
            const cpx<T> v = Uop[(int64_t)j * N + kb + k];
            vr = v.re;
            vi = v.im;
        }
        g.ur[pass] = vr;
        g.ui[pass] = vi;
    }
}

template <typename T, int NBUF>
__device__ __forceinline__ void gemm_store_chunk(cpx<T> (&Ls)[NBUF][gk_v<T>][GT + GPAD],
                                                 cpx<T> (&Us)[NBUF][gk_v<T>][GT + GPAD],
                                                 const gemm_stage<T>& g, int buf, int tid) {
#pragma unroll
    for (int pass = 0; pass < gk_v<T> / 4; ++pass)
        Ls[buf][(tid >> 6) + 4 * pass][tid & 63] = cmk(g.lr[pass], g.li[pass]);
#pragma unroll
    for (int pass = 0; pass < gk_v<T> / 4; ++pass)
        Us[buf][tid % gk_v<T>][tid / gk_v<T> + (256 / gk_v<T>) * pass] = cmk(g.ur[pass], g.ui[pass]);
}

// DBUF: double-buffered LDS chunks (next chunk's global loads in flight
// during the current chunk's MFMAs).  Measured on the 1024 x N=1024 batch,
// the single-buffered form is faster (higher occupancy): 96 vs 91 TFLOP/s in
// FP32, 53.5 vs 42.9 in FP64 on the largest trailing update.
template <typename T, bool SUB, bool DBUF = false>
__global__ __launch_bounds__(256, gemm_cfg<T>::OCC) void k_lu_gemm(int k0, int K, int roff, int rlim, int coff,
                                                 int clim, const int* __restrict__ prefix, int batch,
                                                 const int* __restrict__ Ns, const int64_t* __restrict__ a_off,
                                                 const int64_t* __restrict__ linv_off, cpx<T>* __restrict__ Abase,
                                                 const cpx<T>* __restrict__ linv) {
    typedef typename mfma_traits<T>::acc_t acc_t;
    const int blk = xcd_tile(blockIdx.x, gridDim.x);
    const int b = find_prefix(prefix, batch, blk);
    const int tile = blk - prefix[b];
    const int N = Ns[b];
    cpx<T>* A = Abase + a_off[b];
    int row0, col0, nrows, ncols, nb;
    const cpx<T>* Lop;
    int ldl;
    if (SUB) {
        const int rb = k0 + roff, cb = k0 + coff;
        const int re = rlim > 0 ? min(N, rb + rlim) : N;
        const int ce = clim > 0 ? min(N, cb + clim) : N;
        const int tcols = (ce - cb + GT - 1) / GT;
        const int tr = tile / tcols, tc = tile - tr * tcols;
        row0 = rb + tr * GT;
        col0 = cb + tc * GT;
        nrows = min(GT, re - row0);
        ncols = min(GT, ce - col0);
        nb = min(K, N - k0);
        Lop = A + (int64_t)k0 * N + row0;   // L (i, k) at (k0 + k) N + row0 + i
        ldl = N;
    } else {
        nb = min(NB, N - k0);
        row0 = k0;
        col0 = k0 + coff + tile * GT;
        nrows = nb;
        ncols = min(GT, N - col0);
        Lop = linv + linv_off[b] + (int64_t)(k0 / NB) * NB * NB;   // Linv column-major (i, k) at k NB + i
        ldl = NB;
    }
    const cpx<T>* Uop = A + (int64_t)col0 * N + k0;   // U (k, j) at j N + k0 + k
    cpx<T>* C = A + (int64_t)col0 * N + row0;
    constexpr int NBUF = DBUF ? 2 : 1;
    __shared__ cpx<T> Ls[NBUF][gk_v<T>][GT + GPAD];
    __shared__ cpx<T> Us[NBUF][gk_v<T>][GT + GPAD];

    const int tid = threadIdx.x;
    const int lane = tid & 63, wid = tid >> 6;
    const int wj = wid >> 1, wi = wid & 1;
    const cpx<T> zero = cmk((T)0, (T)0);
    // complex products by Gauss's three real products (the 3M method):
    // P1 = Ur Lr, P2 = Ui Li, P3 = (Ur + Ui)(Lr + Li); Re = P1 - P2, Im = P3 - P1 - P2
    acc_t acc1[2][2], acc2[2][2], acc3[2][2];
#pragma unroll
    for (int mj = 0; mj < 2; ++mj)
#pragma unroll
        for (int ni = 0; ni < 2; ++ni) {
            acc1[mj][ni] = (acc_t)(0);
            acc2[mj][ni] = (acc_t)(0);
            acc3[mj][ni] = (acc_t)(0);
        }
    gemm_stage<T> stg;

    const int nchunks = (nb + gk_v<T> - 1) / gk_v<T>;
    if (DBUF) {
        gemm_load_chunk<T, SUB>(stg, 0, tid, nrows, ncols, nb, Lop, ldl, Uop, N);
        gemm_store_chunk<T, NBUF>(Ls, Us, stg, 0, tid);
        __syncthreads();
    }
    for (int ch = 0; ch < nchunks; ++ch) {
        const int buf = DBUF ? (ch & 1) : 0;
        const bool more = ch + 1 < nchunks;
        if (DBUF) {
            if (more) gemm_load_chunk<T, SUB>(stg, (ch + 1) * gk_v<T>, tid, nrows, ncols, nb, Lop, ldl, Uop, N);
        } else {
            gemm_load_chunk<T, SUB>(stg, ch * gk_v<T>, tid, nrows, ncols, nb, Lop, ldl, Uop, N);
            gemm_store_chunk<T, NBUF>(Ls, Us, stg, 0, tid);
            __syncthreads();
        }
#pragma unroll
        for (int kk = 0; kk < gk_v<T>; kk += 4) {
            const int kr = kk + (lane >> 4);
            cpx<T> uf[2], lf[2];
#pragma unroll
            for (int mj = 0; mj < 2; ++mj) uf[mj] = Us[buf][kr][wj * 32 + mj * 16 + (lane & 15)];
#pragma unroll
            for (int ni = 0; ni < 2; ++ni) lf[ni] = Ls[buf][kr][wi * 32 + ni * 16 + (lane & 15)];
            T us[2], ls[2];
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                us[q] = uf[q].re + uf[q].im;
                ls[q] = lf[q].re + lf[q].im;
            }
#pragma unroll
            for (int mj = 0; mj < 2; ++mj) {
#pragma unroll
                for (int ni = 0; ni < 2; ++ni) {
                    acc1[mj][ni] = mfma_traits<T>::mac(uf[mj].re, lf[ni].re, acc1[mj][ni]);
                    acc2[mj][ni] = mfma_traits<T>::mac(uf[mj].im, lf[ni].im, acc2[mj][ni]);
                    acc3[mj][ni] = mfma_traits<T>::mac(us[mj], ls[ni], acc3[mj][ni]);
                }
            }
        }
        if (DBUF) {
            if (more) {
                gemm_store_chunk<T, NBUF>(Ls, Us, stg, buf ^ 1, tid);
                __syncthreads();
            }
        } else {
            __syncthreads();
        }
    }
    // epilogue: element v of this lane is D(j = row(lane, v), i = lane % 16) of each block
#pragma unroll
    for (int mj = 0; mj < 2; ++mj)
#pragma unroll
        for (int ni = 0; ni < 2; ++ni)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int j = wj * 32 + mj * 16 + mfma_traits<T>::row(lane, v);
                const int i = wi * 32 + ni * 16 + (lane & 15);
                if (i < nrows && j < ncols) {
                    cpx<T>* p = C + (int64_t)j * N + i;
                    const T p1 = acc1[mj][ni][v], p2 = acc2[mj][ni][v];
                    const T dre = p1 - p2, dim = acc3[mj][ni][v] - p1 - p2;
                    if (SUB) {
                        const cpx<T> o = *p;
                        *p = cmk(o.re - dre, o.im - dim);
                    } else {
                        *p = cmk(dre, dim);
                    }
                }
            }
}

// ---------------------------------------------------------------------------
// Host side: schedule and launches
// ---------------------------------------------------------------------------
// tiles of one GEMM op for a matrix of order N (mirrors the kernel's geometry)
static int gemm_tiles(int kind, int N, const fhw_lu_op& op) {
    if (N - op.k0 <= 0) return 0;
    if (kind == FHW_LU_OP_TRSM) {
        const int nc = N - (op.k0 + op.coff);
        return nc > 0 ? (nc + GT - 1) / GT : 0;
    }
    const int rb = op.k0 + op.roff, cb = op.k0 + op.coff;
    const int re = op.rlim > 0 ? std::min(N, rb + op.rlim) : N;
    const int ce = op.clim > 0 ? std::min(N, cb + op.clim) : N;
    if (re <= rb || ce <= cb) return 0;
    return ((re - rb + GT - 1) / GT) * ((ce - cb + GT - 1) / GT);
}

// Right-looking blocked LU with panels in pairs (p, p+1), k1 = k0 + 64:
//   panel p; pivots of p on the columns right of it; U = inv(L11) A on
//   those columns; update of panel p+1's 64 columns only (depth 64);
//   panel p+1; its pivots on the columns right of it and on panel p's L
//   columns (rows >= k1); update of the 64-row band k1.. of the trailing
//   columns (depth 64); U of panel p+1; then ONE update of the trailing block
//   below and right of the pair with depth 128 (both panels' L and U), which
//   reads and writes that block once per pair instead of once per panel.
// The solves replay panel p+1's pivots before panel p's update of the rows
// below (panel p's L rows carry them).
void lu_build_schedule(const int32_t* N, int32_t batch, fhw_lu_sched& sch) {
    int32_t maxN = 0;
    for (int q = 0; q < batch; ++q) maxN = std::max(maxN, N[q]);
    sch.nsteps = (maxN + NB - 1) / NB;
    sch.ops.clear();
    sch.prefix.clear();
    auto gemm = [&](int kind, int k0, int K, int roff, int rlim, int coff, int clim) {
        fhw_lu_op op{};
        op.kind = kind; op.k0 = k0; op.K = K; op.roff = roff; op.rlim = rlim; op.coff = coff; op.clim = clim;
        op.prefix_off = (int64_t)sch.prefix.size();
        int acc = 0;
        for (int q = 0; q < batch; ++q) {
            sch.prefix.push_back(acc);
            acc += gemm_tiles(kind, N[q], op);
        }
        sch.prefix.push_back(acc);
        op.grid = acc;
        if (acc > 0) sch.ops.push_back(op);
        else sch.prefix.resize((size_t)op.prefix_off);
    };
    auto swap = [&](int k0, int cbeg, int ccount) {
        int maxc = 0;
        for (int q = 0; q < batch; ++q) {
            if (N[q] <= k0) continue;
            const int ce = ccount > 0 ? std::min(N[q], cbeg + ccount) : N[q];
            maxc = std::max(maxc, ce - cbeg);
        }
        if (maxc <= 0) return;
        fhw_lu_op op{};
        op.kind = FHW_LU_OP_SWAP; op.k0 = k0; op.cbeg = cbeg; op.ccount = ccount; op.grid = (maxc + 255) / 256;
        sch.ops.push_back(op);
    };
    // One panel launch per rows-per-thread class (R = 1, 2, 4, 8, 16 for
    // 256 threads): each matrix still being factored runs the register shape
    // of its own panel height, not of the tallest panel in the batch.  A class
    // of fewer matrices than CUs is folded into the next taller class (it
    // would run alone as one under-filled wave of workgroups), and so is every
    // class of a batch of at most 256 matrices (one workgroup per CU or fewer:
    // each launch costs a full panel latency).  The matrices of a launch are
    // listed largest first, so the longest workgroups start first; a launch
    // over every matrix of an equal-order batch needs no list.
    bool uniform = true;
    for (int q = 1; q < batch; ++q) uniform = uniform && N[q] == N[0];
    auto panel = [&](int k0) {
        std::vector<int32_t> cls[5];
        for (int q = 0; q < batch; ++q) {
            const int rows = N[q] - k0;
            if (rows <= 0) continue;
            const int r = (rows + PANEL_THREADS - 1) / PANEL_THREADS;
            cls[r <= 1 ? 0 : (r <= 2 ? 1 : (r <= 4 ? 2 : (r <= 8 ? 3 : 4)))].push_back(q);
        }
        for (int c = 0; c < 4; ++c) {
            if (cls[c].empty()) continue;
            int up = c + 1;
            while (up < 5 && cls[up].empty()) ++up;
            if (up < 5 && (batch <= 256 || (int)cls[c].size() < 256)) {
                cls[up].insert(cls[up].end(), cls[c].begin(), cls[c].end());
                cls[c].clear();
            }
        }
        bool any = false;
        for (int c = 4; c >= 0; --c) {
            std::vector<int32_t>& ids = cls[c];
            if (ids.empty()) continue;
            any = true;
            fhw_lu_op op{};
            op.kind = FHW_LU_OP_PANEL; op.k0 = k0; op.R = 1 << c;
            op.grid = (int32_t)ids.size();
            if (uniform && (int32_t)ids.size() == batch) {
                op.prefix_off = -1;
            } else {
                std::stable_sort(ids.begin(), ids.end(), [&](int32_t x, int32_t y) { return N[x] > N[y]; });
                op.prefix_off = (int64_t)sch.prefix.size();
                sch.prefix.insert(sch.prefix.end(), ids.begin(), ids.end());
            }
            sch.ops.push_back(op);
        }
        if (!any) return;
        fhw_lu_op op{};
        op.kind = FHW_LU_OP_DIAGINV; op.k0 = k0;
        sch.ops.push_back(op);
    };
    for (int p = 0; p < sch.nsteps; p += 2) {
        const int k0 = p * NB, k1 = k0 + NB;
        panel(k0);
        swap(k0, k1, 0);
        gemm(FHW_LU_OP_TRSM, k0, 0, 0, 0, NB, 0);
        if (p + 1 >= sch.nsteps) {
            gemm(FHW_LU_OP_SUB, k0, NB, NB, 0, NB, 0);
            continue;
        }
        gemm(FHW_LU_OP_SUB, k0, NB, NB, 0, NB, NB);           // panel p+1's columns
        panel(k1);
        swap(k1, k1 + NB, 0);                                  // pivots of p+1, right columns
        swap(k1, k0, NB);                                      // ... and panel p's L columns
        gemm(FHW_LU_OP_SUB, k0, NB, NB, NB, 2 * NB, 0);       // band rows k1 .. k1+63
        gemm(FHW_LU_OP_TRSM, k1, 0, 0, 0, NB, 0);
        gemm(FHW_LU_OP_SUB, k0, 2 * NB, 2 * NB, 0, 2 * NB, 0);   // depth-128 trailing update
    }
}

template <typename T>
static void lu_set_lds_limits() {
    static std::atomic<uint64_t> done{0};
    fhw_once_on_device(done, [] {
        (void)hipFuncSetAttribute((const void*)k_lu_diaginv<T>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)sizeof(inv_lds<T>));
    });
}

// rows per thread R (from the tallest panel of the launch, for 256 threads)
// and sub-panel width W of the panel kernel, chosen to keep R*W complex values
// per thread in registers.  Batches of at most 256 matrices (one per CU or
// fewer) use 1024 threads per matrix instead: a quarter of the rows per
// thread, so each matrix's latency-bound panel work is spread wider.
template <typename T>
static hipError_t launch_panel(hipStream_t s, int R, const fhw_batch_dev& bd, int k0, cpx<T>* A, int32_t* piv,
                               int32_t* st, int grid, const int32_t* ids) {
#define FHW_PANEL(RR, WW, EE, PT) FHW_PANEL_D(RR, WW, EE, PT, 0)
#define FHW_PANEL_D(RR, WW, EE, PT, DD)                                                                       \
    hipLaunchKernelGGL((k_lu_panel<T, RR, WW, EE, PT, DD>), dim3(grid), dim3(PT), 0, s, k0, bd.N, bd.a_off, \
                       bd.piv_off, A, piv, st, ids)
#define FHW_PANEL_T(RR, WE, PT) FHW_PANEL_X(RR, WE, PT)
#define FHW_PANEL_X(...) FHW_PANEL(__VA_ARGS__)
    // large batches: (threads, W, WPE, PD) from the table, ceil(256 R / threads) rows per thread
#define FHW_PANEL_B(RR, TWE) FHW_PANEL_BX(RR, TWE)
#define FHW_PANEL_BX(RR, PTB, WW, EE, DD) FHW_PANEL_D((RR * 256 + PTB - 1) / PTB, WW, EE, PTB, DD)
    // (W, waves per SIMD) per case from panel_table.h, among the spill-free
    // register allocations; tall panels (R = 8 and 16, over 1024 rows) take
    // their workgroup size from the table too
    if (bd.batch <= 256) {
        const int R4 = (R + 3) / 4;   // rows per thread with 1024 threads
        if constexpr (sizeof(T) == 4) {
            switch (R4) {
                case 1: FHW_PANEL_T(1, FHW_PT_F32_1024_R1, 1024); break;
                case 2: FHW_PANEL_T(2, FHW_PT_F32_1024_R2, 1024); break;
                default: FHW_PANEL_T(4, FHW_PT_F32_1024_R4, 1024); break;
            }
        } else {
            switch (R4) {
                case 1: FHW_PANEL_T(1, FHW_PT_F64_1024_R1, 1024); break;
                case 2: FHW_PANEL_T(2, FHW_PT_F64_1024_R2, 1024); break;
                default: FHW_PANEL_T(4, FHW_PT_F64_1024_R4, 1024); break;
            }
        }
    } else if constexpr (sizeof(T) == 4) {
        switch (R) {
            case 1: FHW_PANEL_B(1, FHW_PB_F32_R1); break;
            case 2: FHW_PANEL_B(2, FHW_PB_F32_R2); break;
            case 4: FHW_PANEL_B(4, FHW_PB_F32_R4); break;
            case 8: FHW_PANEL_B(8, FHW_PB_F32_R8); break;
            default: FHW_PANEL_B(16, FHW_PB_F32_R16); break;
        }
    } else {
        switch (R) {
            case 1: FHW_PANEL_B(1, FHW_PB_F64_R1); break;
            case 2: FHW_PANEL_B(2, FHW_PB_F64_R2); break;
            case 4: FHW_PANEL_B(4, FHW_PB_F64_R4); break;
            case 8: FHW_PANEL_B(8, FHW_PB_F64_R8); break;
            default: FHW_PANEL_B(16, FHW_PB_F64_R16); break;
        }
    }
#undef FHW_PANEL_BX
#undef FHW_PANEL_B
#undef FHW_PANEL_X
#undef FHW_PANEL_T
#undef FHW_PANEL_D
#undef FHW_PANEL
    return hipGetLastError();
}

template <typename T>
static hipError_t lu_factor_t(hipStream_t s, const fhw_batch_dev& bd, const fhw_lu_sched& sch,
                              const int32_t* d_prefix, cpx<T>* A, int32_t* piv, cpx<T>* linv, int32_t* st,
                              fhw_prof* prof) {
    lu_set_lds_limits<T>();
    for (const fhw_lu_op& op : sch.ops) {
        hipError_t e = hipSuccess;
        switch (op.kind) {
            case FHW_LU_OP_PANEL:
                prof_begin(prof, FHW_STAGE_LU_PANEL, s);
                e = launch_panel<T>(s, op.R, bd, op.k0, A, piv, st, op.grid,
                                    op.prefix_off < 0 ? nullptr : d_prefix + op.prefix_off);
                prof_end(prof, s);
                break;
            case FHW_LU_OP_DIAGINV:
                prof_begin(prof, FHW_STAGE_LU_DIAGINV, s);
                hipLaunchKernelGGL((k_lu_diaginv<T>), dim3(bd.batch), dim3(INV_THREADS), sizeof(inv_lds<T>), s, op.k0,
                                   bd.N, bd.a_off, bd.linv_off, A, linv);
                prof_end(prof, s);
                break;
            case FHW_LU_OP_SWAP:
                prof_begin(prof, FHW_STAGE_LU_SWAP, s);
                hipLaunchKernelGGL((k_lu_swap<T>), dim3(bd.batch, op.grid), dim3(256), 0, s, op.k0, op.cbeg, op.ccount,
                                   bd.N, bd.a_off, bd.piv_off, A, piv);
                prof_end(prof, s);
                break;
            case FHW_LU_OP_TRSM:
                prof_begin(prof, FHW_STAGE_LU_TRSM, s);
                hipLaunchKernelGGL((k_lu_gemm<T, false>), dim3(op.grid), dim3(256), 0, s, op.k0, 0, 0, 0, op.coff, 0,
                                   d_prefix + op.prefix_off, bd.batch, bd.N, bd.a_off, bd.linv_off, A,
                                   (const cpx<T>*)linv);
                prof_end(prof, s);
                break;
            default:
                prof_begin(prof, FHW_STAGE_LU_UPDATE, s);
                hipLaunchKernelGGL((k_lu_gemm<T, true>), dim3(op.grid), dim3(256), 0, s, op.k0, op.K, op.roff, op.rlim,
                                   op.coff, op.clim, d_prefix + op.prefix_off, bd.batch, bd.N, bd.a_off, bd.linv_off,
                                   A, (const cpx<T>*)linv);
                prof_end(prof, s);
                break;
        }
        if (e == hipSuccess) e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

void lu_prepare(int precision) {
    if (precision == FHW_FP64) lu_set_lds_limits<double>();
    else lu_set_lds_limits<float>();
}

hipError_t launch_lu_factor(hipStream_t s, const fhw_batch_dev& b, const fhw_lu_sched& sch,
                            const int32_t* d_prefix, void* A, int32_t* piv, void* linv, int32_t* d_status,
                            int precision, fhw_prof* prof) {
    if (precision == FHW_FP64)
        return lu_factor_t<double>(s, b, sch, d_prefix, (zd*)A, piv, (zd*)linv, d_status, prof);
    return lu_factor_t<float>(s, b, sch, d_prefix, (zf*)A, piv, (zf*)linv, d_status, prof);
}
