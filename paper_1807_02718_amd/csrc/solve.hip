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

// Whether any row of a panel was exchanged (one wave, lane per row): most
// panels of these systems pivot on their diagonal, and the serial replay
// (one dependent pivot load per row) is then skipped.
__device__ __forceinline__ bool panel_pivots(const int* piv, int k0, int nb, int lane) {
    const bool sw = lane < nb && piv[k0 + lane] != k0 + lane;
    return __ballot(sw) != 0;
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
// WIDE (batches of at most 256 matrices): 1024 threads per matrix, and the
// diagonal-block products use all of them (16 per row, fully unrolled),
// shortening each matrix's chain of dependent loads; larger batches keep 256
// threads, one thread per row in the diagonal blocks, reading only the triangle.
template <typename T, bool WIDE, int TH = WIDE ? 1024 : SOLVE_THREADS>
__global__ __launch_bounds__(TH) void k_lu_solve(const int* __restrict__ Ns,
                                                            const int64_t* __restrict__ a_off,
                                                            const int64_t* __restrict__ piv_off,
                                                            const int64_t* __restrict__ linv_off,
                                                            const int64_t* __restrict__ v_off,
                                                            const cpx<T>* __restrict__ LUbase,
                                                            const int* __restrict__ pivbase,
                                                            const cpx<T>* __restrict__ linvbase, zd* __restrict__ v,
                                                            zd* __restrict__ acc, const int* __restrict__ skip,
                                                            int batch, fhw_grp grp) {
    static_assert((NB + (TH / 64) * NB) * sizeof(zd) <= FHW_SOLVE_STATIC_LDS, "static LDS of the solve");
    extern __shared__ zd xs[];
    __shared__ zd rhs[NB];
    __shared__ zd part[TH / 64][NB];
    // (matrix b, vector q) of this workgroup from the 1D grid of 8 ceil(batch
    // / 8) grp.n workgroups: workgroups go to the XCDs round-robin by linear
    // index, so matrix b's vectors all run on XCD b mod 8, where their reads
    // of its factors meet in one L2 (one vector per matrix: b = index)
    const int xcd = blockIdx.x & 7, k = blockIdx.x >> 3;
    const int jb = k / grp.n, q = k - jb * grp.n;
    const int b = xcd + 8 * jb;
    if (b >= batch) return;
    {
        v += q * grp.sv;
        if (acc) acc += q * grp.sacc;
        if (skip) skip += q * grp.sflag;
    }
    if (skip && skip[b]) return;
    const int N = Ns[b];
    const cpx<T>* LU = LUbase + a_off[b];
    const int* piv = pivbase + piv_off[b];
    const cpx<T>* Lb = linvbase + linv_off[b];
    zd* vb = v + v_off[b];
    const int tid = threadIdx.x;
    const int lane = tid & 63, wid = tid >> 6;
    for (int i = tid; i < N; i += TH) xs[i] = vb[i];
    const int np = (N + NB - 1) / NB;
    __syncthreads();
    // ---- forward.  Panels were factored in pairs (2q, 2q+1) and panel 2q's
    // L rows below the pair's first panel carry the pivots of panel 2q+1, so
    // those pivots are replayed before panel 2q's update of the rows below.
    for (int p = 0; p < np; ++p) {
        const int k0 = p * NB;
        const int nb = min(NB, N - k0);
        if (wid == 0 && (p & 1) == 0 && panel_pivots(piv, k0, nb, lane)) {
            if (lane == 0) replay_pivots(xs, piv, k0, nb);
        }
        __syncthreads();
        const cpx<T>* D = Lb + (int64_t)p * NB * NB;
        if constexpr (WIDE) {
            // y = inv(L11) x_block: row lane, 16 columns per wave, all loads in flight
            {
                zd sacc = cmk(0.0, 0.0);
#pragma unroll
                for (int u = 0; u < NB / (TH / 64); ++u) {
                    const int c = wid * (NB / (TH / 64)) + u;
                    const cpx<T> l = D[c * NB + lane];
                    if (c < lane && lane < nb) sacc = cfma(sacc, cmk((double)l.re, (double)l.im), xs[k0 + c]);
                }
                part[wid][lane] = sacc;
            }
            __syncthreads();
            if (tid < nb) {
                zd y = xs[k0 + tid];
#pragma unroll
                for (int q = 0; q < TH / 64; ++q) y = cadd(y, part[q][tid]);
                xs[k0 + tid] = y;
            }
            __syncthreads();
        } else {
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
        }
        if ((p & 1) == 0 && p + 1 < np) {
            const int nb2 = min(NB, N - k0 - NB);
            if (wid == 0 && panel_pivots(piv, k0 + NB, nb2, lane)) {
                if (lane == 0) replay_pivots(xs, piv, k0 + NB, nb2);
            }
            __syncthreads();
        }
        // rows below: RP rows per thread and pass.  Large batches: eight
        // columns per round trip (FP32 factors: two rows, sixteen 8-byte
        // loads in flight; FP64: one row).  A lone matrix on its CU is bound
        // by the round trips of this sweep, not by bytes: with FP32 factors,
        // one row per thread and CH = 16 columns per round trip, then the
        // eight-column steps and the tail as before, so each column meets the
        // same partial sum in the same order either way (FP64 factors keep
        // eight: sixteen measured slower there, with more register pressure)
        constexpr int RP = (sizeof(T) == 4 && !WIDE) ? 2 : 1;
        constexpr int CH = (WIDE && sizeof(T) == 4) ? 16 : 8;
        for (int i = k0 + nb + tid; i < N; i += RP * TH) {
            const cpx<T>* Li = LU + (int64_t)k0 * N + i;
            bool live[RP];
#pragma unroll
            for (int rr = 0; rr < RP; ++rr) live[rr] = i + rr * TH < N;
            zd sa[RP][4];
#pragma unroll
            for (int rr = 0; rr < RP; ++rr)
#pragma unroll
                for (int u = 0; u < 4; ++u) sa[rr][u] = cmk(0.0, 0.0);
            int c = 0;
            if constexpr (CH > 8) {
                for (; c + CH <= nb; c += CH) {
                    cpx<T> lw[CH];
#pragma unroll
                    for (int u = 0; u < CH; ++u) lw[u] = Li[(int64_t)(c + u) * N];
#pragma unroll
                    for (int u = 0; u < CH; ++u)
                        sa[0][u & 3] = cfma(sa[0][u & 3], cmk((double)lw[u].re, (double)lw[u].im), xs[k0 + c + u]);
                }
            }
            for (; c + 8 <= nb; c += 8) {
                cpx<T> la[RP][8];
#pragma unroll
                for (int u = 0; u < 8; ++u)
#pragma unroll
                    for (int rr = 0; rr < RP; ++rr)
                        la[rr][u] = live[rr] ? ld_maybe_stream<!WIDE>(&Li[(int64_t)(c + u) * N + rr * TH])
                                             : cmk((T)0, (T)0);
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const zd xc = xs[k0 + c + u];
#pragma unroll
                    for (int rr = 0; rr < RP; ++rr)
                        sa[rr][u & 3] = cfma(sa[rr][u & 3], cmk((double)la[rr][u].re, (double)la[rr][u].im), xc);
                }
            }
            for (; c < nb; ++c) {
#pragma unroll
                for (int rr = 0; rr < RP; ++rr) {
                    const cpx<T> l = live[rr] ? ld_maybe_stream<!WIDE>(&Li[(int64_t)c * N + rr * TH]) : cmk((T)0, (T)0);
                    sa[rr][0] = cfma(sa[rr][0], cmk((double)l.re, (double)l.im), xs[k0 + c]);
                }
            }
#pragma unroll
            for (int rr = 0; rr < RP; ++rr)
                if (live[rr])
                    xs[i + rr * TH] = csub(xs[i + rr * TH], cadd(cadd(sa[rr][0], sa[rr][1]), cadd(sa[rr][2], sa[rr][3])));
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
            constexpr int NW = TH / 64;
            // four independent partial sums per lane, eight loads in flight
            zd s4[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) s4[u] = cmk(0.0, 0.0);
            int c = c0 + wid;
            for (; c + 7 * NW < N; c += 8 * NW) {
                cpx<T> u8[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) u8[u] = ld_maybe_stream<!WIDE>(&Ur[(int64_t)(c + u * NW) * N]);
#pragma unroll
                for (int u = 0; u < 8; ++u)
                    s4[u & 3] = cfma(s4[u & 3], cmk((double)u8[u].re, (double)u8[u].im), xs[c + u * NW]);
            }
            for (; c < N; c += NW) {
                const cpx<T> u = ld_maybe_stream<!WIDE>(&Ur[(int64_t)c * N]);
                s4[0] = cfma(s4[0], cmk((double)u.re, (double)u.im), xs[c]);
            }
            s = cadd(cadd(s4[0], s4[1]), cadd(s4[2], s4[3]));
        }
        part[wid][lane] = s;
        __syncthreads();
        if (tid < nb) {
            zd t = xs[k0 + tid];
#pragma unroll
            for (int q = 0; q < TH / 64; ++q) t = csub(t, part[q][tid]);
            rhs[tid] = t;
        }
        __syncthreads();
        const cpx<T>* D = Lb + (int64_t)p * NB * NB;
        if constexpr (WIDE) {
            // x_block = inv(U11) rhs: row lane, 16 columns per wave
            {
                zd sacc = cmk(0.0, 0.0);
#pragma unroll
                for (int u = 0; u < NB / (TH / 64); ++u) {
                    const int c = wid * (NB / (TH / 64)) + u;
                    const cpx<T> d = D[c * NB + lane];
                    if (c >= lane && c < nb) sacc = cfma(sacc, cmk((double)d.re, (double)d.im), rhs[c]);
                }
                part[wid][lane] = sacc;
            }
            __syncthreads();
            if (tid < nb) {
                zd y = part[0][tid];
#pragma unroll
                for (int q = 1; q < TH / 64; ++q) y = cadd(y, part[q][tid]);
                xs[k0 + tid] = y;
            }
            __syncthreads();
        } else {
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
    }
    if (acc) {
        zd* ab = acc + v_off[b];
        for (int i = tid; i < N; i += TH) ab[i] = cadd(ab[i], xs[i]);
    } else {
        for (int i = tid; i < N; i += TH) vb[i] = xs[i];
    }
}

// The solves of NV vectors of a group at once, each factor entry loaded once
// for all of them (the vectors of a group share the matrix).  One workgroup
// of FHW_SM_TH threads per (matrix, run of NV vectors); dynamic LDS holds the
// NV solution vectors [NV][N] and the diagonal-block right-hand sides
// [NV][NB].  The forward sweep takes the same steps and pivot order as
// k_lu_solve; the backward sweep runs column-oriented (each solved block
// updates the rows above it, one thread per row), so no cross-wave partial
// sums are needed.  A vector whose skip flag is set is carried along but
// neither written nor accumulated.
#ifndef FHW_SM_TH
#define FHW_SM_TH 512    // threads per workgroup (1024: 14.5 ms, 256: 12.1 ms against 10.3 ms per group solve)
#endif
#ifndef FHW_SM_NV
#define FHW_SM_NV 4      // vectors per workgroup (halved when their LDS does not fit)
#endif
#ifndef FHW_SM_LD
#define FHW_SM_LD 8      // factor loads in flight per thread
#endif
#ifndef FHW_SM_MIN_BATCH
#define FHW_SM_MIN_BATCH 256   // smaller batches solve vector by vector (more workgroups)
#endif
#define SM_TH FHW_SM_TH
#define SM_LD FHW_SM_LD
template <typename T, int NV>
__global__ __launch_bounds__(SM_TH) void k_lu_solve_multi(const int* __restrict__ Ns,
                                                        const int64_t* __restrict__ a_off,
                                                        const int64_t* __restrict__ piv_off,
                                                        const int64_t* __restrict__ linv_off,
                                                        const int64_t* __restrict__ v_off,
                                                        const cpx<T>* __restrict__ LUbase,
                                                        const int* __restrict__ pivbase,
                                                        const cpx<T>* __restrict__ linvbase, zd* __restrict__ v,
                                                        zd* __restrict__ acc, const int* __restrict__ skip,
                                                        int ldx, int batch, fhw_grp grp) {
    constexpr int NW = SM_TH / 64;
    extern __shared__ zd smem[];
    zd* xs = smem;                                  // [NV][ldx]
    zd* rhs = smem + NV * ldx;                      // [NV][NB]
    // (matrix b, run of NV vectors) from the 1D grid of 8 ceil(batch / 8)
    // runs workgroups, numbered as in k_lu_solve: a matrix's runs go out one
    // after another on XCD b mod 8, so they stream its factors together
    const int runs = (grp.n + NV - 1) / NV;
    const int xcd = blockIdx.x & 7, kq = blockIdx.x >> 3;
    const int jb = kq / runs;
    const int b = xcd + 8 * jb;
    if (b >= batch) return;
    const int q0 = (kq - jb * runs) * NV;
    const int nv = min(NV, grp.n - q0);
    bool live[NV];
    bool any = false;
#pragma unroll
    for (int u = 0; u < NV; ++u) {
        live[u] = u < nv && !(skip && skip[(int64_t)(q0 + u) * grp.sflag + b]);
        any = any || live[u];
    }
    if (!any) return;
    const int N = Ns[b];
    const cpx<T>* LU = LUbase + a_off[b];
    const int* piv = pivbase + piv_off[b];
    const cpx<T>* Lb = linvbase + linv_off[b];
    const int64_t vo = v_off[b];
    const int tid = threadIdx.x;
    const int lane = tid & 63, wid = tid >> 6;
#pragma unroll
    for (int u = 0; u < NV; ++u)
        for (int i = tid; i < N; i += SM_TH)
            xs[u * ldx + i] = u < nv ? v[(int64_t)(q0 + u) * grp.sv + vo + i] : cmk(0.0, 0.0);
    const int np = (N + NB - 1) / NB;
    __syncthreads();
    // thread (row = lane, vector = wid + NW k) in the diagonal-block products
    for (int p = 0; p < np; ++p) {
        const int k0 = p * NB;
        const int nb = min(NB, N - k0);
        if (wid == 0 && (p & 1) == 0 && panel_pivots(piv, k0, nb, lane)) {
            if (tid < NV) replay_pivots(xs + tid * ldx, piv, k0, nb);
        }
        __syncthreads();
        const cpx<T>* D = Lb + (int64_t)p * NB * NB;
        {
            zd y[(NV + NW - 1) / NW];
#pragma unroll
            for (int k = 0; k < (NV + NW - 1) / NW; ++k) {
                const int u = wid + NW * k;
                if (u < NV && lane < nb) {
                    zd t = xs[u * ldx + k0 + lane];
                    for (int c = 0; c < lane; ++c) {
                        const cpx<T> l = D[c * NB + lane];
                        t = cfma(t, cmk((double)l.re, (double)l.im), xs[u * ldx + k0 + c]);
                    }
                    y[k] = t;
                }
            }
            __syncthreads();
#pragma unroll
            for (int k = 0; k < (NV + NW - 1) / NW; ++k) {
                const int u = wid + NW * k;
                if (u < NV && lane < nb) xs[u * ldx + k0 + lane] = y[k];
            }
            __syncthreads();
        }
        if ((p & 1) == 0 && p + 1 < np) {
            const int nb2 = min(NB, N - k0 - NB);
            if (wid == 0 && panel_pivots(piv, k0 + NB, nb2, lane)) {
                if (tid < NV) replay_pivots(xs + tid * ldx, piv, k0 + NB, nb2);
            }
            __syncthreads();
        }
        for (int i = k0 + nb + tid; i < N; i += SM_TH) {
            const cpx<T>* Li = LU + (int64_t)k0 * N + i;
            zd sv[NV];
#pragma unroll
            for (int u = 0; u < NV; ++u) sv[u] = cmk(0.0, 0.0);
            int c = 0;
            // SM_LD columns' loads in flight before their products
            for (; c + SM_LD <= nb; c += SM_LD) {
                cpx<T> l4[SM_LD];
#pragma unroll
                for (int e = 0; e < SM_LD; ++e) l4[e] = Li[(int64_t)(c + e) * N];
#pragma unroll
                for (int e = 0; e < SM_LD; ++e) {
                    const zd l = cmk((double)l4[e].re, (double)l4[e].im);
#pragma unroll
                    for (int u = 0; u < NV; ++u) sv[u] = cfma(sv[u], l, xs[u * ldx + k0 + c + e]);
                }
            }
            for (; c < nb; ++c) {
                const cpx<T> l1 = Li[(int64_t)c * N];
                const zd l = cmk((double)l1.re, (double)l1.im);
#pragma unroll
                for (int u = 0; u < NV; ++u) sv[u] = cfma(sv[u], l, xs[u * ldx + k0 + c]);
            }
#pragma unroll
            for (int u = 0; u < NV; ++u) xs[u * ldx + i] = csub(xs[u * ldx + i], sv[u]);
        }
        __syncthreads();
    }
    // Backward, column-oriented like the forward sweep: per block from the
    // last, x_block = inv(U11) b_block, then the rows above take
    // b_i -= U(i, block) x_block, one thread per row (coalesced down the
    // columns); no cross-wave partial sums.
    for (int p = np - 1; p >= 0; --p) {
        const int k0 = p * NB;
        const int nb = min(NB, N - k0);
        for (int e = tid; e < NV * NB; e += SM_TH) {
            const int u = e / NB, l = e - u * NB;
            if (l < nb) rhs[u * NB + l] = xs[u * ldx + k0 + l];
        }
        __syncthreads();
        const cpx<T>* D = Lb + (int64_t)p * NB * NB;
#pragma unroll
        for (int k = 0; k < (NV + NW - 1) / NW; ++k) {
            const int u = wid + NW * k;
            if (u < NV && lane < nb) {
                zd y = cmk(0.0, 0.0);
                for (int c = lane; c < nb; ++c) {
                    const cpx<T> d = D[c * NB + lane];
                    y = cfma(y, cmk((double)d.re, (double)d.im), rhs[u * NB + c]);
                }
                xs[u * ldx + k0 + lane] = y;
            }
        }
        __syncthreads();
        for (int i = tid; i < k0; i += SM_TH) {
            const cpx<T>* Ui = LU + (int64_t)k0 * N + i;
            zd sv[NV];
#pragma unroll
            for (int u = 0; u < NV; ++u) sv[u] = cmk(0.0, 0.0);
            int c = 0;
            for (; c + SM_LD <= nb; c += SM_LD) {
                cpx<T> u8[SM_LD];
#pragma unroll
                for (int e = 0; e < SM_LD; ++e) u8[e] = Ui[(int64_t)(c + e) * N];
#pragma unroll
                for (int e = 0; e < SM_LD; ++e) {
                    const zd uu = cmk((double)u8[e].re, (double)u8[e].im);
#pragma unroll
                    for (int u = 0; u < NV; ++u) sv[u] = cfma(sv[u], uu, xs[u * ldx + k0 + c + e]);
                }
            }
            for (; c < nb; ++c) {
                const cpx<T> u1 = Ui[(int64_t)c * N];
                const zd uu = cmk((double)u1.re, (double)u1.im);
#pragma unroll
                for (int u = 0; u < NV; ++u) sv[u] = cfma(sv[u], uu, xs[u * ldx + k0 + c]);
            }
#pragma unroll
            for (int u = 0; u < NV; ++u) xs[u * ldx + i] = csub(xs[u * ldx + i], sv[u]);
        }
        __syncthreads();
    }
#pragma unroll
    for (int u = 0; u < NV; ++u) {
        if (!live[u]) continue;
        if (acc) {
            zd* ab = acc + (int64_t)(q0 + u) * grp.sacc + vo;
            for (int i = tid; i < N; i += SM_TH) ab[i] = cadd(ab[i], xs[u * ldx + i]);
        } else {
            zd* vb = v + (int64_t)(q0 + u) * grp.sv + vo;
            for (int i = tid; i < N; i += SM_TH) vb[i] = xs[u * ldx + i];
        }
    }
}

template <typename T, int NV>
static size_t solve_multi_lds(int ldx) {
    return sizeof(zd) * ((size_t)NV * ldx + (size_t)NV * NB);
}

// r = g - A x with the FP64 column-major matrix; norms[2b] = ||r||_2,
// norms[2b+1] = ||g||_2.  Marks done[b] (and sweeps[b] = sweep) once
// ||r|| <= tol ||g||.  Matrices already done are skipped.  pending (optional)
// counts the matrices of this launch that are still above the tolerance.
// Grid (matrix, row block of 256/PH rows): thread (row, column phase) with PH
// column phases summed in a fixed order (PH = 4 for small batches, so that
// one matrix spreads over many workgroups; PH = 1 for large ones, so that x
// is staged fewer times); per-block partial norms; the last block of a matrix
// to finish (a counter, reset by that block) adds the partials in block
// order, so the norms are deterministic.
template <int PH>
__global__ __launch_bounds__(SOLVE_THREADS) void k_residual(const int* __restrict__ Ns,
                                                            const int64_t* __restrict__ a_off,
                                                            const int64_t* __restrict__ v_off,
                                                            const zd* __restrict__ Abase, const zd* __restrict__ x,
                                                            const zd* __restrict__ g, zd* __restrict__ r,
                                                            double* __restrict__ part, int* __restrict__ count,
                                                            int nblk_max, double* __restrict__ norms, double tol,
                                                            int* __restrict__ done, int* __restrict__ sweeps,
                                                            int sweep, int* __restrict__ pending, fhw_grp grp) {
    constexpr int RES_ROWS = SOLVE_THREADS / PH;
    {
        const int q = blockIdx.z;   // incidence of the group
        x += q * grp.sx;
        g += q * grp.sg;
        r += q * grp.sr;
        part += q * grp.spart;
        count += q * grp.scount;
        norms += q * grp.snorm;
        if (done) done += q * grp.sflag;
        if (sweeps) sweeps += q * grp.sflag;
    }
    extern __shared__ zd xs[];
    __shared__ zd cs[PH][RES_ROWS];
    __shared__ double wred[2][RES_ROWS / 64];
    __shared__ int last;
    const int b = blockIdx.x;
    if (done && done[b]) return;
    const int N = Ns[b];
    const int nblk = (N + RES_ROWS - 1) / RES_ROWS;
    const int yb = blockIdx.y;
    if (yb >= nblk) return;
    const zd* A = Abase + a_off[b];
    const zd* xb = x + v_off[b];
    const zd* gb = g + v_off[b];
    zd* rb = r + v_off[b];
    const int tid = threadIdx.x;
    const int il = tid % RES_ROWS, cg = tid / RES_ROWS;
    for (int i = tid; i < N; i += SOLVE_THREADS) xs[i] = xb[i];
    __syncthreads();
    const int i = yb * RES_ROWS + il;
    zd s = cmk(0.0, 0.0);
    if (i < N) {
        constexpr int NC = PH;
        zd s4[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) s4[u] = cmk(0.0, 0.0);
        int c = cg;
        for (; c + 3 * NC < N; c += 4 * NC) {
            zd a4[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) a4[u] = ld_maybe_stream<PH == 1>(&A[(int64_t)(c + u * NC) * N + i]);
#pragma unroll
            for (int u = 0; u < 4; ++u) s4[u] = cfma(s4[u], a4[u], xs[c + u * NC]);
        }
        for (; c < N; c += NC) s4[0] = cfma(s4[0], ld_maybe_stream<PH == 1>(&A[(int64_t)c * N + i]), xs[c]);
        s = cadd(cadd(s4[0], s4[1]), cadd(s4[2], s4[3]));
    }
    cs[cg][il] = s;
    __syncthreads();
    if (cg == 0) {
        double rr = 0.0, gg = 0.0;
        if (i < N) {
            zd t = cs[0][il];
#pragma unroll
            for (int q = 1; q < PH; ++q) t = cadd(t, cs[q][il]);
            const zd gi = gb[i];
            const zd ri = csub(gi, t);
            rb[i] = ri;
            rr = ri.re * ri.re + ri.im * ri.im;
            gg = gi.re * gi.re + gi.im * gi.im;
        }
        rr = wave_sum(rr);
        gg = wave_sum(gg);
        if ((il & 63) == 0) { wred[0][il >> 6] = rr; wred[1][il >> 6] = gg; }
    }
    __syncthreads();
    if (tid == 0) {
        double rr = 0.0, gg = 0.0;
        for (int q = 0; q < RES_ROWS / 64; ++q) { rr += wred[0][q]; gg += wred[1][q]; }
        double* pb = part + 2 * ((int64_t)b * nblk_max + yb);
        pb[0] = rr;
        pb[1] = gg;
        __threadfence();
        last = (atomicAdd(&count[b], 1) == nblk - 1);
    }
    __syncthreads();
    if (last && tid == 0) {
        __threadfence();
        double R2 = 0.0, G2 = 0.0;
        const double* pb = part + 2 * (int64_t)b * nblk_max;
        for (int q = 0; q < nblk; ++q) {
            R2 += pb[2 * q];
            G2 += pb[2 * q + 1];
        }
        count[b] = 0;
        norms[2 * b] = sqrt(R2);
        norms[2 * b + 1] = sqrt(G2);
        if (done && R2 <= tol * tol * G2) {
            done[b] = 1;
            if (sweeps) sweeps[b] = sweep;
        } else if (pending) {
            atomicAdd(pending, 1);
        }
    }
}

// The residuals of a whole group in one pass over A: r_q = g_q - A x_q for
// the n <= FHW_INC_GROUP vectors of the group (vector q at x + q sx, ...),
// each matrix entry loaded once for all of them.  Grid (matrix, 256-row
// block), one row per thread; x staged in LDS RM_CH columns at a time for all
// vectors.  Norms, flags and the block-counter protocol as k_residual, per
// vector: a matrix is skipped when every vector of the group is done, and a
// vector already done keeps its flags (its norms are recomputed from the same
// x, in the same order, so they are unchanged).
// GT: the group width the kernel is built for (2, 4, 8 or 16, the group's n
// rounded up): x of the absent vectors q >= n is staged as zeros and every
// vector accumulates unconditionally, so the inner loop is branch-free.
#define RM_CH 128
#define RM_LD 4          // matrix loads in flight per thread (8 and 16 measured slower)
template <int GT>
__global__ __launch_bounds__(SOLVE_THREADS) void k_residual_multi(const int* __restrict__ Ns,
                                                                const int64_t* __restrict__ a_off,
                                                                const int64_t* __restrict__ v_off,
                                                                const zd* __restrict__ Abase,
                                                                const zd* __restrict__ x, const zd* __restrict__ g,
                                                                zd* __restrict__ r, double* __restrict__ part,
                                                                int* __restrict__ count, int nblk_max,
                                                                double* __restrict__ norms, double tol,
                                                                int* __restrict__ done, int* __restrict__ sweeps,
                                                                int sweep, int* __restrict__ pending, fhw_grp grp) {
    constexpr int G = GT;
    static_assert(GT <= FHW_INC_GROUP, "a group holds at most FHW_INC_GROUP vectors");
    __shared__ zd xs[G][RM_CH];
    __shared__ double wred[G][2][SOLVE_THREADS / 64];
    __shared__ int last;
    const int n = grp.n;
    const int b = blockIdx.x;
    if (done) {
        bool all = true;
        for (int q = 0; q < n; ++q) all = all && done[q * grp.sflag + b];
        if (all) return;
    }
    const int N = Ns[b];
    const int nblk = (N + SOLVE_THREADS - 1) / SOLVE_THREADS;
    const int yb = blockIdx.y;
    if (yb >= nblk) return;
    const zd* A = Abase + a_off[b];
    const int64_t vo = v_off[b];
    const int tid = threadIdx.x;
    const int lane = tid & 63, wid = tid >> 6;
    const int i = yb * SOLVE_THREADS + tid;
    zd s[G];
#pragma unroll
    for (int q = 0; q < G; ++q) s[q] = cmk(0.0, 0.0);
    for (int c0 = 0; c0 < N; c0 += RM_CH) {
        const int cnt = min(RM_CH, N - c0);
        __syncthreads();
        for (int e = tid; e < G * cnt; e += SOLVE_THREADS) {
            const int q = e / cnt, c = e - q * cnt;
            xs[q][c] = q < n ? x[q * grp.sx + vo + c0 + c] : cmk(0.0, 0.0);
        }
        __syncthreads();
        if (i < N) {
            const zd* Ac = A + (int64_t)c0 * N + i;
            int c = 0;
            for (; c + RM_LD <= cnt; c += RM_LD) {
                zd a4[RM_LD];
#pragma unroll
                for (int u = 0; u < RM_LD; ++u) a4[u] = ld_stream(&Ac[(int64_t)(c + u) * N]);
#pragma unroll
                for (int u = 0; u < RM_LD; ++u) {
#pragma unroll
                    for (int q = 0; q < G; ++q) s[q] = cfma(s[q], a4[u], xs[q][c + u]);
                }
            }
            for (; c < cnt; ++c) {
                const zd a = ld_stream(&Ac[(int64_t)c * N]);
#pragma unroll
                for (int q = 0; q < G; ++q) s[q] = cfma(s[q], a, xs[q][c]);
            }
        }
    }
    // (a single-exit loop, so that it unrolls and s stays in registers)
#pragma unroll
    for (int q = 0; q < G; ++q) {
        if (q < n) {
            double rr = 0.0, gg = 0.0;
            if (i < N) {
                const zd gi = g[q * grp.sg + vo + i];
                const zd ri = csub(gi, s[q]);
                r[q * grp.sr + vo + i] = ri;
                rr = ri.re * ri.re + ri.im * ri.im;
                gg = gi.re * gi.re + gi.im * gi.im;
            }
            rr = wave_sum(rr);
            gg = wave_sum(gg);
            if (lane == 0) {
                wred[q][0][wid] = rr;
                wred[q][1][wid] = gg;
            }
        }
    }
    __syncthreads();
    if (tid < n) {
        const int q = tid;
        double rr = 0.0, gg = 0.0;
        for (int w = 0; w < SOLVE_THREADS / 64; ++w) {
            rr += wred[q][0][w];
            gg += wred[q][1][w];
        }
        double* pb = part + q * grp.spart + 2 * ((int64_t)b * nblk_max + yb);
        pb[0] = rr;
        pb[1] = gg;
    }
    __syncthreads();
    if (tid == 0) {
        __threadfence();
        last = (atomicAdd(&count[b], 1) == nblk - 1);
    }
    __syncthreads();
    if (last && tid < n) {
        __threadfence();
        const int q = tid;
        double R2 = 0.0, G2 = 0.0;
        const double* pb = part + q * grp.spart + 2 * (int64_t)b * nblk_max;
        for (int k = 0; k < nblk; ++k) {
            R2 += pb[2 * k];
            G2 += pb[2 * k + 1];
        }
        double* nq = norms + q * grp.snorm;
        nq[2 * b] = sqrt(R2);
        nq[2 * b + 1] = sqrt(G2);
        if (done && !done[q * grp.sflag + b]) {
            if (R2 <= tol * tol * G2) {
                done[q * grp.sflag + b] = 1;
                if (sweeps) sweeps[q * grp.sflag + b] = sweep;
            } else if (pending) {
                atomicAdd(pending, 1);
            }
        }
    }
    if (last && tid == 0) count[b] = 0;
}

__global__ void k_c128_to_c64(const zd* __restrict__ src, zf* __restrict__ dst, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) dst[i] = cmk((float)src[i].re, (float)src[i].im);
}

hipError_t launch_lu_solve(hipStream_t s, const fhw_batch_dev& b, int32_t maxN, const void* LU, const int32_t* piv,
                           const void* linv, void* x, const int32_t* d_skip, int precision, const fhw_grp& grp) {
    return launch_lu_solve_acc(s, b, maxN, LU, piv, linv, x, nullptr, d_skip, precision, grp);
}

hipError_t launch_lu_solve_acc(hipStream_t s, const fhw_batch_dev& b, int32_t maxN, const void* LU,
                               const int32_t* piv, const void* linv, void* x, void* acc, const int32_t* d_skip,
                               int precision, const fhw_grp& grp) {
    if (grp.n < 1 || grp.n > 65535) return hipErrorInvalidValue;
    // several vectors on a large batch: one pass over each matrix's factors
    // per run of FHW_SM_NV vectors (or half as many), when their LDS fits the
    // device's limit
    int dev = 0, lds_max = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
        lds_max = 0;
    constexpr int NV1 = FHW_SM_NV, NV2 = FHW_SM_NV / 2;
    const int nv_fit = solve_multi_lds<double, NV1>(maxN) <= (size_t)lds_max                ? NV1
                       : NV2 > 1 && solve_multi_lds<double, NV2>(maxN) <= (size_t)lds_max ? NV2
                                                                                            : 1;
    if (grp.n > 1 && b.batch > FHW_SM_MIN_BATCH && nv_fit > 1) {
        static std::atomic<uint64_t> mattr{0};
        fhw_once_on_device(mattr, [&] {
            const int dyn = lds_max;
            (void)hipFuncSetAttribute((const void*)k_lu_solve_multi<double, NV1>,
                                      hipFuncAttributeMaxDynamicSharedMemorySize, dyn);
            (void)hipFuncSetAttribute((const void*)k_lu_solve_multi<double, NV2>,
                                      hipFuncAttributeMaxDynamicSharedMemorySize, dyn);
            (void)hipFuncSetAttribute((const void*)k_lu_solve_multi<float, NV1>,
                                      hipFuncAttributeMaxDynamicSharedMemorySize, dyn);
            (void)hipFuncSetAttribute((const void*)k_lu_solve_multi<float, NV2>,
                                      hipFuncAttributeMaxDynamicSharedMemorySize, dyn);
        });
        const int ldx = maxN;
#define FHW_SOLVE_M(TT, NVV)                                                                                   \
    hipLaunchKernelGGL((k_lu_solve_multi<TT, NVV>), dim3((unsigned)(8 * ((b.batch + 7) / 8) * ((grp.n + NVV - 1) / NVV))), \
                       dim3(SM_TH), (solve_multi_lds<TT, NVV>(ldx)), s, b.N, b.a_off, b.piv_off, b.linv_off, b.v_off,  \
                       (const cpx<TT>*)LU, piv, (const cpx<TT>*)linv, (zd*)x, (zd*)acc, d_skip, ldx, b.batch, grp)
        const bool full = nv_fit == NV1;
        if (precision == FHW_FP64) {
            if (full) FHW_SOLVE_M(double, NV1); else FHW_SOLVE_M(double, NV2);
        } else {
            if (full) FHW_SOLVE_M(float, NV1); else FHW_SOLVE_M(float, NV2);
        }
#undef FHW_SOLVE_M
        return hipGetLastError();
    }
    size_t lds = (size_t)maxN * sizeof(zd);
    static std::atomic<uint64_t> attr{0};
    fhw_once_on_device(attr, [&] {
        // solution vectors up to N = 4096 (64 KiB) beside the static LDS
        const int dyn = 4096 * (int)sizeof(zd);
        (void)hipFuncSetAttribute((const void*)k_lu_solve<double, true>, hipFuncAttributeMaxDynamicSharedMemorySize, dyn);
        (void)hipFuncSetAttribute((const void*)k_lu_solve<double, false>, hipFuncAttributeMaxDynamicSharedMemorySize, dyn);
        (void)hipFuncSetAttribute((const void*)k_lu_solve<float, true>, hipFuncAttributeMaxDynamicSharedMemorySize, dyn);
        (void)hipFuncSetAttribute((const void*)k_lu_solve<float, false>, hipFuncAttributeMaxDynamicSharedMemorySize, dyn);
    });
#define FHW_SOLVE(TT, WW)                                                                                     \
    hipLaunchKernelGGL((k_lu_solve<TT, WW>), dim3((unsigned)(8 * ((b.batch + 7) / 8) * grp.n)),                    \
                       dim3(WW ? 1024 : SOLVE_THREADS), lds, s, b.N, b.a_off, b.piv_off, b.linv_off, b.v_off,           \
                       (const cpx<TT>*)LU, piv, (const cpx<TT>*)linv, (zd*)x, (zd*)acc, d_skip, b.batch, grp)
    const bool wide = b.batch <= 256;
    if (precision == FHW_FP64) {
        if (wide) FHW_SOLVE(double, true); else FHW_SOLVE(double, false);
    } else {
        if (wide) FHW_SOLVE(float, true); else FHW_SOLVE(float, false);
    }
#undef FHW_SOLVE
    return hipGetLastError();
}

hipError_t launch_residual_t(hipStream_t s, const fhw_batch_dev& b, int32_t maxN, const void* A64, const void* x,
                             const void* g, void* r, double* part, int32_t* count, double* norms, double tol,
                             int32_t* done, int32_t* sweeps, int sweep, int32_t* pending, const fhw_grp& grp) {
    if (grp.n < 1 || grp.n > 65535) return hipErrorInvalidValue;
    size_t lds = (size_t)maxN * sizeof(zd);
    static std::atomic<uint64_t> attr{0};
    fhw_once_on_device(attr, [&] {
        const int dyn = 4096 * (int)sizeof(zd);
        (void)hipFuncSetAttribute((const void*)k_residual<1>, hipFuncAttributeMaxDynamicSharedMemorySize, dyn);
        (void)hipFuncSetAttribute((const void*)k_residual<4>, hipFuncAttributeMaxDynamicSharedMemorySize, dyn);
    });
    // a group of several vectors: one pass over each matrix for all of them,
    // at any batch size (the per-vector kernel reads each matrix once per
    // vector; a serving round of 30 systems with 16 vectors each took 6 ms of
    // per-vector residuals per launch)
    if (grp.n > 1 && grp.n <= FHW_INC_GROUP) {
        const int nblk = (maxN + SOLVE_THREADS - 1) / SOLVE_THREADS;
#define FHW_RES_M(GG)                                                                                           \
    hipLaunchKernelGGL(k_residual_multi<GG>, dim3(b.batch, nblk), dim3(SOLVE_THREADS), 0, s, b.N, b.a_off, b.v_off, \
                       (const zd*)A64, (const zd*)x, (const zd*)g, (zd*)r, part, count, nblk, norms, tol, done,    \
                       sweeps, sweep, pending, grp)
        if (grp.n <= 2) FHW_RES_M(2);
        else if (grp.n <= 4) FHW_RES_M(4);
        else if (grp.n <= 8) FHW_RES_M(8);
        else FHW_RES_M(16);
#undef FHW_RES_M
        return hipGetLastError();
    }
    // 256-row blocks when they alone give >= 1024 workgroups, else 64-row blocks
    const bool wide = (int64_t)b.batch * grp.n * ((maxN + 255) / 256) >= 1024;
    const int rows = wide ? SOLVE_THREADS : SOLVE_THREADS / 4;
    const int nblk = (maxN + rows - 1) / rows;
    if (wide)
        hipLaunchKernelGGL(k_residual<1>, dim3(b.batch, nblk, grp.n), dim3(SOLVE_THREADS), lds, s, b.N, b.a_off,
                           b.v_off, (const zd*)A64, (const zd*)x, (const zd*)g, (zd*)r, part, count, nblk, norms, tol,
                           done, sweeps, sweep, pending, grp);
    else
        hipLaunchKernelGGL(k_residual<4>, dim3(b.batch, nblk, grp.n), dim3(SOLVE_THREADS), lds, s, b.N, b.a_off,
                           b.v_off, (const zd*)A64, (const zd*)x, (const zd*)g, (zd*)r, part, count, nblk, norms, tol,
                           done, sweeps, sweep, pending, grp);
    return hipGetLastError();
}

// Status words of nf (incidence, system) pairs kept in caller-provided
// device memory: cleared before the solves, summarised after them.
__global__ void k_status_clear(int32_t* __restrict__ done, int32_t* __restrict__ sweeps,
                               int32_t* __restrict__ notdone, int64_t nf) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nf) {
        done[i] = 0;
        sweeps[i] = 0;
    }
    if (i == 0) *notdone = 0;
}

// resid[j] = ||r|| / ||g|| after the refinement (-1 without it); sweeps_out[j]
// = the sweep at which pair j met the tolerance, refine_max if it never did
// (0 without refinement); notdone counts the pairs that never did.
__global__ void k_status_finish(const int32_t* __restrict__ done, const int32_t* __restrict__ sweeps,
                                const double* __restrict__ norms, int64_t nf, int refine, int refine_max,
                                double* __restrict__ resid, int32_t* __restrict__ sweeps_out,
                                int32_t* __restrict__ notdone) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= nf) return;
    if (!refine) {
        resid[j] = -1.0;
        sweeps_out[j] = 0;
        return;
    }
    const double rn = norms[2 * j], gn = norms[2 * j + 1];
    resid[j] = gn > 0.0 ? rn / gn : 0.0;
    sweeps_out[j] = done[j] ? sweeps[j] : refine_max;
    if (!done[j]) atomicAdd(notdone, 1);
}

hipError_t launch_status_clear(hipStream_t s, int32_t* done, int32_t* sweeps, int32_t* notdone, int64_t nf) {
    const int64_t blocks = std::max<int64_t>(1, (nf + 255) / 256);
    hipLaunchKernelGGL(k_status_clear, dim3((unsigned)blocks), dim3(256), 0, s, done, sweeps, notdone, nf);
    return hipGetLastError();
}

hipError_t launch_status_finish(hipStream_t s, const int32_t* done, const int32_t* sweeps, const double* norms,
                                int64_t nf, int refine, int refine_max, double* resid, int32_t* sweeps_out,
                                int32_t* notdone) {
    const int64_t blocks = std::max<int64_t>(1, (nf + 255) / 256);
    hipLaunchKernelGGL(k_status_finish, dim3((unsigned)blocks), dim3(256), 0, s, done, sweeps, norms, nf, refine,
                       refine_max, resid, sweeps_out, notdone);
    return hipGetLastError();
}

hipError_t launch_convert_c128_c64(hipStream_t s, const void* src, void* dst, int64_t n) {
    int blocks = (int)std::min<int64_t>((n + 255) / 256, 65536);
    hipLaunchKernelGGL(k_c128_to_c64, dim3(blocks), dim3(256), 0, s, (const zd*)src, (zf*)dst, n);
    return hipGetLastError();
}
