// Layer-potential evaluation of the frequency-domain field (eqs.
// freq_domain_repr and Ukslow_repr, step F5):
//   V(r, omega_j) = int_Gamma psi_j G dsigma
//               ~= (2 pi / N_j) sum_i (i/4) H0(kappa_j |r - x_i|) |x'_i| psi_j,i
// written on the full DFT grid with V(r, -omega) = conj V(r, omega) and the
// omega = 0 entry set by the caller.
#include "fhw_device.h"
#include "fhw_internal.h"

// One wave per (observation point, frequency); lanes stride over the nodes,
// fixed-order wave reduction.
__global__ __launch_bounds__(256, 4) void k_field(const fhw_field_item* __restrict__ items, int F,
                                               const zd* __restrict__ psi, const double* __restrict__ obs, int N_r,
                                               double zero_value, zd* __restrict__ V) {
    __shared__ double s_poly[FHW_BES_POLY_LEN];   // Bessel interval polynomials, gathered per lane
    for (int e = threadIdx.x; e < FHW_BES_POLY_LEN; e += blockDim.x) s_poly[e] = fhw_bes_poly[e];
    __syncthreads();
    const int wave = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (wave >= N_r * F) return;
    const int r = wave / F;
    const int j = wave - r * F;           // frequency index, omega = (j+1) W/F
    const fhw_field_item it = items[j];
    const int N = it.N;
    const double* x1 = it.geom;
    const double* x2 = it.geom + N;
    const double* sp = it.geom + 6 * N;
    const zd* ps = psi + it.psi_off;
    const double o1 = obs[2 * r], o2 = obs[2 * r + 1];
    zd acc = cmk(0.0, 0.0);
    for (int i = lane; i < N; i += 64) {
        const double d1 = o1 - x1[i], d2 = o2 - x2[i];
        const double z = it.kappa * sqrt(d1 * d1 + d2 * d2);
        double J0, Y0;
        fhw_bessel0(z, J0, Y0, s_poly);
        // (i/4) H0 = (-Y0/4, J0/4), weighted by |x'_i|
        const zd gk = cmk(-0.25 * Y0 * sp[i], 0.25 * J0 * sp[i]);
        acc = cfma(acc, gk, ps[i]);
    }
    acc.re = wave_sum(acc.re);
    acc.im = wave_sum(acc.im);
    if (lane == 0) {
        const double wq = 2.0 * FHW_PI / (double)N;
        const zd val = cmk(wq * acc.re, wq * acc.im);
        zd* Vr = V + (int64_t)r * 2 * F;
        if (j < F - 1) Vr[F + 1 + j] = val;   // omega = (j+1) dw
        Vr[F - 1 - j] = cconj(val);          // omega = -(j+1) dw
        if (j == 0) Vr[F] = cmk(zero_value, 0.0);
    }
}

// Kernel of the combined potential at observation point (o1, o2) for a node
// at (x1, x2) with speed sp = |x'| and unit normal (n1, n2):
//   |x'| [ (i kappa/4) H1(kappa rho) nu . (r - x)/rho + (eta/4) H0(kappa rho) ]
__device__ __forceinline__ zd combined_kernel_at(double x1, double x2, double sp, double n1, double n2, double o1,
                                                double o2, double kappa, double eta,
                                                const double* poly = fhw_bes_poly) {
    const double d1 = o1 - x1, d2 = o2 - x2;
    const double rho = sqrt(d1 * d1 + d2 * d2);
    double J0, Y0, J1, Y1;
    fhw_bessel01(kappa * rho, J0, Y0, J1, Y1, poly);
    const double cn = (n1 * d1 + n2 * d2) / rho;
    const double a = 0.25 * kappa * cn, e = 0.25 * eta;
    return cmk(sp * (e * J0 - a * Y1), sp * (e * Y0 + a * J1));
}

// The same for node i of a geometry array (x1, x2, ..., |x'| at 6N, nu at 7N, 8N).
__device__ __forceinline__ zd combined_kernel(const double* geom, int N, int i, double o1, double o2, double kappa,
                                             double eta, const double* poly = fhw_bes_poly) {
    return combined_kernel_at(geom[i], geom[N + i], geom[6 * N + i], geom[7 * N + i], geom[8 * N + i], o1, o2,
                              kappa, eta, poly);
}

// The field of n_blk density blocks at once (the windows of general boundary
// data, by the combined potential; every system at the same N).  One
// workgroup per (frequency, group of FB_P observation points, group of up to
// FB_BLK windows).  The nodes go by in chunks of FB_CH: the kernel of each
// (point, node) pair of the chunk is formed once into LDS, beside the chunk's
// densities of every window; then each thread adds its (point, window) pair's
// products over its share of the chunk (S threads per pair, S a power of two:
// as many as 256 threads allow).  The shares are summed in a fixed order at
// the end.  Kernel evaluation and accumulation never hold registers at the
// same time, and a kernel value serves every window of the group.  LDS rows
// are padded by one entry so that the rows read side by side fall in
// different banks.  LIST: the F systems are an explicit list (the graded
// low-frequency nodes) written as V[r][1 + j] with V[r][0] = zero_value,
// instead of the full DFT grid.
#ifndef FHW_FB_P
#define FHW_FB_P 16      // observation points per workgroup (8: 4.2 ms, 4: 4.8 ms against 3.7 ms for 16)
#endif
#ifndef FHW_FB_WPE
#define FHW_FB_WPE 4     // waves per SIMD (register budget)
#endif
#define FB_P FHW_FB_P
#define FB_BLK 16
#define FB_CH 64
static_assert(FB_P * FB_BLK <= 256, "one (point, window) pair per thread at least");
template <bool LIST>
__global__ __launch_bounds__(256, FHW_FB_WPE) void k_field_blocks(const fhw_field_item* __restrict__ items, int F,
                                                      const zd* __restrict__ psi, int64_t psi_bstride, int n_blk,
                                                      const double* __restrict__ obs, int N_r, double zero_value,
                                                      zd* __restrict__ V, int64_t V_bstride) {
    __shared__ zd G[FB_P][FB_CH + 1];
    __shared__ zd Ps[FB_BLK][FB_CH + 1];
    __shared__ zd part[256];
    __shared__ double s_poly[FHW_BES_POLY_LEN];
    const int tid = threadIdx.x;
    for (int e = tid; e < FHW_BES_POLY_LEN; e += 256) s_poly[e] = fhw_bes_poly[e];
    __syncthreads();
    const int lane = tid & 63, wid = tid >> 6;
    const int n_rg = (N_r + FB_P - 1) / FB_P;
    const int j = blockIdx.x / n_rg;            // the point groups of one frequency are neighbours
    const int r0 = (blockIdx.x - j * n_rg) * FB_P;
    const int q0 = blockIdx.y * FB_BLK;
    const int nb = min(FB_BLK, n_blk - q0);
    const fhw_field_item it = items[j];
    const int N = it.N;
    const double* g = it.geom;
    const zd* ps = psi + it.psi_off + (int64_t)q0 * psi_bstride;
    const int pairs = FB_P * nb;                 // (point p, window u), u fastest
    int S = 1;
    while (2 * S * pairs <= 256 && S < FB_CH) S *= 2;
    const int pr = tid / S, sub = tid - pr * S;
    const int pp = pr / nb, pu = pr - pp * nb;
    zd acc = cmk(0.0, 0.0);
    for (int c0 = 0; c0 < N; c0 += FB_CH) {
        const int i = c0 + lane;
        if (i < N) {
            const double x1 = g[i], x2 = g[N + i], sp = g[6 * N + i], n1 = g[7 * N + i], n2 = g[8 * N + i];
#pragma unroll 1
            for (int p = wid; p < FB_P; p += 4) {
                const int r = r0 + p;
                G[p][lane] = r < N_r ? combined_kernel_at(x1, x2, sp, n1, n2, obs[2 * r], obs[2 * r + 1], it.kappa,
                                                          it.eta, s_poly)
                                     : cmk(0.0, 0.0);
            }
        } else {
            for (int p = wid; p < FB_P; p += 4) G[p][lane] = cmk(0.0, 0.0);
        }
        for (int e = tid; e < nb * FB_CH; e += 256) {
            const int u = e / FB_CH, ii = e - u * FB_CH;
            Ps[u][ii] = c0 + ii < N ? ps[(int64_t)u * psi_bstride + c0 + ii] : cmk(0.0, 0.0);
        }
        __syncthreads();
        if (pr < pairs) {
            for (int ii = sub; ii < FB_CH; ii += S) acc = cfma(acc, G[pp][ii], Ps[pu][ii]);
        }
        __syncthreads();
    }
    part[tid] = acc;
    __syncthreads();
    if (tid < pairs) {
        zd sum = cmk(0.0, 0.0);
        for (int k = 0; k < S; ++k) sum = cadd(sum, part[tid * S + k]);
        const int p = tid / nb, u = tid - p * nb;
        const int r = r0 + p;
        if (r < N_r) {
            const double wq = 2.0 * FHW_PI / (double)N;
            const zd val = cmk(wq * sum.re, wq * sum.im);
            if constexpr (LIST) {
                zd* Vr = V + (int64_t)(q0 + u) * V_bstride + (int64_t)r * (F + 1);
                Vr[1 + j] = val;
                if (j == 0) Vr[0] = cmk(zero_value, 0.0);
            } else {
                zd* Vr = V + (int64_t)(q0 + u) * V_bstride + (int64_t)r * 2 * F;
                if (j < F - 1) Vr[F + 1 + j] = val;
                Vr[F - 1 - j] = cconj(val);
                if (j == 0) Vr[F] = cmk(zero_value, 0.0);
            }
        }
    }
}

// V[r][0] = zero_value, V[r][1 + j] = field of item j (j < n_items): the
// field at an explicit list of systems (the graded low-frequency nodes); COMB:
// by the combined potential instead of the single layer.
template <bool COMB>
__global__ __launch_bounds__(256, 4) void k_field_list(const fhw_field_item* __restrict__ items, int n_items,
                                                    const zd* __restrict__ psi, const double* __restrict__ obs,
                                                    int N_r, double zero_value, zd* __restrict__ V) {
    const int wave = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (wave >= N_r * n_items) return;
    const int r = wave / n_items;
    const int j = wave - r * n_items;
    const fhw_field_item it = items[j];
    const int N = it.N;
    const double* x1 = it.geom;
    const double* x2 = it.geom + N;
    const double* sp = it.geom + 6 * N;
    const zd* ps = psi + it.psi_off;
    const double o1 = obs[2 * r], o2 = obs[2 * r + 1];
    zd acc = cmk(0.0, 0.0);
    for (int i = lane; i < N; i += 64) {
        zd gk;
        if constexpr (COMB) {
            gk = combined_kernel(it.geom, N, i, o1, o2, it.kappa, it.eta);
        } else {
            const double d1 = o1 - x1[i], d2 = o2 - x2[i];
            const double z = it.kappa * sqrt(d1 * d1 + d2 * d2);
            double J0, Y0;
            fhw_bessel0(z, J0, Y0);
            gk = cmk(-0.25 * Y0 * sp[i], 0.25 * J0 * sp[i]);
        }
        acc = cfma(acc, gk, ps[i]);
    }
    acc.re = wave_sum(acc.re);
    acc.im = wave_sum(acc.im);
    if (lane == 0) {
        const double wq = 2.0 * FHW_PI / (double)N;
        zd* Vr = V + (int64_t)r * (n_items + 1);
        Vr[1 + j] = cmk(wq * acc.re, wq * acc.im);
        if (j == 0) Vr[0] = cmk(zero_value, 0.0);
    }
}

__global__ void k_hankel01(const double* __restrict__ z, int64_t n, zd* __restrict__ h) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double J0, Y0, J1, Y1;
    fhw_bessel01(z[i], J0, Y0, J1, Y1);
    h[2 * i] = cmk(J0, Y0);
    h[2 * i + 1] = cmk(J1, Y1);
}

hipError_t launch_field(hipStream_t s, const fhw_field_item* d_items, int32_t F, const void* psi, const double* obs,
                        int32_t N_r, double zero_value, void* V) {
    const int64_t waves = (int64_t)N_r * F;
    if (waves <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_field, dim3((unsigned)((waves + 3) / 4)), dim3(256), 0, s, d_items, F, (const zd*)psi, obs,
                       N_r, zero_value, (zd*)V);
    return hipGetLastError();
}

hipError_t launch_field_blocks(hipStream_t s, const fhw_field_item* d_items, int32_t F, const void* psi,
                               int64_t psi_bstride, int32_t n_blk, const double* obs, int32_t N_r,
                               double zero_value, void* V, int64_t V_bstride, bool list) {
    if (N_r <= 0 || F <= 0 || n_blk <= 0) return hipSuccess;
    const int64_t blocks = (int64_t)F * ((N_r + FB_P - 1) / FB_P);
    const int64_t gy = (n_blk + FB_BLK - 1) / FB_BLK;
    if (blocks > 0x7fffffff || gy > 65535) return hipErrorInvalidValue;
    if (list)
        hipLaunchKernelGGL(k_field_blocks<true>, dim3((unsigned)blocks, (unsigned)gy), dim3(256), 0, s, d_items, F,
                           (const zd*)psi, psi_bstride, n_blk, obs, N_r, zero_value, (zd*)V, V_bstride);
    else
        hipLaunchKernelGGL(k_field_blocks<false>, dim3((unsigned)blocks, (unsigned)gy), dim3(256), 0, s, d_items, F,
                           (const zd*)psi, psi_bstride, n_blk, obs, N_r, zero_value, (zd*)V, V_bstride);
    return hipGetLastError();
}

hipError_t launch_field_list(hipStream_t s, const fhw_field_item* d_items, int32_t n_items, const void* psi,
                             const double* obs, int32_t N_r, double zero_value, void* V, bool combined) {
    const int64_t waves = (int64_t)N_r * n_items;
    if (waves <= 0) return hipSuccess;
    if (combined)
        hipLaunchKernelGGL(k_field_list<true>, dim3((unsigned)((waves + 3) / 4)), dim3(256), 0, s, d_items, n_items,
                           (const zd*)psi, obs, N_r, zero_value, (zd*)V);
    else
        hipLaunchKernelGGL(k_field_list<false>, dim3((unsigned)((waves + 3) / 4)), dim3(256), 0, s, d_items,
                           n_items, (const zd*)psi, obs, N_r, zero_value, (zd*)V);
    return hipGetLastError();
}

hipError_t launch_hankel01(hipStream_t s, const double* z, int64_t n, void* h) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_hankel01, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, z, n, (zd*)h);
    return hipGetLastError();
}
