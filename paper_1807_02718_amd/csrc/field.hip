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
        fhw_bessel0(z, J0, Y0);
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

// Kernel of the combined potential at observation point (o1, o2) for node i:
//   |x'_i| [ (i kappa/4) H1(kappa rho) nu_i . (r - x_i)/rho + (eta/4) H0(kappa rho) ]
__device__ __forceinline__ zd combined_kernel(const double* geom, int N, int i, double o1, double o2, double kappa,
                                             double eta) {
    const double d1 = o1 - geom[i], d2 = o2 - geom[N + i];
    const double rho = sqrt(d1 * d1 + d2 * d2);
    double J0, Y0, J1, Y1;
    fhw_bessel01(kappa * rho, J0, Y0, J1, Y1);
    const double cn = (geom[7 * N + i] * d1 + geom[8 * N + i] * d2) / rho;
    const double sp = geom[6 * N + i];
    const double a = 0.25 * kappa * cn, e = 0.25 * eta;
    return cmk(sp * (e * J0 - a * Y1), sp * (e * Y0 + a * J1));
}

// The field of n_blk density blocks at once (the windows of general boundary
// data, by the combined potential): one wave per (point, frequency) as in
// k_field; the kernel of a node is formed once and applied to up to FB_BLK
// blocks.
#define FB_BLK 8
__global__ __launch_bounds__(256, 4) void k_field_blocks(const fhw_field_item* __restrict__ items, int F,
                                                      const zd* __restrict__ psi, int64_t psi_bstride, int n_blk,
                                                      const double* __restrict__ obs, int N_r, double zero_value,
                                                      zd* __restrict__ V, int64_t V_bstride) {
    const int wave = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (wave >= N_r * F) return;
    const int r = wave / F;
    const int j = wave - r * F;
    const fhw_field_item it = items[j];
    const int N = it.N;
    const double o1 = obs[2 * r], o2 = obs[2 * r + 1];
    const double wq = 2.0 * FHW_PI / (double)N;
    for (int q0 = blockIdx.y * FB_BLK; q0 < n_blk; q0 += gridDim.y * FB_BLK) {
        const int nb = min(FB_BLK, n_blk - q0);
        const zd* ps = psi + it.psi_off + (int64_t)q0 * psi_bstride;
        zd acc[FB_BLK];
#pragma unroll
        for (int u = 0; u < FB_BLK; ++u) acc[u] = cmk(0.0, 0.0);
        for (int i = lane; i < N; i += 64) {
            const zd gk = combined_kernel(it.geom, N, i, o1, o2, it.kappa, it.eta);
#pragma unroll
            for (int u = 0; u < FB_BLK; ++u)
                if (u < nb) acc[u] = cfma(acc[u], gk, ps[(int64_t)u * psi_bstride + i]);
        }
#pragma unroll
        for (int u = 0; u < FB_BLK; ++u) {
            if (u >= nb) break;
            const double re = wave_sum(acc[u].re), im = wave_sum(acc[u].im);
            if (lane == 0) {
                const zd val = cmk(wq * re, wq * im);
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
                               double zero_value, void* V, int64_t V_bstride) {
    const int64_t waves = (int64_t)N_r * F;
    if (waves <= 0 || n_blk <= 0) return hipSuccess;
    const int gy = (n_blk + FB_BLK - 1) / FB_BLK;
    hipLaunchKernelGGL(k_field_blocks, dim3((unsigned)((waves + 3) / 4), gy), dim3(256), 0, s, d_items, F,
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
