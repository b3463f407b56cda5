// Nystrom matrix of the direct combined-field equation (eq. CFIE_direct)
//   (1/2) psi + K*psi - i eta S psi = dB/dn - i eta B
// with Kress's splitting of the logarithmic singularities of the single-layer
// kernel (i/4) H0(kappa r) and of the normal-derivative kernel
// (i kappa/4) H1(kappa r) (nu_i . d)/r (Sec. 2.3; Colton & Kress Sec. 3.5).
// Bessel/Hankel values are evaluated in registers in FP64.
#include "fhw_device.h"
#include "fhw_internal.h"

#define ASM_THREADS 256
#define ASM_PER_THREAD 8
#define ASM_PER_BLOCK (ASM_THREADS * ASM_PER_THREAD)

__device__ __forceinline__ int find_item(const int64_t* prefix, int n, int64_t blk) {
    int lo = 0, hi = n - 1;   // largest q with prefix[q] <= blk
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (prefix[mid] <= blk) lo = mid; else hi = mid - 1;
    }
    return lo;
}

__global__ __launch_bounds__(ASM_THREADS) void k_assemble(const fhw_assemble_item* __restrict__ items,
                                                          const int64_t* __restrict__ prefix, int n_items,
                                                          double p1, double p2, zd* __restrict__ A,
                                                          zf* __restrict__ A32, zd* __restrict__ g) {
    const int q = find_item(prefix, n_items, blockIdx.x);
    const fhw_assemble_item it = items[q];
    const int N = it.N;
    const int n = N >> 1;
    const int64_t NN = (int64_t)N * N;
    const int64_t base = (int64_t)(blockIdx.x - prefix[q]) * ASM_PER_BLOCK;
    const double* x1 = it.geom;
    const double* x2 = it.geom + N;
    const double* ddx1 = it.geom + 4 * N;
    const double* ddx2 = it.geom + 5 * N;
    const double* sp = it.geom + 6 * N;
    const double* nu1 = it.geom + 7 * N;
    const double* nu2 = it.geom + 8 * N;
    const double kappa = it.kappa, eta = it.eta;
    const double inv4pi = 1.0 / (4.0 * FHW_PI);
    const double wq = FHW_PI / (double)n;
    zd* Aq = A + it.a_off;
    zf* A32q = A32 ? A32 + it.a_off : nullptr;

    for (int s = 0; s < ASM_PER_THREAD; ++s) {
        const int64_t e = base + (int64_t)s * ASM_THREADS + threadIdx.x;
        if (e >= NN) break;
        // column-major: e = j*N + i (consecutive threads, consecutive rows i)
        const int j = (int)(e / N);
        const int i = (int)(e - (int64_t)j * N);
        const int l = (i - j + N) % N;
        const double Rw = it.R[l];
        const double spj = sp[j];
        double K1r, K1i, K2r, K2i;
        if (i != j) {
            const double d1 = x1[j] - x1[i], d2 = x2[j] - x2[i];
            const double r = sqrt(d1 * d1 + d2 * d2);
            const double z = kappa * r;
            double J0, Y0, J1, Y1;
            fhw_bessel01(z, J0, Y0, J1, Y1);
            const double lam = it.logtab[l];
            const double nud_r = (nu1[i] * d1 + nu2[i] * d2) / r;
            // M = (i/4)(J0 + i Y0), M1 = -J0/(4pi), M2 = M - M1 lam
            const double M1 = -J0 * inv4pi;
            const double M2r = -0.25 * Y0 - M1 * lam;
            const double M2i = 0.25 * J0;
            // L = (i kappa/4)(J1 + i Y1) nud/r, L1 = -(kappa/4pi) J1 nud/r, L2 = L - L1 lam
            const double L1 = -kappa * inv4pi * J1 * nud_r;
            const double L2r = -0.25 * kappa * Y1 * nud_r - L1 * lam;
            const double L2i = 0.25 * kappa * J1 * nud_r;
            K1r = L1;
            K1i = -eta * M1;
            K2r = L2r + eta * M2i;
            K2i = L2i - eta * M2r;
        } else {
            const double M2r = -(0.57721566490153286061 + log(0.5 * kappa * spj)) / (2.0 * FHW_PI);
            const double M2i = 0.25;
            const double L2r = (nu1[i] * ddx1[i] + nu2[i] * ddx2[i]) * inv4pi / (spj * spj);
            K1r = 0.0;
            K1i = eta * inv4pi;
            K2r = L2r + eta * M2i;
            K2i = -eta * M2r;
        }
        double ar = spj * (Rw * K1r + wq * K2r);
        double ai = spj * (Rw * K1i + wq * K2i);
        if (i == j) ar += 0.5;
        Aq[e] = cmk(ar, ai);
        if (A32q) A32q[e] = cmk((float)ar, (float)ai);
        if (j == 0) {
            // g_i = i (kappa p.nu_i - eta) exp(i kappa p.x_i)
            const double alpha = kappa * (p1 * nu1[i] + p2 * nu2[i]) - eta;
            double sn, cs;
            sincos(kappa * (p1 * x1[i] + p2 * x2[i]), &sn, &cs);
            g[it.g_off + i] = cmk(-alpha * sn, alpha * cs);
        }
    }
}

hipError_t launch_assemble_blocks(hipStream_t s, const fhw_assemble_item* d_items, const int64_t* d_prefix,
                                  int32_t n_items, int64_t total_blocks, double p1, double p2, void* A,
                                  void* A32, void* g) {
    if (total_blocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_assemble, dim3((unsigned)total_blocks), dim3(ASM_THREADS), 0, s, d_items, d_prefix,
                       n_items, p1, p2, (zd*)A, (zf*)A32, (zd*)g);
    return hipGetLastError();
}

int64_t assemble_blocks_for(int32_t N) {
    int64_t NN = (int64_t)N * N;
    return (NN + ASM_PER_BLOCK - 1) / ASM_PER_BLOCK;
}
