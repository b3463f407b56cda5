// Nystrom matrix of the direct combined-field equation (eq. CFIE_direct)
//   (1/2) psi + K*psi - i eta S psi = dB/dn - i eta B
// with Kress's splitting of the logarithmic singularities of the single-layer
// kernel (i/4) H0(kappa r) and of the normal-derivative kernel
// (i kappa/4) H1(kappa r) (nu_i . d)/r (Sec. 2.3; Colton & Kress Sec. 3.5).
// Bessel/Hankel values are evaluated in registers in FP64.
#include "fhw_device.h"
#include "fhw_internal.h"

#define ASM_THREADS 256
#define AT 32   // tile edge

__device__ __forceinline__ int find_item(const int64_t* prefix, int n, int64_t blk) {
    int lo = 0, hi = n - 1;   // largest q with prefix[q] <= blk
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (prefix[mid] <= blk) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// Entry for target node t and source node s from the pair's kernel pieces:
//   K1 = L1 - i eta M1,  K2 = L2 - i eta M2,  A = |x'_s| (R_l K1 + (pi/n) K2)
// with L1 = cL n, L2 = (cY n - L1 lam) + i cJ n and n = (nu_t . d)/r.
__device__ __forceinline__ zd cfie_entry(double n_t, double cL, double cY, double cJ, double M1, double M2r,
                                         double M2i, double lam, double Rw, double wq, double eta, double sps) {
    const double L1 = cL * n_t;
    const double L2r = cY * n_t - L1 * lam;
    const double L2i = cJ * n_t;
    const double K1r = L1, K1i = -eta * M1;
    const double K2r = L2r + eta * M2i, K2i = L2i - eta * M2r;
    return cmk(sps * (Rw * K1r + wq * K2r), sps * (Rw * K1i + wq * K2i));
}

// COMB: the combined potential's matrix (1/2) phi + K phi - i eta S phi, K
// the double layer: the normal factor of entry (i, j) is nu_j . (x_i - x_j)/r
// (the source's) where the direct equation's adjoint kernel has nu_i . (x_j -
// x_i)/r (the target's); everything else, diagonal limits included, is shared.
// One workgroup per 32x32 tile (I, J), I >= J, of one matrix (column-major).
// Each thread takes pairs (i, j) = (i0 + tid%32, j0 + tid/32 + 8k), k < 4.
// The Bessel values of |x_i - x_j| serve A(i, j) (written directly, lanes
// along i) and A(j, i) (staged in LDS, then written with lanes along j).
// Diagonal tiles take i > j in the pair loop, mirror the strict part and
// write their diagonal entries after it (so that no other tile evaluates the
// diagonal limits).  Tiles with J = 0 also write the RHS.
template <bool COMB, bool NT>
__global__ __launch_bounds__(ASM_THREADS, 4) void k_assemble(const fhw_assemble_item* __restrict__ items,
                                                          const int64_t* __restrict__ prefix, int n_items,
                                                          double p1, double p2, zd* __restrict__ A,
                                                          zf* __restrict__ A32, zd* __restrict__ g) {
    __shared__ zd mirror[AT][AT + 1];
    const int q = find_item(prefix, n_items, blockIdx.x);
    const fhw_assemble_item it = items[q];
    const int N = it.N;
    const int n = N >> 1;
    // lower-triangular tile index t -> (I, J), I >= J
    const int t = (int)(blockIdx.x - prefix[q]);
    int I = (int)((sqrtf(8.0f * (float)t + 1.0f) - 1.0f) * 0.5f);
    while ((I + 1) * (I + 2) / 2 <= t) ++I;
    while (I * (I + 1) / 2 > t) --I;
    const int J = t - I * (I + 1) / 2;
    const int i0 = I * AT, j0 = J * AT;
    const double* x1 = it.geom;
    const double* x2 = it.geom + N;
    const double* ddx1 = it.geom + 4 * N;
    const double* ddx2 = it.geom + 5 * N;
    const double* sp = it.geom + 6 * N;
    const double* nu1 = it.geom + 7 * N;
    const double* nu2 = it.geom + 8 * N;
    const double kappa = it.kappa, eta = it.eta;
    const double inv4pi = 1.0 / (4.0 * FHW_PI);
    const double wq = FHW_PI * fhw_rcp((double)n);
    zd* Aq = A + it.a_off;
    zf* A32q = A32 ? A32 + it.a_off : nullptr;

    const int il = threadIdx.x & (AT - 1);
    const int jg = threadIdx.x >> 5;
    const int i = i0 + il;
    const bool iok = i < N;
    // The tile's source-node data and the Kress tables at its 2 AT - 1 index
    // differences l = (i - j) mod N and N - l, staged once in LDS.
    __shared__ double sj[5][AT];
    __shared__ double st[4][2 * AT];
    if (threadIdx.x < AT) {
        const int j = j0 + threadIdx.x;
        const bool ok = j < N;
        sj[0][threadIdx.x] = ok ? x1[j] : 0.0;
        sj[1][threadIdx.x] = ok ? x2[j] : 0.0;
        sj[2][threadIdx.x] = ok ? sp[j] : 0.0;
        sj[3][threadIdx.x] = ok ? nu1[j] : 0.0;
        sj[4][threadIdx.x] = ok ? nu2[j] : 0.0;
    } else if (threadIdx.x < 3 * AT - 1) {
        const int e = threadIdx.x - AT;   // l = i0 - j0 - (AT - 1) + e (mod N), in [-(AT - 1), N) as i0 >= j0
        const int l0 = i0 - j0 - (AT - 1) + e;
        const int l = l0 < 0 ? l0 + N : l0;
        const int lm = (l == 0) ? 0 : N - l;
        st[0][e] = it.logtab[l];
        st[1][e] = it.R[l];
        st[2][e] = it.logtab[lm];
        st[3][e] = it.R[lm];
    }
    // the Bessel interval polynomials too (assembly 7.3 -> 6.5 ms per FP32-mode step)
    __shared__ double s_poly[FHW_BES_POLY_LEN];
    for (int e = threadIdx.x; e < FHW_BES_POLY_LEN; e += ASM_THREADS) s_poly[e] = fhw_bes_poly[e];
    double xi1 = 0, xi2 = 0, ni1 = 0, ni2 = 0, spi = 0;
    if (iok) { xi1 = x1[i]; xi2 = x2[i]; ni1 = nu1[i]; ni2 = nu2[i]; spi = sp[i]; }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < AT / 8; ++k) {
        const int jl = jg + 8 * k;
        const int j = j0 + jl;
        if (!iok || j >= N || (I == J && i <= j)) continue;
        const double spj = sj[2][jl];
        const int dd = il - jl + AT - 1;   // index of l = (i - j) mod N in st
        const double d1 = sj[0][jl] - xi1, d2 = sj[1][jl] - xi2;   // d = x_j - x_i
        const double r2 = d1 * d1 + d2 * d2;
        const double ir = fhw_rsqrt(r2);   // 1 / r
        const double r = r2 * ir;
        double J0, Y0, J1, Y1;
        fhw_bessel01(kappa * r, J0, Y0, J1, Y1, s_poly);
        const double lam = st[0][dd];
        const double M1 = -J0 * inv4pi;
        const double M2r = -0.25 * Y0 - M1 * lam;
        const double M2i = 0.25 * J0;
        const double cL = -kappa * inv4pi * J1;
        const double cY = -0.25 * kappa * Y1;
        const double cJ = 0.25 * kappa * J1;
        const double n_i = (ni1 * d1 + ni2 * d2) * ir;          // target i: nu_i . (x_j - x_i) / r
        const double n_j = -(sj[3][jl] * d1 + sj[4][jl] * d2) * ir;   // target j: nu_j . (x_i - x_j) / r
        const zd e_ij = cfie_entry(COMB ? n_j : n_i, cL, cY, cJ, M1, M2r, M2i, lam, st[1][dd], wq, eta, spj);
        const zd e_ji = cfie_entry(COMB ? n_i : n_j, cL, cY, cJ, M1, M2r, M2i, st[2][dd], st[3][dd], wq, eta, spi);
        st_maybe_stream<NT>(&Aq[(int64_t)j * N + i], e_ij);
        if (A32q) st_maybe_stream<NT>(&A32q[(int64_t)j * N + i], cmk((float)e_ij.re, (float)e_ij.im));
        mirror[jl][il] = e_ji;
    }
    if (I == J && iok && (il & 7) == jg) {
        // diagonal entry (i, i): the kernels' limits as x_j -> x_i (one thread per row)
        const double M2r = -(0.57721566490153286061 + log(0.5 * kappa * spi)) * (0.5 / FHW_PI);
        const double M2i = 0.25;
        const double L2r = (ni1 * ddx1[i] + ni2 * ddx2[i]) * inv4pi * fhw_rcp(spi * spi);
        const double K1r = 0.0, K1i = eta * inv4pi;
        const double K2r = L2r + eta * M2i, K2i = -eta * M2r;
        const double Rw = it.R[0];
        const zd e = cmk(spi * (Rw * K1r + wq * K2r) + 0.5, spi * (Rw * K1i + wq * K2i));
        st_maybe_stream<NT>(&Aq[(int64_t)i * N + i], e);
        if (A32q) st_maybe_stream<NT>(&A32q[(int64_t)i * N + i], cmk((float)e.re, (float)e.im));
    }
    if (J == 0 && jg == 0 && iok) {
        // g_i = i (kappa p.nu_i - eta) exp(i kappa p.x_i)
        const double alpha = kappa * (p1 * ni1 + p2 * ni2) - eta;
        double sn, cs;
        sincos(kappa * (p1 * xi1 + p2 * xi2), &sn, &cs);
        g[it.g_off + i] = cmk(-alpha * sn, alpha * cs);
    }
    __syncthreads();
    // mirrored tile: entry (row j0 + jl, column i0 + il) at (i0 + il) * N + j0 + jl; lanes along jl
    const int jl2 = threadIdx.x & (AT - 1);
    const int ig = threadIdx.x >> 5;
    const int jrow = j0 + jl2;
#pragma unroll
    for (int k = 0; k < AT / 8; ++k) {
        const int il2 = ig + 8 * k;
        const int icol = i0 + il2;
        // diagonal tiles computed pairs i > j only: mirror the strict part
        if (jrow < N && icol < N && (I != J || icol > jrow)) {
            const zd v = mirror[jl2][il2];
            st_maybe_stream<NT>(&Aq[(int64_t)icol * N + jrow], v);
            if (A32q) st_maybe_stream<NT>(&A32q[(int64_t)icol * N + jrow], cmk((float)v.re, (float)v.im));
        }
    }
}

hipError_t launch_assemble_blocks(hipStream_t s, const fhw_assemble_item* d_items, const int64_t* d_prefix,
                                  int32_t n_items, int64_t total_blocks, double p1, double p2, void* A,
                                  void* A32, void* g, bool combined) {
    if (total_blocks <= 0) return hipSuccess;
    // stores with the nontemporal hint once the matrices (32 KB of FP64
    // entries per tile pair) outgrow the 256 MB last-level cache
#define FHW_ASM(CB, NTB)                                                                                     \
    hipLaunchKernelGGL((k_assemble<CB, NTB>), dim3((unsigned)total_blocks), dim3(ASM_THREADS), 0, s, d_items, \
                       d_prefix, n_items, p1, p2, (zd*)A, (zf*)A32, (zd*)g)
    const bool nt = total_blocks > 8192;
    if (combined) {
        if (nt) FHW_ASM(true, true);
        else FHW_ASM(true, false);
    } else {
        if (nt) FHW_ASM(false, true);
        else FHW_ASM(false, false);
    }
#undef FHW_ASM
    return hipGetLastError();
}

int64_t assemble_blocks_for(int32_t N) {
    const int64_t T = (N + AT - 1) / AT;
    return T * (T + 1) / 2;
}

// Boundary data g = dB/dnu - i eta B of eq. CFIE_direct for a group of
// incidences at every node of each frequency (one workgroup per frequency and
// incidence):
//   plane wave   B = exp(i kappa p.x):  g = i (kappa p.nu - eta) exp(i kappa p.x)
//   point source B = (i/4) H0(kappa rho), rho = |x - r0|, r0 outside the curve:
//                dB/dnu = -(i kappa / 4) H1(kappa rho) nu.(x - r0) / rho
__global__ __launch_bounds__(ASM_THREADS) void k_rhs(const fhw_assemble_item* __restrict__ items, fhw_rhs_group rg,
                                                     int64_t sg, zd* __restrict__ g) {
    const fhw_assemble_item it = items[blockIdx.x];
    const int q = blockIdx.y;   // incidence of the group
    const int kind = rg.kind[q];
    const double v0 = rg.v[q][0], v1 = rg.v[q][1];
    g += (int64_t)q * sg;
    const int N = it.N;
    const double kappa = it.kappa, eta = it.eta;
    const double* x1 = it.geom;
    const double* x2 = it.geom + N;
    const double* nu1 = it.geom + 7 * N;
    const double* nu2 = it.geom + 8 * N;
    for (int i = threadIdx.x; i < N; i += ASM_THREADS) {
        zd gi;
        if (kind == FHW_INC_PLANE) {
            const double alpha = kappa * (v0 * nu1[i] + v1 * nu2[i]) - eta;
            double sn, cs;
            sincos(kappa * (v0 * x1[i] + v1 * x2[i]), &sn, &cs);
            gi = cmk(-alpha * sn, alpha * cs);
        } else {
            const double d1 = x1[i] - v0, d2 = x2[i] - v1;
            const double rho = sqrt(d1 * d1 + d2 * d2);
            double J0, Y0, J1, Y1;
            fhw_bessel01(kappa * rho, J0, Y0, J1, Y1);
            const double cn = (nu1[i] * d1 + nu2[i] * d2) / rho;
            const double Br = -0.25 * Y0, Bi = 0.25 * J0;                                 // (i/4) H0
            const double dBr = 0.25 * kappa * cn * Y1, dBi = -0.25 * kappa * cn * J1;   // -(i kappa/4) H1 cn
            gi = cmk(dBr + eta * Bi, dBi - eta * Br);
        }
        g[it.g_off + i] = gi;
    }
}

hipError_t launch_rhs(hipStream_t s, const fhw_assemble_item* d_items, int32_t n_items, const fhw_rhs_group& rg,
                      int64_t sg, void* g) {
    if (n_items <= 0 || rg.n <= 0) return hipSuccess;
    if (rg.n > FHW_INC_GROUP) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_rhs, dim3(n_items, rg.n), dim3(ASM_THREADS), 0, s, d_items, rg, sg, (zd*)g);
    return hipGetLastError();
}
