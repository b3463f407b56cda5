// Device helpers shared by the gfx950 kernels: complex arithmetic and the
// in-register FP64 Bessel/Hankel evaluation.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "bessel_tables.h"

#define FHW_PI 3.14159265358979323846
#define FHW_INV_SQRT2 0.70710678118654752440
#define FHW_SQRT_2_OVER_PI 0.79788456080286535588   // sqrt(2 / pi)

template <typename T>
struct __align__(2 * sizeof(T)) cpx {
    T re, im;
};
typedef cpx<double> zd;
typedef cpx<float> zf;

template <typename T>
__device__ __forceinline__ cpx<T> cmk(T r, T i) { cpx<T> z; z.re = r; z.im = i; return z; }
template <typename T>
__device__ __forceinline__ cpx<T> cadd(cpx<T> a, cpx<T> b) { return cmk(a.re + b.re, a.im + b.im); }
template <typename T>
__device__ __forceinline__ cpx<T> csub(cpx<T> a, cpx<T> b) { return cmk(a.re - b.re, a.im - b.im); }
template <typename T>
__device__ __forceinline__ cpx<T> cmul(cpx<T> a, cpx<T> b) {
    return cmk(a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re);
}
// a - b*c
template <typename T>
__device__ __forceinline__ cpx<T> cfms(cpx<T> a, cpx<T> b, cpx<T> c) {
    return cmk(a.re - b.re * c.re + b.im * c.im, a.im - b.re * c.im - b.im * c.re);
}
// a + b*c
template <typename T>
__device__ __forceinline__ cpx<T> cfma(cpx<T> a, cpx<T> b, cpx<T> c) {
    return cmk(a.re + b.re * c.re - b.im * c.im, a.im + b.re * c.im + b.im * c.re);
}
template <typename T>
__device__ __forceinline__ cpx<T> cconj(cpx<T> a) { return cmk(a.re, -a.im); }
template <typename T>
__device__ __forceinline__ T cabs1(cpx<T> a) { return fabs(a.re) + fabs(a.im); }
// 1/a by scaling (Smith-free: |a| is O(1) for pivots of these systems, but
// scale anyway to avoid overflow/underflow in |a|^2)
template <typename T>
__device__ __forceinline__ cpx<T> crcp(cpx<T> a) {
    T s = fmax(fabs(a.re), fabs(a.im));
    T ar = a.re / s, ai = a.im / s;
    T d = s * (ar * ar + ai * ai);
    return cmk(ar / d, -ai / d);
}

// Streaming accesses with the nontemporal hint, for data touched once per
// kernel (a matrix read once by a residual, written once by the assembly):
// one 16- or 8-byte access each, as the plain ones.
typedef double fhw_v2d __attribute__((ext_vector_type(2)));
typedef float fhw_v2f __attribute__((ext_vector_type(2)));
__device__ __forceinline__ zd ld_stream(const zd* p) {
    const fhw_v2d t = __builtin_nontemporal_load((const fhw_v2d*)p);
    return cmk(t.x, t.y);
}
__device__ __forceinline__ zf ld_stream(const zf* p) {
    const fhw_v2f t = __builtin_nontemporal_load((const fhw_v2f*)p);
    return cmk(t.x, t.y);
}
__device__ __forceinline__ void st_stream(zd* p, zd v) {
    const fhw_v2d t = {v.re, v.im};
    __builtin_nontemporal_store(t, (fhw_v2d*)p);
}
__device__ __forceinline__ void st_stream(zf* p, zf v) {
    const fhw_v2f t = {v.re, v.im};
    __builtin_nontemporal_store(t, (fhw_v2f*)p);
}
// The hint only where the data cannot stay cached anyway (large batches):
// a repeated solve of one system finds its matrix in the last-level cache.
template <bool STREAM, typename V>
__device__ __forceinline__ V ld_maybe_stream(const V* p) {
    if constexpr (STREAM) return ld_stream(p);
    else return *p;
}
template <bool STREAM, typename V>
__device__ __forceinline__ void st_maybe_stream(V* p, V v) {
    if constexpr (STREAM) st_stream(p, v);
    else *p = v;
}

// ---------------------------------------------------------------------------
// J0, Y0, J1, Y1 for z > 0 in FP64 (tables and regions in bessel_tables.h)
// ---------------------------------------------------------------------------
// acc * y + c with the coefficient c as a scalar (SGPR) operand of the
// three-operand FMA: the compiler's two-operand form needs c in a vector
// register, which costs two extra vector moves per term for FP64 constants.
__device__ __forceinline__ double fhw_fma_sc(double acc, double y, double c) {
    double r;
    asm("v_fma_f64 %0, %1, %2, %3" : "=v"(r) : "v"(acc), "v"(y), "s"(c));
    return r;
}

// Polynomial with compile-time coefficients (fully unrolled)
__device__ __forceinline__ double fhw_horner(const double* c, int n, double y) {
    double acc = c[n - 1];
#pragma unroll
    for (int k = n - 2; k >= 0; --k) acc = fhw_fma_sc(acc, y, c[k]);
    return acc;
}

// Polynomial whose coefficients each lane reads itself (per-lane interval)
__device__ __forceinline__ double fhw_horner_v(const double* c, int n, double u) {
    double acc = c[n - 1];
#pragma unroll
    for (int k = n - 2; k >= 0; --k) acc = fma(acc, u, c[k]);
    return acc;
}

// 1/sqrt(x), x > 0 finite: the hardware estimate refined by two Newton steps
// y <- y (3 - x y^2) / 2 (each squares the relative error).
__device__ __forceinline__ double fhw_rsqrt(double x) {
    double y = __builtin_amdgcn_rsq(x);
    const double h = 0.5 * x;
    y = y * fma(-h * y, y, 1.5);
    y = y * fma(-h * y, y, 1.5);
    return y;
}

// sin and cos of w = z - pi/4 for z >= 0 (the Hankel phase): Cody and Waite's
// additive reduction w = k pi/2 + r, written as r = z - m pi/4 with m = 2k + 1
// odd, pi/4 split in two doubles (the leading one pi/4 rounded, the second the
// rounded remainder; with fused products the reduction error stays near one
// ulp of r up to z ~ 1e15), then the Taylor series of sin r and cos r on
// |r| <= pi/4 through r^17 and r^16 (first omitted terms below 1e-17) and the
// quadrant k mod 4.  About half the instructions of the general sincos.
#define FHW_PIO4_HI 0x1.921fb54442d18p-1
#define FHW_PIO4_LO 0x1.1a62633145c07p-55
#define FHW_2_OVER_PI 0x1.45f306dc9c883p-1
__device__ __forceinline__ void fhw_sincos_shift(double z, double& sw, double& cw) {
    const double k = __builtin_rint(fma(z, FHW_2_OVER_PI, -0.5));
    const double m = fma(2.0, k, 1.0);
    double r = fma(-m, FHW_PIO4_HI, z);
    r = fma(-m, FHW_PIO4_LO, r);
    const double x = r * r;
    // sin r = r + r x (-1/3! + x (1/5! - ...)),  cos r = 1 - x/2 + x^2 (1/4! - x (1/6! - ...))
    double ps = 0x1.952c77030ad4ap-49;                 //  1/17!
    ps = fhw_fma_sc(ps, x, -0x1.ae7f3e733b81fp-41);   // -1/15!
    ps = fhw_fma_sc(ps, x, 0x1.6124613a86d09p-33);    //  1/13!
    ps = fhw_fma_sc(ps, x, -0x1.ae64567f544e4p-26);   // -1/11!
    ps = fhw_fma_sc(ps, x, 0x1.71de3a556c734p-19);    //  1/9!
    ps = fhw_fma_sc(ps, x, -0x1.a01a01a01a01ap-13);   // -1/7!
    ps = fhw_fma_sc(ps, x, 0x1.1111111111111p-7);     //  1/5!
    ps = fhw_fma_sc(ps, x, -0x1.5555555555555p-3);    // -1/3!
    double pc = 0x1.ae7f3e733b81fp-45;                 //  1/16!
    pc = fhw_fma_sc(pc, x, -0x1.93974a8c07c9dp-37);   // -1/14!
    pc = fhw_fma_sc(pc, x, 0x1.1eed8eff8d898p-29);    //  1/12!
    pc = fhw_fma_sc(pc, x, -0x1.27e4fb7789f5cp-22);   // -1/10!
    pc = fhw_fma_sc(pc, x, 0x1.a01a01a01a01ap-16);    //  1/8!
    pc = fhw_fma_sc(pc, x, -0x1.6c16c16c16c17p-10);   // -1/6!
    pc = fhw_fma_sc(pc, x, 0x1.5555555555555p-5);     //  1/4!
    const double sr = fma(r * x, ps, r);
    const double cr = fma(x * x, pc, fma(-0.5, x, 1.0));
    // (sin, cos)(k pi/2 + r): k odd swaps them (cos, -sin); k = 2, 3 mod 4 negates both
    const int q = (int)k;
    const bool odd = (q & 1) != 0;
    double a = odd ? cr : sr;
    double b = odd ? -sr : cr;
    if (q & 2) { a = -a; b = -b; }
    sw = a;
    cw = b;
}

// 1/x, x finite and nonzero: the hardware estimate refined by two Newton
// steps y <- y + y (1 - x y) (each squares the relative error).
__device__ __forceinline__ double fhw_rcp(double x) {
    double y = __builtin_amdgcn_rcp(x);
    y = fma(y, fma(-x, y, 1.0), y);
    y = fma(y, fma(-x, y, 1.0), y);
    return y;
}

// Auxiliary P_nu, Q_nu (H_nu = sqrt(2/(pi z)) (P + iQ) e^{i(z - nu pi/2 - pi/4)})
// for z > FHW_BES_Z_SERIES, given iz = 1/z.  want1: also nu = 1.  poly: the
// interval polynomials fhw_bes_poly (Chebyshev fits in 1/z, in power form in
// the interval's u), or a copy of them in LDS (each lane gathers its own
// interval's coefficients; from LDS the gathers are short).
#define FHW_BES_POLY_LEN (FHW_BES_N_INTERVALS * FHW_BES_INTERVAL_LEN)
template <bool want1>
__device__ __forceinline__ void fhw_bes_pq(double z, double iz, double& P0, double& Q0, double& P1, double& Q1,
                                           const double* poly) {
    if (z >= FHW_BES_Z_ASYM) {
        double y = iz * iz;
        P0 = fhw_horner(fhw_bes_asym_p0, FHW_BES_N_ASYM, y);
        Q0 = iz * fhw_horner(fhw_bes_asym_q0, FHW_BES_N_ASYM, y);
        if (want1) {
            P1 = fhw_horner(fhw_bes_asym_p1, FHW_BES_N_ASYM, y);
            Q1 = iz * fhw_horner(fhw_bes_asym_q1, FHW_BES_N_ASYM, y);
        }
        return;
    }
    int iv = 0;
#pragma unroll
    for (int q = 1; q < FHW_BES_N_INTERVALS; ++q) iv += (z >= fhw_bes_breaks[q]) ? 1 : 0;
    // u = (2/z - (xa + xb)) / (xb - xa) on [xa, xb] = [1/break_{iv+1}, 1/break_iv],
    // with the interval's shift and scale read ahead of its coefficients
    const double* c = poly + iv * FHW_BES_INTERVAL_LEN;
    const double u = (2.0 * iz - c[0]) * c[1];
    c += 2;
    P0 = fhw_horner_v(c, FHW_BES_N_POLY, u);
    Q0 = fhw_horner_v(c + FHW_BES_N_POLY, FHW_BES_N_POLY, u);
    if (want1) {
        P1 = fhw_horner_v(c + 2 * FHW_BES_N_POLY, FHW_BES_N_POLY, u);
        Q1 = fhw_horner_v(c + 3 * FHW_BES_N_POLY, FHW_BES_N_POLY, u);
    }
}

// All four of J0, Y0, J1, Y1 at z > 0.
__device__ __forceinline__ void fhw_bessel01(double z, double& J0, double& Y0, double& J1, double& Y1,
                                             const double* poly = fhw_bes_poly) {
    if (z <= FHW_BES_Z_SERIES) {
        double y = 0.25 * z * z;
        double j0 = fhw_horner(fhw_bes_series_j0, FHW_BES_N_SERIES, y);
        double s0 = fhw_horner(fhw_bes_series_s0, FHW_BES_N_SERIES, y);
        double j1 = 0.5 * z * fhw_horner(fhw_bes_series_j1, FHW_BES_N_SERIES, y);
        double s1 = fhw_horner(fhw_bes_series_s1, FHW_BES_N_SERIES, y);
        double lg = log(0.5 * z);
        J0 = j0;
        Y0 = (2.0 / FHW_PI) * ((lg + fhw_bes_euler_gamma) * j0 + s0);
        J1 = j1;
        Y1 = (2.0 / FHW_PI) * (lg * j1 - fhw_rcp(z)) - (z * (0.5 / FHW_PI)) * s1;
        return;
    }
    double P0, Q0, P1, Q1;
    const double rz = fhw_rsqrt(z);
    fhw_bes_pq<true>(z, rz * rz, P0, Q0, P1, Q1, poly);
    double s0, c0;
    fhw_sincos_shift(z, s0, c0);                                         // sin, cos of z - pi/4
    double c1 = s0, s1 = -c0;                                            // cos, sin of z - 3pi/4
    double amp = FHW_SQRT_2_OVER_PI * rz;                                // sqrt(2 / (pi z))
    J0 = amp * (P0 * c0 - Q0 * s0);
    Y0 = amp * (P0 * s0 + Q0 * c0);
    J1 = amp * (P1 * c1 - Q1 * s1);
    Y1 = amp * (P1 * s1 + Q1 * c1);
}

// J0, Y0 only (H0 = J0 + i Y0).
__device__ __forceinline__ void fhw_bessel0(double z, double& J0, double& Y0, const double* poly = fhw_bes_poly) {
    if (z <= FHW_BES_Z_SERIES) {
        double y = 0.25 * z * z;
        double j0 = fhw_horner(fhw_bes_series_j0, FHW_BES_N_SERIES, y);
        double s0 = fhw_horner(fhw_bes_series_s0, FHW_BES_N_SERIES, y);
        J0 = j0;
        Y0 = (2.0 / FHW_PI) * ((log(0.5 * z) + fhw_bes_euler_gamma) * j0 + s0);
        return;
    }
    double P0, Q0, P1, Q1;
    const double rz = fhw_rsqrt(z);
    fhw_bes_pq<false>(z, rz * rz, P0, Q0, P1, Q1, poly);
    double s0, c0;
    fhw_sincos_shift(z, s0, c0);
    double amp = FHW_SQRT_2_OVER_PI * rz;
    J0 = amp * (P0 * c0 - Q0 * s0);
    Y0 = amp * (P0 * s0 + Q0 * c0);
}

// ---------------------------------------------------------------------------
// Wave-level reductions (64 lanes), fixed order => deterministic
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}
