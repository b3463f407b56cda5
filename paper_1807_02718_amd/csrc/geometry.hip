// Boundary nodes and Kress log-quadrature weights (Sec. 2.3: Nystrom method of
// Colton & Kress, Sec. 3.5, on N = 2n equispaced parameter nodes).
#include "fhw_device.h"
#include "fhw_internal.h"

// One thread per node.  Angles d*t_i are reduced exactly as integers
// (d*i mod N) before sincospi, so node values do not depend on rounding of
// 2*pi*i/N.
__global__ void k_geometry(const double* __restrict__ curve, int degree, int N, double* __restrict__ g) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const int D1 = degree + 1;
    const double* cx = curve;
    const double* sx = curve + D1;
    const double* cy = curve + 2 * D1;
    const double* sy = curve + 3 * D1;
    double x1 = 0, x2 = 0, d1 = 0, d2 = 0, e1 = 0, e2 = 0;
    for (int d = 0; d <= degree; ++d) {
        long long q = ((long long)d * i) % N;
        double s, c;
        sincospi(2.0 * (double)q / (double)N, &s, &c);
        double dd = (double)d;
        x1 += cx[d] * c + sx[d] * s;
        x2 += cy[d] * c + sy[d] * s;
        d1 += dd * (sx[d] * c - cx[d] * s);
        d2 += dd * (sy[d] * c - cy[d] * s);
        e1 -= dd * dd * (cx[d] * c + sx[d] * s);
        e2 -= dd * dd * (cy[d] * c + sy[d] * s);
    }
    double sp = sqrt(d1 * d1 + d2 * d2);
    g[0 * N + i] = x1;
    g[1 * N + i] = x2;
    g[2 * N + i] = d1;
    g[3 * N + i] = d2;
    g[4 * N + i] = e1;
    g[5 * N + i] = e2;
    g[6 * N + i] = sp;
    g[7 * N + i] = d2 / sp;
    g[8 * N + i] = -d1 / sp;
}

// R_l = -(2 pi / n) sum_{m=1}^{n-1} cos(m l pi / n)/m - (-1)^l pi / n^2 and
// log(4 sin^2(l pi / N)); one thread per l, fixed summation order.
__global__ void k_kress(int N, double* __restrict__ R, double* __restrict__ logtab) {
    int l = blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= N) return;
    const int n = N / 2;
    double acc = 0.0;
    for (int m = 1; m < n; ++m) {
        long long q = ((long long)m * l) % N;   // angle m l pi / n = 2 pi q / N
        acc += cospi(2.0 * (double)q / (double)N) / (double)m;
    }
    double sgn = (l & 1) ? -1.0 : 1.0;
    R[l] = -(2.0 * FHW_PI / n) * acc - sgn * FHW_PI / ((double)n * (double)n);
    logtab[l] = (l == 0) ? 0.0 : 2.0 * log(2.0 * fabs(sinpi((double)l / (double)N)));
}

hipError_t launch_geometry(hipStream_t s, const double* curve, int32_t degree, int32_t N, double* geom) {
    hipLaunchKernelGGL(k_geometry, dim3((N + 255) / 256), dim3(256), 0, s, curve, degree, N, geom);
    return hipGetLastError();
}

hipError_t launch_kress(hipStream_t s, int32_t N, double* R, double* logtab) {
    hipLaunchKernelGGL(k_kress, dim3((N + 255) / 256), dim3(256), 0, s, N, R, logtab);
    return hipGetLastError();
}
