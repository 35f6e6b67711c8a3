// Spherical Bessel sequences shared by the table generator and the expansion kernels.
#pragma once
#include <hip/hip_runtime.h>

#include <cmath>

namespace fmm {

// ------------------------------------------------------------------ spherical Bessel
// j[0..N] at x > 0 by Miller's algorithm (downward recurrence from well above max(N, x)).
__host__ __device__ inline void sph_jn_seq(double x, int N, double *j) {
    if (x < 1e-300) {
        j[0] = 1.0;
        for (int n = 1; n <= N; ++n) j[n] = 0.0;
        return;
    }
    int top = (N > (int)x ? N : (int)x);
    int start = top + 40 + (int)(4.0 * sqrt((double)top + 1.0));
    double fp1 = 0.0, f = 1e-300;
    for (int n = start; n >= 1; --n) {
        double fm1 = (2.0 * n + 1.0) / x * f - fp1;
        fp1 = f;
        f = fm1;
        if (n - 1 <= N) j[n - 1] = f;
        if (n <= N) j[n] = fp1;
        if (fabs(f) > 1e250) {  // rescale everything stored so far
            f *= 1e-250;
            fp1 *= 1e-250;
            int lo = n - 1;
            for (int q = lo; q <= N && q <= start; ++q) j[q] *= 1e-250;
        }
    }
    // normalise with the larger of j0, j1
    double s = sin(x), c = cos(x);
    double j0 = s / x, j1 = s / (x * x) - c / x;
    double scale = (fabs(j0) >= fabs(j1) || N < 1) ? j0 / j[0] : j1 / j[1];
    for (int n = 0; n <= N; ++n) j[n] *= scale;
}

__host__ __device__ inline void sph_yn_seq(double x, int N, double *y) {
    double s = sin(x), c = cos(x);
    y[0] = -c / x;
    if (N >= 1) y[1] = -c / (x * x) - s / x;
    for (int n = 1; n < N; ++n) y[n + 1] = (2.0 * n + 1.0) / x * y[n] - y[n - 1];
}

}  // namespace fmm
