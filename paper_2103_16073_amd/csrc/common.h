// Shared helpers for the fmmbem HIP library: complex arithmetic on double2/float2, index
// conventions of the spherical expansions, and HIP error plumbing.
#pragma once
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstdio>
#include <stdexcept>
#include <string>

#define FMM_PI 3.14159265358979323846

// ---------------------------------------------------------------- errors
struct FmmError : public std::runtime_error {
    int code;
    FmmError(int c, const std::string &m) : std::runtime_error(m), code(c) {}
};

#define HIP_OK(expr)                                                                                 \
    do {                                                                                             \
        hipError_t e__ = (expr);                                                                     \
        if (e__ != hipSuccess)                                                                       \
            throw FmmError(e__ == hipErrorOutOfMemory ? -2 : -3,                                     \
                           std::string(#expr) + ": " + hipGetErrorString(e__) + " @" + __FILE__ + \
                               ":" + std::to_string(__LINE__));                                      \
    } while (0)

#define LAUNCH_OK() HIP_OK(hipGetLastError())

// ---------------------------------------------------------------- complex on double2
__host__ __device__ inline double2 cmk(double r, double i) { return make_double2(r, i); }
__host__ __device__ inline double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__host__ __device__ inline double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__host__ __device__ inline double2 cmul(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__host__ __device__ inline double2 cmulc(double2 a, double2 b) {  // a * conj(b)
    return make_double2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
__host__ __device__ inline double2 cconj(double2 a) { return make_double2(a.x, -a.y); }
__host__ __device__ inline double2 cscale(double2 a, double s) { return make_double2(a.x * s, a.y * s); }
__host__ __device__ inline double2 cfma(double2 a, double2 b, double2 c) {  // a*b + c
    return make_double2(fma(a.x, b.x, fma(-a.y, b.y, c.x)), fma(a.x, b.y, fma(a.y, b.x, c.y)));
}
__host__ __device__ inline double2 cdiv(double2 a, double2 b) {
    double d = b.x * b.x + b.y * b.y;
    return make_double2((a.x * b.x + a.y * b.y) / d, (a.y * b.x - a.x * b.y) / d);
}
__host__ __device__ inline double2 cmuli(double2 a) { return make_double2(-a.y, a.x); }  // i*a
// i^m for integer m
__host__ __device__ inline double2 ipow(int m) {
    int r = ((m % 4) + 4) % 4;
    return r == 0 ? make_double2(1, 0) : r == 1 ? make_double2(0, 1) : r == 2 ? make_double2(-1, 0) : make_double2(0, -1);
}

__host__ __device__ inline float2 fcmul(float2 a, float2 b) {
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// ---------------------------------------------------------------- expansion indexing
// coefficient (n, m), |m| <= n < p, stored at n*n + n + m
__host__ __device__ inline int cidx(int n, int m) { return n * n + n + m; }
// coaxial table: blocks m = 0..p-1 of (p-m)^2 entries, rows n' = m..p-1, cols n = m..p-1
__host__ __device__ inline int64_t coax_block_off(int p, int m) {
    // sum_{j<m} (p-j)^2
    int64_t s = 0;
    (void)s;
    int64_t P = p;
    // closed form: sum_{j=0}^{m-1} (P-j)^2 = sum_{q=P-m+1}^{P} q^2
    auto sq = [](int64_t q) { return q * (q + 1) * (2 * q + 1) / 6; };
    return sq(P) - sq(P - m);
}
__host__ __device__ inline int64_t coax_table_size(int p) { return coax_block_off(p, p); }
// rotation table: block n at n(4n^2-1)/3, size (2n+1)^2
__host__ __device__ inline int64_t rot_block_off(int n) { return (int64_t)n * (4 * (int64_t)n * n - 1) / 3; }
__host__ __device__ inline int64_t rot_table_size(int p) { return rot_block_off(p); }

// a_n^m and b_n^m of the coaxial recursions (Section 3.3.1)
__host__ __device__ inline double coef_a(int n, int m) {
    int am = m < 0 ? -m : m;
    if (n < am) return 0.0;
    return sqrt((double)(n + 1 + am) * (double)(n + 1 - am) / ((double)(2 * n + 1) * (double)(2 * n + 3)));
}
__host__ __device__ inline double coef_b(int n, int m) {
    int am = m < 0 ? -m : m;
    if (am > n) return 0.0;
    double v = sqrt((double)(n - m - 1) * (double)(n - m) / ((double)(2 * n - 1) * (double)(2 * n + 1)));
    return m >= 0 ? v : -v;
}

// Recurrence of the normalised associated Legendre functions used by the regular basis
// (no Condon-Shortley phase), 0 <= m <= n:
//   P_m^m = g_m sin^m,  g_m = (4 pi)^{-1/2} prod_{q=1}^{m} sqrt((2q+1)/(2q)),
//   P_n^m = a_nm cos P_{n-1}^m - b_nm P_{n-2}^m  (n > m),
//   a_nm = sqrt((4n^2-1)/(n^2-m^2)),  b_nm = sqrt(((n-1)^2-m^2)(2n+1)/((2n-3)(n^2-m^2))) (0 for n = m+1).
// Table entry t = n(n+1)/2 + m holds (a_nm, b_nm, g_m) at 3t .. 3t+2; a table built for pmax holds
// every smaller one as a prefix.
__host__ __device__ inline int leg_tri(int n, int m) { return n * (n + 1) / 2 + m; }
__host__ __device__ inline int64_t leg_table_len(int pmax) { return 3 * (int64_t)(pmax + 1) * (pmax + 2) / 2; }

// squared distance without contraction, so that every kernel and the host classify
// near pairs identically
__device__ inline double dist2_exact(double ax, double ay, double az, double bx, double by, double bz) {
    double dx = __dsub_rn(bx, ax), dy = __dsub_rn(by, ay), dz = __dsub_rn(bz, az);
    return __dadd_rn(__dadd_rn(__dmul_rn(dx, dx), __dmul_rn(dy, dy)), __dmul_rn(dz, dz));
}

inline int ceil_div(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }

// spare entries allocated after every translation/rotation table (kernels read whole row chunks)
constexpr int64_t TABLE_PAD = 64;

// scalar-generic complex type: Cx<double>::T = double2, Cx<float>::T = float2
template <class R> struct Cx;
template <> struct Cx<double> { using T = double2; };
template <> struct Cx<float> { using T = float2; };

// tables used by one translation batch in the scalar type R
template <class R> struct TransTables {
    const typename Cx<R>::T *coax;
    const R *H, *HT;
    // the same tables in the fused tiles' fragment order (batches with p_src = p_tgt <= 16)
    const R *frH = nullptr, *frHT = nullptr, *frC = nullptr;
};
