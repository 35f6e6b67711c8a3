// Flexible GMRES (the paper's outer solver, Section 4.3) with FP64 Arnoldi on the device and a
// preconditioner slot: identity, diagonal (the paper's indirect-BEM choice: a constant added to
// the diagonal), or the exact inverse of the operator restricted to each octree leaf.
//
// Arnoldi uses classical Gram-Schmidt with a second pass when the first one cancelled most of the
// new vector (norm drop below 1/sqrt(2), the Daniel-Gragg-Kaufman-Stewart test): each pass is one
// batched set of inner products (two-stage, fixed-order reductions, so runs are bitwise
// reproducible) and one batched update.  Givens rotations and the small least-squares problem live on the host; one
// short host<->device copy per pass.
#include <chrono>
#include <functional>
#include <type_traits>

#include "internal.h"

namespace fmm {

constexpr int DOT_BLOCKS = 512;

// Krylov vectors are stored as double2 or (mixed-precision solves) float2; every inner product and
// update is computed in FP64.
__device__ inline double2 ldc(const double2 *p, int64_t i) { return p[i]; }
__device__ inline double2 ldc(const float2 *p, int64_t i) {
    const float2 v = p[i];
    return make_double2(v.x, v.y);
}
__device__ inline void stc(double2 *p, int64_t i, double2 v) { p[i] = v; }
__device__ inline void stc(float2 *p, int64_t i, double2 v) { p[i] = make_float2((float)v.x, (float)v.y); }

// partial[v * gridDim.x + blk] = sum_{i in blk's stride} conj(V_v[i]) w[i].  A workgroup takes
// DOT_G vectors (blockIdx.y group): each element of w it loads serves all of them, so w is read
// nv / DOT_G times rather than nv times (with FP32 Krylov vectors, w's 16 bytes per element would
// otherwise be twice the vector's own 8).
constexpr int DOT_G = 8;
template <class S>
__global__ void __launch_bounds__(256) k_dot_partial(int64_t n, const S *V, int64_t ldv, int nv, const double2 *w,
                                                     double2 *partial) {
    const int v0 = blockIdx.y * DOT_G, ng = min(DOT_G, nv - v0);
    double2 s[DOT_G];
#pragma unroll
    for (int g = 0; g < DOT_G; ++g) s[g] = cmk(0, 0);
    const int64_t i0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x, di = (int64_t)gridDim.x * blockDim.x;
    if (ng == DOT_G) {
        // whole group: the DOT_G loads of a row are issued before any of them is used
        for (int64_t i = i0; i < n; i += di) {
            const double2 wi = w[i];
            double2 x[DOT_G];
#pragma unroll
            for (int g = 0; g < DOT_G; ++g) x[g] = ldc(V + (int64_t)(v0 + g) * ldv, i);
#pragma unroll
            for (int g = 0; g < DOT_G; ++g) s[g] = cadd(s[g], cmulc(wi, x[g]));  // conj(V_v) w
        }
    } else {
        for (int64_t i = i0; i < n; i += di) {
            const double2 wi = w[i];
#pragma unroll
            for (int g = 0; g < DOT_G; ++g)
                if (g < ng) s[g] = cadd(s[g], cmulc(wi, ldc(V + (int64_t)(v0 + g) * ldv, i)));
        }
    }
    __shared__ double2 red[DOT_G][256];
#pragma unroll
    for (int g = 0; g < DOT_G; ++g) red[g][threadIdx.x] = s[g];
    __syncthreads();
    for (int q = blockDim.x / 2; q > 0; q >>= 1) {
        if ((int)threadIdx.x < q)
#pragma unroll
            for (int g = 0; g < DOT_G; ++g) red[g][threadIdx.x] = cadd(red[g][threadIdx.x], red[g][threadIdx.x + q]);
        __syncthreads();
    }
    if ((int)threadIdx.x < ng) partial[(int64_t)(v0 + threadIdx.x) * gridDim.x + blockIdx.x] = red[threadIdx.x][0];
}

__global__ void __launch_bounds__(256) k_dot_final(int nblk, const double2 *partial, double2 *out) {
    const int v = blockIdx.x;
    double2 s = cmk(0, 0);
    for (int i = threadIdx.x; i < nblk; i += blockDim.x) s = cadd(s, partial[(int64_t)v * nblk + i]);
    __shared__ double2 red[256];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int q = blockDim.x / 2; q > 0; q >>= 1) {
        if ((int)threadIdx.x < q) red[threadIdx.x] = cadd(red[threadIdx.x], red[threadIdx.x + q]);
        __syncthreads();
    }
    if (threadIdx.x == 0) out[v] = red[0];
}

// w -= sum_v h[v] V_v, in the order of v; vectors are read COMBO_U at a time, all loads of a
// group issued before the group's updates (one load per iteration would leave one 1 KB request in
// flight per wavefront)
constexpr int COMBO_U = 8;
template <class S>
__global__ void k_sub_combo(int64_t n, const S *V, int64_t ldv, int nv, const double2 *h, double2 *w) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double2 s = w[i];
    int v = 0;
    for (; v + COMBO_U <= nv; v += COMBO_U) {
        double2 x[COMBO_U];
#pragma unroll
        for (int u = 0; u < COMBO_U; ++u) x[u] = ldc(V, (int64_t)(v + u) * ldv + i);
#pragma unroll
        for (int u = 0; u < COMBO_U; ++u) s = csub(s, cmul(h[v + u], x[u]));
    }
    for (; v < nv; ++v) s = csub(s, cmul(h[v], ldc(V, (int64_t)v * ldv + i)));
    w[i] = s;
}

// x += sum_v y[v] Z_v (same grouping)
template <class S>
__global__ void k_add_combo(int64_t n, const S *Z, int64_t ldz, int nv, const double2 *y, double2 *x) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double2 s = x[i];
    int v = 0;
    for (; v + COMBO_U <= nv; v += COMBO_U) {
        double2 z[COMBO_U];
#pragma unroll
        for (int u = 0; u < COMBO_U; ++u) z[u] = ldc(Z, (int64_t)(v + u) * ldz + i);
#pragma unroll
        for (int u = 0; u < COMBO_U; ++u) s = cadd(s, cmul(y[v + u], z[u]));
    }
    for (; v < nv; ++v) s = cadd(s, cmul(y[v], ldc(Z, (int64_t)v * ldz + i)));
    x[i] = s;
}

// y = a x (stored in y's type)
template <class S>
__global__ void k_scale_copy(int64_t n, double a, const double2 *x, S *y) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) stc(y, i, cscale(x[i], a));
}

template <class S>
__global__ void k_widen(int64_t n, const S *x, double2 *y) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] = ldc(x, i);
}

__global__ void k_sub(int64_t n, const double2 *a, const double2 *b, double2 *out) {  // out = a - b
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = csub(a[i], b[i]);
}

__global__ void k_mul_diag(int64_t n, const double2 *d, const double2 *v, double2 *z) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) z[i] = cmul(d[i], v[i]);
}

// ------------------------------------------------------------------ preconditioners
// inverse diagonal, caller order: 1 / (1/2 + M_ii - i k beta_i L_ii + shift)
__global__ void k_diag_inv(int64_t n, const int32_t *perm, const int32_t *near_start, const int32_t *near_col,
                           const double2 *nL, const double2 *nM, const double2 *beta, double k, double shift,
                           double2 *dinv) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double2 a = cmk(0.5 + shift, 0.0);
    for (int e = near_start[i]; e < near_start[i + 1]; ++e)
        if (near_col[e] == i) {
            double2 ikb = cmk(-k * beta[i].y, k * beta[i].x);
            a = cadd(a, csub(nM[e], cmul(ikb, nL[e])));
        }
    dinv[perm[i]] = cdiv(cmk(1, 0), a);
}

// inverse diagonal of the combined (Burton-Miller) direct operator, caller order:
//   1/2 + shift + (alpha i k / 2) beta_i + M_ii - i k beta_i L_ii + alpha (M'_ii - i k beta_i L'_ii)
__global__ void k_diag_bm_inv(int64_t n, const int32_t *perm, const int32_t *near_start, const int32_t *near_col,
                              const double2 *nL, const double2 *nM, const double2 *nLp, const double2 *nMp,
                              const double2 *beta, double k, double2 alpha, double shift, double2 *dinv) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double2 ikb = cscale(cmuli(beta[i]), k);
    double2 a = cadd(cmk(0.5 + shift, 0.0), cscale(cmul(alpha, ikb), 0.5));
    for (int e = near_start[i]; e < near_start[i + 1]; ++e)
        if (near_col[e] == i) {
            a = cadd(a, csub(nM[e], cmul(ikb, nL[e])));
            a = cadd(a, cmul(alpha, csub(nMp[e], cmul(ikb, nLp[e]))));
        }
    dinv[perm[i]] = cdiv(cmk(1, 0), a);
}

// dense operator block of each leaf, row-major n_b x n_b at blk_off[b] (sorted element order)
__global__ void __launch_bounds__(256) k_leaf_blocks(int nleaf, const int32_t *leaf_start, const int64_t *blk_off,
                                                     const double4 *ec, const double4 *en, const double2 *beta,
                                                     double k, double rc2, const int32_t *near_start,
                                                     const int32_t *near_col, const double2 *nL, const double2 *nM,
                                                     double2 *A) {
    const int b = blockIdx.x;
    const int s = leaf_start[b], nb = leaf_start[b + 1] - s;
    double2 *Ab = A + blk_off[b];
    const double inv4pi = 1.0 / (4.0 * FMM_PI);
    for (int e = threadIdx.x; e < nb * nb; e += blockDim.x) {
        int i = s + e / nb, j = s + e % nb;
        double4 ci = ec[i], cj = ec[j];
        double d2 = dist2_exact(ci.x, ci.y, ci.z, cj.x, cj.y, cj.z);
        double2 v = cmk(0, 0);
        if (i != j && d2 >= rc2) {
            double4 nj = en[j];
            double r = sqrt(d2), sn, cs;
            sincos(k * r, &sn, &cs);
            double2 G = cmk(cs / r * inv4pi * cj.w, sn / r * inv4pi * cj.w);  // A_j G
            double u = ((cj.x - ci.x) * nj.x + (cj.y - ci.y) * nj.y + (cj.z - ci.z) * nj.z) / d2;
            double2 M = cmul(G, cmk(-u, k * r * u));
            double2 ikb = cmk(-k * beta[j].y, k * beta[j].x);
            v = csub(M, cmul(ikb, G));
        }
        if (i == j) v.x += 0.5;
        Ab[e] = v;
    }
    __syncthreads();
    for (int r = threadIdx.x; r < nb; r += blockDim.x) {
        int i = s + r;
        for (int e = near_start[i]; e < near_start[i + 1]; ++e) {
            int j = near_col[e];
            if (j < s || j >= s + nb) continue;
            double2 ikb = cmk(-k * beta[j].y, k * beta[j].x);
            Ab[(int64_t)r * nb + (j - s)] = cadd(Ab[(int64_t)r * nb + (j - s)], csub(nM[e], cmul(ikb, nL[e])));
        }
    }
}

// dense block of the indirect operator (Eq. ibem5) on each leaf's unknowns, row-major
// 2 n_b x 2 n_b at blk_off[b]: rows (psi- equation of the leaf's elements, then psi+ equation),
// columns (psi- of the leaf's elements, then psi+), elements in sorted order.  With
// sigma_j = -i k (beta-_j psi-_j + beta+_j psi+_j) and mu_j = psi-_j - psi+_j, the equations are
//   V_i + (psi-_i + psi+_i) / 2                            (V = sum_j L_ij sigma_j + M_ij mu_j)
//   W_i + i k (beta-_i psi-_i - beta+_i psi+_i) / 2        (W = sum_j L'_ij sigma_j + M'_ij mu_j)
// the pair entries L, M, L', M' from the near tables where |c_i - c_j| < r_c, from the one-point
// rule of the near field elsewhere.
__global__ void __launch_bounds__(256) k_leaf_blocks_ind(int nleaf, const int32_t *leaf_start, const int64_t *blk_off,
                                                         const double4 *ec, const double4 *en, const double2 *bm,
                                                         const double2 *bp, double k, double rc2,
                                                         const int32_t *near_start, const int32_t *near_col,
                                                         const double2 *nL, const double2 *nM, const double2 *nLp,
                                                         const double2 *nMp, double2 *A) {
    const int b = blockIdx.x;
    const int s = leaf_start[b], nb = leaf_start[b + 1] - s, n2 = 2 * nb;
    double2 *Ab = A + blk_off[b];
    const double inv4pi = 1.0 / (4.0 * FMM_PI);
    // the four entries of pair (i, j) into the 2 x 2 sub-block (rows i, i + nb; columns j, j + nb)
    auto put = [&](int r, int q, double2 L, double2 M, double2 Lp, double2 Mp, bool add) {
        const int j = s + q;
        const double2 ikm = cscale(cmuli(bm[j]), k), ikp = cscale(cmuli(bp[j]), k);  // i k beta-+_j
        const double2 e00 = csub(M, cmul(ikm, L)), e01 = csub(cscale(M, -1.0), cmul(ikp, L));
        const double2 e10 = csub(Mp, cmul(ikm, Lp)), e11 = csub(cscale(Mp, -1.0), cmul(ikp, Lp));
        double2 *r0 = Ab + (int64_t)r * n2, *r1 = Ab + (int64_t)(r + nb) * n2;
        if (add) {
            r0[q] = cadd(r0[q], e00);
            r0[q + nb] = cadd(r0[q + nb], e01);
            r1[q] = cadd(r1[q], e10);
            r1[q + nb] = cadd(r1[q + nb], e11);
        } else {
            r0[q] = e00;
            r0[q + nb] = e01;
            r1[q] = e10;
            r1[q + nb] = e11;
        }
    };
    for (int e = threadIdx.x; e < nb * nb; e += blockDim.x) {
        const int r = e / nb, q = e % nb, i = s + r, j = s + q;
        const double4 ci = ec[i], cj = ec[j];
        const double d2 = dist2_exact(ci.x, ci.y, ci.z, cj.x, cj.y, cj.z);
        double2 L = cmk(0, 0), M = L, Lp = L, Mp = L;
        if (i != j && d2 >= rc2) {
            const double4 ni = en[i], nj = en[j];
            const double dx = cj.x - ci.x, dy = cj.y - ci.y, dz = cj.z - ci.z;
            const double r1 = sqrt(d2), ir = 1.0 / r1, ir2 = ir * ir;
            double sn, cs;
            sincos(k * r1, &sn, &cs);
            const double2 E = cmk(cs * inv4pi * cj.w, sn * inv4pi * cj.w);  // A_j e^{ikr} / 4 pi
            const double2 G = cscale(E, ir);
            const double dny = dx * nj.x + dy * nj.y + dz * nj.z, dnx = dx * ni.x + dy * ni.y + dz * ni.z;
            const double nn = ni.x * nj.x + ni.y * nj.y + ni.z * nj.z;
            const double2 g1 = cmul(G, cmk(-1.0, k * r1));  // G (ikr - 1)
            L = G;
            M = cscale(g1, dny * ir2);
            Lp = cscale(g1, -dnx * ir2);
            const double2 k3 = cmul(E, cmk(3.0 - k * k * d2, -3.0 * k * r1));
            Mp = csub(cscale(k3, -dnx * dny * ir2 * ir2 * ir), cscale(cmul(E, cmk(-1.0, k * r1)), nn * ir2 * ir));
        }
        put(r, q, L, M, Lp, Mp, false);
    }
    __syncthreads();
    // near-table entries (each row's entries belong to one thread: no two threads touch one row)
    for (int r = threadIdx.x; r < nb; r += blockDim.x) {
        const int i = s + r;
        for (int e = near_start[i]; e < near_start[i + 1]; ++e) {
            const int j = near_col[e];
            if (j < s || j >= s + nb) continue;
            put(r, j - s, nL[e], nM[e], nLp[e], nMp[e], true);
        }
        // local terms
        const double2 ikm = cscale(cmuli(bm[i]), k), ikp = cscale(cmuli(bp[i]), k);
        double2 *r0 = Ab + (int64_t)r * n2, *r1 = Ab + (int64_t)(r + nb) * n2;
        r0[r] = cadd(r0[r], cmk(0.5, 0.0));
        r0[r + nb] = cadd(r0[r + nb], cmk(0.5, 0.0));
        r1[r] = cadd(r1[r], cscale(ikm, 0.5));
        r1[r + nb] = cadd(r1[r + nb], cscale(ikp, -0.5));
    }
}

// dense block of the combined (Burton-Miller) direct operator on each leaf, row-major n_b x n_b:
//   1/2 delta_ij + (alpha i k / 2) beta_i delta_ij + M_ij - i k beta_j L_ij + alpha (M'_ij - i k beta_j L'_ij)
// pair entries from the near tables or the near field's one-point rule, as for the indirect blocks
__global__ void __launch_bounds__(256) k_leaf_blocks_bm(int nleaf, const int32_t *leaf_start, const int64_t *blk_off,
                                                        const double4 *ec, const double4 *en, const double2 *beta,
                                                        double k, double2 alpha, double rc2, const int32_t *near_start,
                                                        const int32_t *near_col, const double2 *nL, const double2 *nM,
                                                        const double2 *nLp, const double2 *nMp, double2 *A) {
    const int b = blockIdx.x;
    const int s = leaf_start[b], nb = leaf_start[b + 1] - s;
    double2 *Ab = A + blk_off[b];
    const double inv4pi = 1.0 / (4.0 * FMM_PI);
    auto entry = [&](int j, double2 L, double2 M, double2 Lp, double2 Mp) {
        const double2 ikb = cscale(cmuli(beta[j]), k);
        return cadd(csub(M, cmul(ikb, L)), cmul(alpha, csub(Mp, cmul(ikb, Lp))));
    };
    for (int e = threadIdx.x; e < nb * nb; e += blockDim.x) {
        const int r = e / nb, q = e % nb, i = s + r, j = s + q;
        const double4 ci = ec[i], cj = ec[j];
        const double d2 = dist2_exact(ci.x, ci.y, ci.z, cj.x, cj.y, cj.z);
        double2 v = cmk(0, 0);
        if (i != j && d2 >= rc2) {
            const double4 ni = en[i], nj = en[j];
            const double dx = cj.x - ci.x, dy = cj.y - ci.y, dz = cj.z - ci.z;
            const double r1 = sqrt(d2), ir = 1.0 / r1, ir2 = ir * ir;
            double sn, cs;
            sincos(k * r1, &sn, &cs);
            const double2 E = cmk(cs * inv4pi * cj.w, sn * inv4pi * cj.w);  // A_j e^{ikr} / 4 pi
            const double2 G = cscale(E, ir);
            const double dny = dx * nj.x + dy * nj.y + dz * nj.z, dnx = dx * ni.x + dy * ni.y + dz * ni.z;
            const double nn = ni.x * nj.x + ni.y * nj.y + ni.z * nj.z;
            const double2 g1 = cmul(G, cmk(-1.0, k * r1));  // G (ikr - 1)
            const double2 k3 = cmul(E, cmk(3.0 - k * k * d2, -3.0 * k * r1));
            const double2 Mp =
                csub(cscale(k3, -dnx * dny * ir2 * ir2 * ir), cscale(cmul(E, cmk(-1.0, k * r1)), nn * ir2 * ir));
            v = entry(j, G, cscale(g1, dny * ir2), cscale(g1, -dnx * ir2), Mp);
        }
        Ab[e] = v;
    }
    __syncthreads();
    for (int r = threadIdx.x; r < nb; r += blockDim.x) {
        const int i = s + r;
        for (int e = near_start[i]; e < near_start[i + 1]; ++e) {
            const int j = near_col[e];
            if (j < s || j >= s + nb) continue;
            Ab[(int64_t)r * nb + (j - s)] = cadd(Ab[(int64_t)r * nb + (j - s)], entry(j, nL[e], nM[e], nLp[e], nMp[e]));
        }
        const double2 ikb = cscale(cmuli(beta[i]), k);
        Ab[(int64_t)r * nb + r] = cadd(Ab[(int64_t)r * nb + r], cadd(cmk(0.5, 0.0), cscale(cmul(alpha, ikb), 0.5)));
    }
}

// in-place Gauss-Jordan inversion with partial pivoting, one workgroup per leaf block
// (block dimension m n_b: m unknowns per element; at most 1024)
__global__ void __launch_bounds__(256) k_leaf_invert(int nleaf, const int32_t *leaf_start, const int64_t *blk_off,
                                                     double2 *A, int32_t *piv_ws, int *status, int m) {
    const int b = blockIdx.x;
    const int nb = m * (leaf_start[b + 1] - leaf_start[b]);
    double2 *M = A + blk_off[b];
    int32_t *piv = piv_ws + (int64_t)m * leaf_start[b];
    __shared__ int sp;
    __shared__ double sbest[256];
    __shared__ int sidx[256];
    __shared__ double2 prow[1024];
    for (int c = 0; c < nb; ++c) {
        // pivot search in column c, rows c..nb-1
        double best = -1.0;
        int bi = c;
        for (int r = c + threadIdx.x; r < nb; r += blockDim.x) {
            double2 v = M[(int64_t)r * nb + c];
            double a = v.x * v.x + v.y * v.y;
            if (a > best) {
                best = a;
                bi = r;
            }
        }
        sbest[threadIdx.x] = best;
        sidx[threadIdx.x] = bi;
        __syncthreads();
        if (threadIdx.x == 0) {
            double bb = -1.0;
            int ii = c;
            for (int t = 0; t < (int)blockDim.x; ++t)
                if (sbest[t] > bb) {
                    bb = sbest[t];
                    ii = sidx[t];
                }
            sp = ii;
            piv[c] = ii;
            if (!(bb > 0.0)) atomicExch(status, 1);
        }
        __syncthreads();
        const int pr = sp;
        if (pr != c)
            for (int q = threadIdx.x; q < nb; q += blockDim.x) {
                double2 t = M[(int64_t)c * nb + q];
                M[(int64_t)c * nb + q] = M[(int64_t)pr * nb + q];
                M[(int64_t)pr * nb + q] = t;
            }
        __syncthreads();
        const double2 pv = M[(int64_t)c * nb + c];
        const double2 ipv = cdiv(cmk(1, 0), pv);
        // scale pivot row: row c <- row c / pv, with the inverse's column c set to 1/pv
        for (int q = threadIdx.x; q < nb; q += blockDim.x) {
            double2 v = (q == c) ? cmk(1, 0) : M[(int64_t)c * nb + q];
            prow[q] = cmul(v, ipv);
        }
        __syncthreads();
        for (int q = threadIdx.x; q < nb; q += blockDim.x) M[(int64_t)c * nb + q] = prow[q];
        __syncthreads();
        // eliminate column c from every other row (each thread owns whole rows)
        for (int r = threadIdx.x; r < nb; r += blockDim.x) {
            if (r == c) continue;
            double2 f = M[(int64_t)r * nb + c];
            for (int q = 0; q < nb; ++q) {
                double2 v = (q == c) ? cmk(0, 0) : M[(int64_t)r * nb + q];
                M[(int64_t)r * nb + q] = csub(v, cmul(f, prow[q]));
            }
        }
        __syncthreads();
    }
    // undo the column permutation implied by the row swaps (in reverse order)
    for (int c = nb - 1; c >= 0; --c) {
        const int pr = piv[c];
        if (pr != c)
            for (int r = threadIdx.x; r < nb; r += blockDim.x) {
                double2 t = M[(int64_t)r * nb + c];
                M[(int64_t)r * nb + c] = M[(int64_t)r * nb + pr];
                M[(int64_t)r * nb + pr] = t;
            }
        __syncthreads();
    }
}

// z = blockdiag(A_BB^{-1}) v, vectors in caller order; m unknowns per element (block index
// q of element s + (q mod n_b) is unknown (q / n_b) n + perm[s + q mod n_b])
__global__ void __launch_bounds__(128) k_leaf_apply(int nleaf, const int32_t *leaf_start, const int64_t *blk_off,
                                                    const double2 *Ainv, const int32_t *perm, const double2 *v,
                                                    double2 *z, int m, int64_t n) {
    const int b = blockIdx.x;
    const int s = leaf_start[b], ne = leaf_start[b + 1] - s, nb = m * ne;
    const double2 *M = Ainv + blk_off[b];
    __shared__ double2 vs[1024];
    auto idx = [&](int q) -> int64_t { return (int64_t)(q / ne) * n + perm[s + q % ne]; };
    for (int q = threadIdx.x; q < nb; q += blockDim.x) vs[q] = v[idx(q)];
    __syncthreads();
    for (int r = threadIdx.x; r < nb; r += blockDim.x) {
        double2 acc = cmk(0, 0);
        for (int q = 0; q < nb; ++q) acc = cfma(M[(int64_t)r * nb + q], vs[q], acc);
        z[idx(r)] = acc;
    }
}

// ------------------------------------------------------------------ host helpers
struct Blas {
    hipStream_t st;
    DeviceBuffers &scr;
    int64_t n;
    std::string tag;  // scratch-name prefix, so nested solves keep separate buffers
    template <class S>
    void dots(const S *V, int64_t ldv, int nv, const double2 *w, double2 *host_out) {
        double2 *part = dget<double2>(scr, tag + "dot_part", (size_t)DOT_BLOCKS * std::max(nv, 1));
        double2 *res = dget<double2>(scr, tag + "dot_res", std::max(nv, 1));
        int nblk = (int)std::min<int64_t>(DOT_BLOCKS, std::max<int64_t>(1, (n + 255) / 256));
        k_dot_partial<S><<<dim3(nblk, (nv + DOT_G - 1) / DOT_G), 256, 0, st>>>(n, V, ldv, nv, w, part);
        LAUNCH_OK();
        k_dot_final<<<nv, 256, 0, st>>>(nblk, part, res);
        LAUNCH_OK();
        HIP_OK(hipMemcpyAsync(host_out, res, sizeof(double2) * nv, hipMemcpyDeviceToHost, st));
        HIP_OK(hipStreamSynchronize(st));
    }
    double nrm(const double2 *w) {
        double2 d;
        dots(w, 0, 1, w, &d);
        return sqrt(std::max(d.x, 0.0));
    }
    template <class S>
    void sub_combo(const S *V, int64_t ldv, int nv, const double2 *h_host, double2 *w) {
        double2 *h = dget<double2>(scr, tag + "combo_h", std::max(nv, 1));
        HIP_OK(hipMemcpyAsync(h, h_host, sizeof(double2) * nv, hipMemcpyHostToDevice, st));
        k_sub_combo<S><<<ceil_div(n, 256), 256, 0, st>>>(n, V, ldv, nv, h, w);
        LAUNCH_OK();
    }
    template <class S>
    void add_combo(const S *Z, int64_t ldz, int nv, const double2 *y_host, double2 *x) {
        double2 *h = dget<double2>(scr, tag + "combo_y", std::max(nv, 1));
        HIP_OK(hipMemcpyAsync(h, y_host, sizeof(double2) * nv, hipMemcpyHostToDevice, st));
        k_add_combo<S><<<ceil_div(n, 256), 256, 0, st>>>(n, Z, ldz, nv, h, x);
        LAUNCH_OK();
    }
    template <class S>
    void scale_copy(double a, const double2 *x, S *y) {
        k_scale_copy<S><<<ceil_div(n, 256), 256, 0, st>>>(n, a, x, y);
        LAUNCH_OK();
    }
    template <class S>
    void widen(const S *x, double2 *y) {
        k_widen<S><<<ceil_div(n, 256), 256, 0, st>>>(n, x, y);
        LAUNCH_OK();
    }
    void sub(const double2 *a, const double2 *b, double2 *out) {
        k_sub<<<ceil_div(n, 256), 256, 0, st>>>(n, a, b, out);
        LAUNCH_OK();
    }
};

static inline double cabs_(double2 a) { return hypot(a.x, a.y); }

// Restarted FGMRES(m).  matvec(x, y) and precond(v, z) act on device vectors of length n; the
// preconditioner may change from one call to the next (an inner solve, a learned map).
// Returns FMMBEM_OK / FMMBEM_ENOCONV / error codes.  rel_res is the true relative residual of the
// last restart, computed with `matvec_check` (the FP64 operator); with final_residual false, a
// solve that stops at maxit skips that last product and reports the Arnoldi estimate instead
// (inner solves).  history, when given, receives the estimate after every iteration.
// S: storage type of the Krylov vectors V and Z (double2, or float2 for mixed-precision solves:
// half the basis traffic; inner products, Hessenberg matrix, rotations, the iterate and the
// restart residual stay FP64).
template <class S>
static int fgmres_t(int64_t n, hipStream_t st, DeviceBuffers &scr, const char *tag,
                    const std::function<void(const double2 *, double2 *)> &matvec,
                    const std::function<void(const double2 *, double2 *)> &matvec_check,
                    const std::function<void(const double2 *, double2 *)> &precond, const double2 *b, double2 *x,
                    double tol, int m, int maxit, bool x0_given, bool final_residual, std::vector<double> *history,
                    int &iters, int &restarts, double &rel_res, const FgmresHooks *hooks, int reorth) {
    constexpr bool wide = std::is_same<S, double2>::value;
    const std::string tg(tag);
    Blas B{st, scr, n, tg};
    S *V = dget<S>(scr, tg + (wide ? "fg_V" : "fg_V32"), (size_t)(m + 1) * n);
    S *Z = dget<S>(scr, tg + (wide ? "fg_Z" : "fg_Z32"), (size_t)m * n);
    double2 *w = dget<double2>(scr, tg + "fg_w", n);
    double2 *r = dget<double2>(scr, tg + "fg_r", n);
    // FP64 copies of the current basis vector and its preconditioned image (narrow storage only)
    double2 *tv = wide ? nullptr : dget<double2>(scr, tg + "fg_tv", n);
    double2 *tz = wide ? nullptr : dget<double2>(scr, tg + "fg_tz", n);
    if (!x0_given) HIP_OK(hipMemsetAsync(x, 0, sizeof(double2) * n, st));
    const double bn = B.nrm(b);
    iters = 0;
    restarts = 0;
    rel_res = 1.0;
    if (!(bn > 0.0)) {
        HIP_OK(hipMemsetAsync(x, 0, sizeof(double2) * n, st));
        rel_res = 0.0;
        return FMMBEM_OK;
    }
    std::vector<double2> H((size_t)(m + 1) * m), g(m + 1), cs(m), sn(m), h1(m + 1), h2(m + 1), y(m);
    auto Hc = [&](int i, int j) -> double2 & { return H[(size_t)i * m + j]; };
    int status = FMMBEM_ENOCONV;
    double est = 1.0;
    while (true) {
        if (!final_residual && restarts > 0 && iters >= maxit) {
            rel_res = est;
            break;
        }
        // true residual
        if (x0_given || restarts > 0) {
            matvec_check(x, w);
            B.sub(b, w, r);
        } else {
            HIP_OK(hipMemcpyAsync(r, b, sizeof(double2) * n, hipMemcpyDeviceToDevice, st));
        }
        double beta = B.nrm(r);
        rel_res = beta / bn;
        if (!std::isfinite(beta)) return FMMBEM_ENAN;
        if (hooks && hooks->on_restart) hooks->on_restart(x, r, rel_res);
        if (rel_res < tol) {
            status = FMMBEM_OK;
            break;
        }
        if (iters >= maxit) break;
        B.scale_copy(1.0 / beta, r, V);
        std::fill(g.begin(), g.end(), cmk(0, 0));
        g[0] = cmk(beta, 0);
        int j = 0;
        bool done = false;
        for (j = 0; j < m && iters < maxit; ++j) {
            S *vjs = V + (size_t)j * n, *zjs = Z + (size_t)j * n;
            const double2 *vj;
            double2 *zj;
            if constexpr (wide) {
                vj = vjs;
                zj = zjs;
            } else {
                B.widen(vjs, tv);
                vj = tv;
                zj = tz;
            }
            precond(vj, zj);
            if constexpr (!wide) B.scale_copy(1.0, zj, zjs);
            matvec(zj, w);
            ++iters;
            // classical Gram-Schmidt; reorth 1 repeats it only when the first pass removed most of w
            // (|w| fell below |w_0|/sqrt(2): the Daniel-Gragg-Kaufman-Stewart criterion), 2 always,
            // 0 never
            const double w0 = reorth == 1 ? B.nrm(w) : 0.0;
            B.dots(V, n, j + 1, w, h1.data());
            B.sub_combo(V, n, j + 1, h1.data(), w);
            double hn = B.nrm(w);
            if (reorth == 2 || (reorth == 1 && !(hn > 0.7071067811865476 * w0))) {
                B.dots(V, n, j + 1, w, h2.data());
                B.sub_combo(V, n, j + 1, h2.data(), w);
                for (int i = 0; i <= j; ++i) h1[i] = cadd(h1[i], h2[i]);
                hn = B.nrm(w);
            }
            for (int i = 0; i <= j; ++i) Hc(i, j) = h1[i];
            if (!std::isfinite(hn)) return FMMBEM_ENAN;
            Hc(j + 1, j) = cmk(hn, 0);
            if (hn > 0) B.scale_copy(1.0 / hn, w, V + (size_t)(j + 1) * n);
            for (int i = 0; i < j; ++i) {
                double2 a = Hc(i, j), c = Hc(i + 1, j);
                Hc(i, j) = cadd(cscale(a, cs[i].x), cmul(sn[i], c));
                Hc(i + 1, j) = csub(cscale(c, cs[i].x), cmul(cconj(sn[i]), a));
            }
            double2 a = Hc(j, j), c = Hc(j + 1, j);
            double den = hypot(cabs_(a), cabs_(c));
            if (den == 0) {
                cs[j] = cmk(1, 0);
                sn[j] = cmk(0, 0);
            } else {
                double aa = cabs_(a);
                cs[j] = cmk(aa / den, 0);
                double2 ph = aa > 0 ? cscale(a, 1.0 / aa) : cmk(1, 0);
                sn[j] = cscale(cmul(ph, cconj(c)), 1.0 / den);
            }
            Hc(j, j) = cadd(cscale(a, cs[j].x), cmul(sn[j], c));
            Hc(j + 1, j) = cmk(0, 0);
            g[j + 1] = cscale(cmul(cconj(sn[j]), g[j]), -1.0);
            g[j] = cscale(g[j], cs[j].x);
            est = cabs_(g[j + 1]) / bn;
            if (history) history->push_back(est);
            if (hooks && hooks->on_iter) hooks->on_iter(iters, est);
            if (est < tol || hn == 0) {
                ++j;
                done = true;
                break;
            }
        }
        // y = H^{-1} g (upper triangular)
        for (int i = j - 1; i >= 0; --i) {
            double2 s = g[i];
            for (int q = i + 1; q < j; ++q) s = csub(s, cmul(Hc(i, q), y[q]));
            if (cabs_(Hc(i, i)) == 0) return FMMBEM_EBREAKDOWN;
            y[i] = cdiv(s, Hc(i, i));
        }
        B.add_combo(Z, n, j, y.data(), x);
        ++restarts;
        x0_given = true;
        (void)done;
    }
    return status;
}

int fgmres(int64_t n, hipStream_t st, DeviceBuffers &scr, const char *tag,
           const std::function<void(const double2 *, double2 *)> &matvec,
           const std::function<void(const double2 *, double2 *)> &matvec_check,
           const std::function<void(const double2 *, double2 *)> &precond, const double2 *b, double2 *x, double tol,
           int m, int maxit, bool x0_given, bool final_residual, std::vector<double> *history, int &iters,
           int &restarts, double &rel_res, const FgmresHooks *hooks, bool basis32, int reorth) {
    if (basis32)
        return fgmres_t<float2>(n, st, scr, tag, matvec, matvec_check, precond, b, x, tol, m, maxit, x0_given,
                                final_residual, history, iters, restarts, rel_res, hooks, reorth);
    return fgmres_t<double2>(n, st, scr, tag, matvec, matvec_check, precond, b, x, tol, m, maxit, x0_given,
                             final_residual, history, iters, restarts, rel_res, hooks, reorth);
}

// Lock-step FGMRES over groups of systems.  A group is nv systems A x_s = b_s that share one
// operator (one context: the same mesh, wavenumber and admittance, one source each): every step of
// a group gathers the preconditioned vectors of its systems still iterating and applies one batched
// product, so the kernel evaluations, basis functions and translation tables of the FMM are shared
// between them.  Each system keeps its own Krylov basis, Hessenberg matrix and restarts, exactly as
// fgmres().  Several groups (contexts of other frequencies or rooms, each with its own N, octree and
// truncation numbers) advance in turn from one host thread: a group's next product is enqueued on
// its own streams as soon as its Arnoldi step is done, and a group's Arnoldi step waits for its own
// stream only, so the products of the other groups keep the device busy meanwhile.
template <class S>
struct BatchSys {
    S *V = nullptr, *Z = nullptr;
    double2 *r = nullptr;
    std::vector<double2> H, g, cs, sn, h1, h2, y;
    double bn = 0.0, est = 1.0;
    int j = 0, cycle = 0;  // cycle = restarts so far
    bool in_cycle = false, done = false;
};

template <class T>
struct GroupSolver {
    static constexpr bool wide = std::is_same<T, double2>::value;
    FgmresGroup &G;
    Blas Bl;
    std::vector<BatchSys<T>> S;
    double2 *tv = nullptr, *Sin = nullptr, *Sout = nullptr;
    double2 *part = nullptr;             // partial sums of the inner products (one stream: shared)
    double2 *dres = nullptr;             // per system: inner products (m + 1), |w_0|^2, |w|^2
    double2 *dy = nullptr;               // per system: the coefficients y of x += Z y
    double2 *hres = nullptr, *hy = nullptr;  // pinned host copies
    std::vector<int> act;                // systems whose product is in flight, in Sin/Sout order
    std::vector<char> second;            // per system: a second Gram-Schmidt pass this step
    std::vector<int> need;               // systems whose true residual is being formed
    bool pending = false;                // work enqueued whose results the host reads next
    explicit GroupSolver(FgmresGroup &g) : G(g), Bl{g.st, *g.scr, g.n, g.tag + "bt_"} {}
    ~GroupSolver() {
        if (hres) (void)hipHostFree(hres);
        if (hy) (void)hipHostFree(hy);
    }
    int RS() const { return G.m + 3; }  // stride of dres / hres per system
    double2 *res(int s) { return dres + (size_t)s * RS(); }
    double2 *hr(int s) { return hres + (size_t)s * RS(); }

    // inner products conj(V_v) w, v < nv, into out (device), enqueued only
    template <class SV>
    void dots_to(const SV *V, int64_t ldv, int nv, const double2 *w, double2 *out) {
        const int nblk = (int)std::min<int64_t>(DOT_BLOCKS, std::max<int64_t>(1, (G.n + 255) / 256));
        k_dot_partial<SV><<<dim3(nblk, (nv + DOT_G - 1) / DOT_G), 256, 0, G.st>>>(G.n, V, ldv, nv, w, part);
        LAUNCH_OK();
        k_dot_final<<<nv, 256, 0, G.st>>>(nblk, part, out);
        LAUNCH_OK();
    }
    void to_host(int s) {  // the system's inner products and norms to the pinned copy
        HIP_OK(hipMemcpyAsync(hr(s), res(s), sizeof(double2) * RS(), hipMemcpyDeviceToHost, G.st));
        pending = true;
    }
    void wait() {
        if (pending) HIP_OK(hipStreamSynchronize(G.st));
        pending = false;
    }

    void init() {
        const int64_t n = G.n;
        const int nv = G.nv, m = G.m;
        S.assign(nv, BatchSys<T>());
        second.assign(nv, 0);
        tv = wide ? nullptr : dget<double2>(*G.scr, G.tag + "bt_tv", n);
        G.iters.assign(nv, 0);
        G.restarts.assign(nv, 0);
        G.rel_res.assign(nv, 1.0);
        G.status.assign(nv, FMMBEM_ENOCONV);
        Sin = dget<double2>(*G.scr, G.tag + "bt_in", (size_t)nv * n);
        Sout = dget<double2>(*G.scr, G.tag + "bt_out", (size_t)nv * n);
        part = dget<double2>(*G.scr, G.tag + "bt_part", (size_t)DOT_BLOCKS * (m + 1));
        dres = dget<double2>(*G.scr, G.tag + "bt_res", (size_t)nv * RS());
        dy = dget<double2>(*G.scr, G.tag + "bt_y", (size_t)nv * (m + 1));
        HIP_OK(hipHostMalloc((void **)&hres, sizeof(double2) * nv * RS()));
        HIP_OK(hipHostMalloc((void **)&hy, sizeof(double2) * nv * (m + 1)));
        for (int s = 0; s < nv; ++s) {
            BatchSys<T> &q = S[s];
            const std::string id = G.tag + std::to_string(s);
            q.V = dget<T>(*G.scr, (wide ? "bt_V" : "bt_V32_") + id, (size_t)(m + 1) * n);
            q.Z = dget<T>(*G.scr, (wide ? "bt_Z" : "bt_Z32_") + id, (size_t)m * n);
            q.r = dget<double2>(*G.scr, "bt_r" + id, n);
            q.H.assign((size_t)(m + 1) * m, cmk(0, 0));
            q.g.assign(m + 1, cmk(0, 0));
            q.cs.assign(m, cmk(0, 0));
            q.sn.assign(m, cmk(0, 0));
            q.h1.assign(m + 1, cmk(0, 0));
            q.h2.assign(m + 1, cmk(0, 0));
            q.y.assign(m, cmk(0, 0));
            double2 *x = G.X + (int64_t)s * n;
            if (!G.x0_given) HIP_OK(hipMemsetAsync(x, 0, sizeof(double2) * n, G.st));
            dots_to(G.B + (int64_t)s * n, 0, 1, G.B + (int64_t)s * n, res(s) + m + 2);
            to_host(s);
        }
    }
    void init_done() {
        for (int s = 0; s < G.nv; ++s) {
            BatchSys<T> &q = S[s];
            q.bn = sqrt(std::max(hr(s)[G.m + 2].x, 0.0));
            if (!(q.bn > 0.0)) {
                HIP_OK(hipMemsetAsync(G.X + (int64_t)s * G.n, 0, sizeof(double2) * G.n, G.st));
                G.rel_res[s] = 0.0;
                G.status[s] = FMMBEM_OK;
                q.done = true;
            }
        }
    }

    // ---- restarts: systems between cycles get their true residual (one batched FP64 product)
    void restart_products() {
        const int64_t n = G.n;
        need.clear();
        std::vector<int> prod;
        for (int s = 0; s < G.nv; ++s)
            if (!S[s].done && !S[s].in_cycle) need.push_back(s);
        if (need.empty()) return;
        for (int s : need)
            if (G.x0_given || S[s].cycle > 0) prod.push_back(s);
        for (size_t k = 0; k < prod.size(); ++k)
            HIP_OK(hipMemcpyAsync(Sin + k * n, G.X + (int64_t)prod[k] * n, sizeof(double2) * n,
                                  hipMemcpyDeviceToDevice, G.st));
        if (!prod.empty()) G.matvec_check((int)prod.size(), Sin, Sout);
        for (size_t k = 0; k < prod.size(); ++k) Bl.sub(G.B + (int64_t)prod[k] * n, Sout + k * n, S[prod[k]].r);
        for (int s : need) {
            BatchSys<T> &q = S[s];
            if (!(G.x0_given || q.cycle > 0))
                HIP_OK(hipMemcpyAsync(q.r, G.B + (int64_t)s * n, sizeof(double2) * n, hipMemcpyDeviceToDevice, G.st));
            dots_to(q.r, 0, 1, q.r, res(s) + G.m + 2);
            to_host(s);
        }
    }
    void restart_decide() {
        for (int s : need) {
            BatchSys<T> &q = S[s];
            const double beta = sqrt(std::max(hr(s)[G.m + 2].x, 0.0));
            G.rel_res[s] = beta / q.bn;
            if (!std::isfinite(beta)) {
                G.status[s] = FMMBEM_ENAN;
                q.done = true;
                continue;
            }
            if (G.rel_res[s] < G.tol) {
                G.status[s] = FMMBEM_OK;
                q.done = true;
                continue;
            }
            if (G.iters[s] >= G.maxit) {
                q.done = true;
                continue;
            }
            Bl.scale_copy(1.0 / beta, q.r, q.V);
            std::fill(q.g.begin(), q.g.end(), cmk(0, 0));
            q.g[0] = cmk(beta, 0);
            q.j = 0;
            q.in_cycle = true;
        }
        need.clear();
    }

    // ---- the next batched product of the systems in a cycle
    bool products() {
        const int64_t n = G.n;
        act.clear();
        for (int s = 0; s < G.nv; ++s)
            if (S[s].in_cycle) act.push_back(s);
        if (act.empty()) return false;
        for (size_t k = 0; k < act.size(); ++k) {
            BatchSys<T> &q = S[act[k]];
            if constexpr (wide) {
                G.precond(q.V + (size_t)q.j * n, q.Z + (size_t)q.j * n);
                HIP_OK(hipMemcpyAsync(Sin + k * n, q.Z + (size_t)q.j * n, sizeof(double2) * n,
                                      hipMemcpyDeviceToDevice, G.st));
            } else {
                Bl.widen(q.V + (size_t)q.j * n, tv);
                G.precond(tv, Sin + k * n);
                Bl.scale_copy(1.0, Sin + k * n, q.Z + (size_t)q.j * n);
            }
        }
        G.matvec((int)act.size(), Sin, Sout);
        return true;
    }

    // ---- Arnoldi step of every system in flight, in phases (the host reads between phases)
    // 1: first classical Gram-Schmidt pass: h = V^H w (and |w|^2 for the second-pass test)
    void gs_dots() {
        for (size_t k = 0; k < act.size(); ++k) {
            const int s = act[k];
            BatchSys<T> &q = S[s];
            double2 *w = Sout + k * G.n;
            ++G.iters[s];
            if (G.reorth == 1) dots_to(w, 0, 1, w, res(s) + G.m + 1);
            dots_to(q.V, G.n, q.j + 1, w, res(s));
            to_host(s);
        }
    }
    // 2: w -= V h, then |w|^2
    void gs_update() {
        for (size_t k = 0; k < act.size(); ++k) {
            const int s = act[k];
            BatchSys<T> &q = S[s];
            double2 *w = Sout + k * G.n;
            for (int i = 0; i <= q.j; ++i) q.h1[i] = hr(s)[i];
            k_sub_combo<T><<<ceil_div(G.n, 256), 256, 0, G.st>>>(G.n, q.V, G.n, q.j + 1, res(s), w);
            LAUNCH_OK();
            dots_to(w, 0, 1, w, res(s) + G.m + 2);
            to_host(s);
        }
    }
    // 3: a second pass where the first removed most of w (Daniel-Gragg-Kaufman-Stewart), as in fgmres
    bool gs_second_dots() {
        bool any = false;
        for (size_t k = 0; k < act.size(); ++k) {
            const int s = act[k];
            BatchSys<T> &q = S[s];
            const double w0 = sqrt(std::max(hr(s)[G.m + 1].x, 0.0)), hn = sqrt(std::max(hr(s)[G.m + 2].x, 0.0));
            second[s] = G.reorth == 2 || (G.reorth == 1 && !(hn > 0.7071067811865476 * w0));
            if (!second[s]) continue;
            dots_to(q.V, G.n, q.j + 1, Sout + k * G.n, res(s));
            to_host(s);
            any = true;
        }
        return any;
    }
    void gs_second_update() {
        for (size_t k = 0; k < act.size(); ++k) {
            const int s = act[k];
            if (!second[s]) continue;
            BatchSys<T> &q = S[s];
            double2 *w = Sout + k * G.n;
            for (int i = 0; i <= q.j; ++i) q.h2[i] = hr(s)[i];
            k_sub_combo<T><<<ceil_div(G.n, 256), 256, 0, G.st>>>(G.n, q.V, G.n, q.j + 1, res(s), w);
            LAUNCH_OK();
            dots_to(w, 0, 1, w, res(s) + G.m + 2);
            to_host(s);
        }
    }
    // 4: Hessenberg column, Givens rotations, the next basis vector; at the end of a cycle x += Z y
    void gs_finish() {
        const int m = G.m;
        for (size_t k = 0; k < act.size(); ++k) {
            const int s = act[k];
            BatchSys<T> &q = S[s];
            auto Hc = [&](int i, int jj) -> double2 & { return q.H[(size_t)i * m + jj]; };
            const int j = q.j;
            double2 *w = Sout + k * G.n;
            if (second[s])
                for (int i = 0; i <= j; ++i) q.h1[i] = cadd(q.h1[i], q.h2[i]);
            const double hn = sqrt(std::max(hr(s)[m + 2].x, 0.0));
            for (int i = 0; i <= j; ++i) Hc(i, j) = q.h1[i];
            if (!std::isfinite(hn) || !std::isfinite(hr(s)[m + 2].x)) {
                G.status[s] = FMMBEM_ENAN;
                q.done = true;
                q.in_cycle = false;
                continue;
            }
            Hc(j + 1, j) = cmk(hn, 0);
            if (hn > 0) Bl.scale_copy(1.0 / hn, w, q.V + (size_t)(j + 1) * G.n);
            for (int i = 0; i < j; ++i) {
                double2 a = Hc(i, j), c = Hc(i + 1, j);
                Hc(i, j) = cadd(cscale(a, q.cs[i].x), cmul(q.sn[i], c));
                Hc(i + 1, j) = csub(cscale(c, q.cs[i].x), cmul(cconj(q.sn[i]), a));
            }
            double2 a = Hc(j, j), c = Hc(j + 1, j);
            const double den = hypot(cabs_(a), cabs_(c));
            if (den == 0) {
                q.cs[j] = cmk(1, 0);
                q.sn[j] = cmk(0, 0);
            } else {
                const double aa = cabs_(a);
                q.cs[j] = cmk(aa / den, 0);
                const double2 ph = aa > 0 ? cscale(a, 1.0 / aa) : cmk(1, 0);
                q.sn[j] = cscale(cmul(ph, cconj(c)), 1.0 / den);
            }
            Hc(j, j) = cadd(cscale(a, q.cs[j].x), cmul(q.sn[j], c));
            Hc(j + 1, j) = cmk(0, 0);
            q.g[j + 1] = cscale(cmul(cconj(q.sn[j]), q.g[j]), -1.0);
            q.g[j] = cscale(q.g[j], q.cs[j].x);
            q.est = cabs_(q.g[j + 1]) / q.bn;
            q.j = j + 1;
            if (q.est < G.tol || hn == 0 || q.j == m || G.iters[s] >= G.maxit) {
                // end of cycle: x += Z y with y = H^{-1} g
                const int jj = q.j;
                for (int i = jj - 1; i >= 0; --i) {
                    double2 sum = q.g[i];
                    for (int t = i + 1; t < jj; ++t) sum = csub(sum, cmul(Hc(i, t), q.y[t]));
                    if (cabs_(Hc(i, i)) == 0) throw FmmError(FMMBEM_EBREAKDOWN, "batched solver breakdown");
                    q.y[i] = cdiv(sum, Hc(i, i));
                }
                double2 *hys = hy + (size_t)s * (m + 1);
                for (int i = 0; i < jj; ++i) hys[i] = q.y[i];
                double2 *dys = dy + (size_t)s * (m + 1);
                HIP_OK(hipMemcpyAsync(dys, hys, sizeof(double2) * jj, hipMemcpyHostToDevice, G.st));
                k_add_combo<T><<<ceil_div(G.n, 256), 256, 0, G.st>>>(G.n, q.Z, G.n, jj, dys, G.X + (int64_t)s * G.n);
                LAUNCH_OK();
                q.in_cycle = false;
                ++q.cycle;
                G.restarts[s] = q.cycle;
            }
        }
        // the pinned coefficients of a cycle's end are read by the copies above before the next
        // phase that could rewrite them (a later cycle of the same system, after several waits)
    }
};

// Every phase is enqueued for all groups before the host waits for any, so one host round trip
// serves every system of every group and the groups' kernels overlap on the device.
void fgmres_groups(std::vector<FgmresGroup> &groups) {
    std::vector<GroupSolver<double2>> wide;
    std::vector<GroupSolver<float2>> narrow;
    wide.reserve(groups.size());
    narrow.reserve(groups.size());
    for (auto &g : groups) {
        if (g.basis32) narrow.emplace_back(g);
        else wide.emplace_back(g);
    }
    auto all = [&](auto &&f) {
        for (auto &g : wide) f(g);
        for (auto &g : narrow) f(g);
    };
    auto any_of = [&](auto &&f) {
        bool r = false;
        for (auto &g : wide) r = f(g) || r;
        for (auto &g : narrow) r = f(g) || r;
        return r;
    };
    auto wait_all = [&]() { all([](auto &g) { g.wait(); }); };
    all([](auto &g) { g.init(); });
    wait_all();
    all([](auto &g) { g.init_done(); });
    all([](auto &g) { g.restart_products(); });
    wait_all();
    all([](auto &g) { g.restart_decide(); });
    while (any_of([](auto &g) { return g.products(); })) {
        all([](auto &g) { g.gs_dots(); });
        wait_all();
        all([](auto &g) { g.gs_update(); });
        wait_all();
        if (any_of([](auto &g) { return g.gs_second_dots(); })) {
            wait_all();
            all([](auto &g) { g.gs_second_update(); });
            wait_all();
        }
        all([](auto &g) { g.gs_finish(); });
        all([](auto &g) { g.restart_products(); });
        wait_all();
        all([](auto &g) { g.restart_decide(); });
    }
    wait_all();
    all([](auto &g) { HIP_OK(hipStreamSynchronize(g.G.st)); });
}

int fgmres_batch(int64_t n, hipStream_t st, DeviceBuffers &scr, int nv,
                 const std::function<void(int, const double2 *, double2 *)> &matvec,
                 const std::function<void(int, const double2 *, double2 *)> &matvec_check,
                 const std::function<void(const double2 *, double2 *)> &precond, const double2 *B, double2 *X,
                 double tol, int m, int maxit, bool x0_given, std::vector<int> &iters, std::vector<int> &restarts,
                 std::vector<double> &rel_res, std::vector<int> &status, bool basis32, int reorth) {
    std::vector<FgmresGroup> g(1);
    FgmresGroup &q = g[0];
    q.n = n;
    q.st = st;
    q.scr = &scr;
    q.nv = nv;
    q.matvec = matvec;
    q.matvec_check = matvec_check;
    q.precond = precond;
    q.B = B;
    q.X = X;
    q.tol = tol;
    q.m = m;
    q.maxit = maxit;
    q.x0_given = x0_given;
    q.basis32 = basis32;
    q.reorth = reorth;
    fgmres_groups(g);
    iters = q.iters;
    restarts = q.restarts;
    rel_res = q.rel_res;
    status = q.status;
    return FMMBEM_OK;
}

}  // namespace fmm
