// FMM matrix-vector product of the direct BIE (Eq. dbem4) on one GPU, FP64 path.
//
// The product y = 1/2 x + L[sigma] + M[mu] at the element centroids, with single-layer density
// sigma = -i k beta x and double-layer density mu = x, is split as in Section 3.3:
//   near  : pairs closer than r_c (and the self pair) use accurate integrals, stored once per
//           (mesh, k) in a CSR table; all other pairs in neighbouring leaves use the one-point
//           rule, evaluated on the fly (P2P);
//   far   : boxes that are well separated exchange multipole/local expansions of Eq. (shft0):
//           P2M at the leaves, M2M up, M2L across, L2L down, L2P at the leaves.  Every
//           translation is rotation - coaxial translation - back-rotation (Section 3.3); the
//           coaxial coefficients come from the stabilised recursion, the rotations from the
//           quarter-turn matrices Delta^n (tables.hip).
//
// Expansion conventions (what the tables and the kernels below share):
//   G(x,y) = i k sum_{n,m} R_n^{-m}(y - C) S_n^m(x - C),  |x - C| > |y - C|,
//   multipole of a box: psi(x) = sum C_n^m S_n^m(x - C); local: psi(x) = sum D_n^m R_n^m(x - C).
//   Y_n^m orthonormal with P_n^|m| without the Condon-Shortley phase (Y_n^{-m} = conj Y_n^m).
// Rotation to align t = |t|(sin b cos a, sin b sin a, cos b) with +z, on a coefficient column c:
//   c <- e^{i m a} (-i)^m c ;  c <- Delta^T c ;  c <- e^{i m b} c ;  c <- Delta c ;  [ * i^m ]
// and back after the coaxial step:
//   [ * (-i)^m ] ;  d <- Delta^T d ;  d <- e^{-i m b} d ;  d <- Delta d ;  d <- i^m e^{-i m a} d.
// The bracketed phases cancel across the coaxial step (which is diagonal in m) and are omitted.
#include "internal.h"

namespace fmm {

__constant__ double GL8X[8] = {-0.96028985649753618, -0.79666647741362673, -0.52553240991632899,
                               -0.18343464249564978, 0.18343464249564978,  0.52553240991632899,
                               0.79666647741362673,  0.96028985649753618};
__constant__ double GL8W[8] = {0.10122853629037669, 0.22238103445337434, 0.31370664587788705,
                               0.36268378337836177, 0.36268378337836177, 0.31370664587788705,
                               0.22238103445337434, 0.10122853629037669};

// sin and cos of x for |x| <= 1e5 (k r of element pairs): x = q pi/2 + y with pi/2 split in two
// parts (Cody-Waite), |y| <= pi/4, then the Taylor polynomials of sin y through y^17 and of cos y
// through y^16 (truncation below 1e-17); the absolute error is a few 1e-16.  Larger arguments use
// the library routine.
__device__ inline void sincos_red(double x, double &s, double &c) {
    if (!(fabs(x) <= 1e5)) {
        sincos(x, &s, &c);
        return;
    }
    const double q = rint(x * 0.63661977236758134308);
    double y = fma(-q, 1.5707963267948966, x);
    y = fma(-q, 6.123233995736766e-17, y);
    // sum_i w^i / (2i+1)!  and  sum_i w^i / (2i)!, w = -y^2, as sums of coefficient x power from the
    // smallest term up: the powers are shared by both sums, and every step adds into its own
    // accumulator (Horner's steps add a constant held in a register, which the generated code copied
    // into the destination first: one more instruction per step); same accuracy (1.5e-16 absolute
    // against extended precision for |x| <= 1e5)
    const double w = -y * y, w2 = w * w, w3 = w2 * w, w4 = w2 * w2, w5 = w4 * w, w6 = w3 * w3, w7 = w4 * w3,
                 w8 = w4 * w4;
    double ts = w8 * (1.0 / 355687428096000.0);
    ts = fma(1.0 / 1307674368000.0, w7, ts);
    ts = fma(1.0 / 6227020800.0, w6, ts);
    ts = fma(1.0 / 39916800.0, w5, ts);
    ts = fma(1.0 / 362880.0, w4, ts);
    ts = fma(1.0 / 5040.0, w3, ts);
    ts = fma(1.0 / 120.0, w2, ts);
    ts = fma(1.0 / 6.0, w, ts);
    ts += 1.0;
    double tc = w8 * (1.0 / 20922789888000.0);
    tc = fma(1.0 / 87178291200.0, w7, tc);
    tc = fma(1.0 / 479001600.0, w6, tc);
    tc = fma(1.0 / 3628800.0, w5, tc);
    tc = fma(1.0 / 40320.0, w4, tc);
    tc = fma(1.0 / 720.0, w3, tc);
    tc = fma(1.0 / 24.0, w2, tc);
    tc = fma(0.5, w, tc);
    tc += 1.0;
    const double sy = y * ts, cy = tc;
    const int iq = (int)q & 3;
    const double a = (iq & 1) ? cy : sy, b = (iq & 1) ? sy : cy;  // sin and cos before the signs
    s = (iq & 2) ? -a : a;
    c = ((iq + 1) & 2) ? -b : b;
}

// ------------------------------------------------------------------ accurate element integrals
// L = int_T G(x,y) dS_y and M = int_T dG/dn_y dS_y for a flat triangle, by polar coordinates
// about the projection x_p of x on the triangle's plane.  With h the signed height of x and
// r^2 = rho^2 + h^2 the radial integrals are exact:
//   int_0^{rho_e} G rho drho        = (e^{ikR} - e^{ik|h|}) / (4 pi i k)
//   int_0^{rho_e} dG/dn_y rho drho  = -h/(4 pi) (e^{ikR}/R - e^{ik|h|}/|h|),   R = r(rho_e)
// leaving an angular integral per edge (signed by the edge orientation seen from x_p), done by
// 8 panels x 8-point Gauss-Legendre after the substitution tan(psi) = sinh(w).
// self != 0: x is the triangle's centroid (h = 0, M = 0 by the principal value).
__device__ void tri_integrals(const double *x, const double *v, double k, int self, double2 &Lout, double2 &Mout) {
    double e1[3] = {v[3] - v[0], v[4] - v[1], v[5] - v[2]};
    double e2[3] = {v[6] - v[0], v[7] - v[1], v[8] - v[2]};
    double nn[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2], e1[0] * e2[1] - e1[1] * e2[0]};
    double nl = sqrt(nn[0] * nn[0] + nn[1] * nn[1] + nn[2] * nn[2]);
    nn[0] /= nl;
    nn[1] /= nl;
    nn[2] /= nl;
    double h = self ? 0.0 : (x[0] - v[0]) * nn[0] + (x[1] - v[1]) * nn[1] + (x[2] - v[2]) * nn[2];
    double xp[3] = {x[0] - h * nn[0], x[1] - h * nn[1], x[2] - h * nn[2]};
    double ah = fabs(h);
    double2 Lacc = cmk(0, 0), Macc = cmk(0, 0);
    double span = 0.0;
    for (int e = 0; e < 3; ++e) {
        int e2i = (e + 1) % 3;
        double a[3] = {v[3 * e] - xp[0], v[3 * e + 1] - xp[1], v[3 * e + 2] - xp[2]};
        double b[3] = {v[3 * e2i] - xp[0], v[3 * e2i + 1] - xp[1], v[3 * e2i + 2] - xp[2]};
        double ed[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]};
        double le = sqrt(ed[0] * ed[0] + ed[1] * ed[1] + ed[2] * ed[2]);
        double eh[3] = {ed[0] / le, ed[1] / le, ed[2] / le};
        double s0 = a[0] * eh[0] + a[1] * eh[1] + a[2] * eh[2];
        double s1 = b[0] * eh[0] + b[1] * eh[1] + b[2] * eh[2];
        double f[3] = {a[0] - s0 * eh[0], a[1] - s0 * eh[1], a[2] - s0 * eh[2]};
        double d = sqrt(f[0] * f[0] + f[1] * f[1] + f[2] * f[2]);
        if (d <= 1e-13 * le) continue;
        double cr[3] = {a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2], a[0] * b[1] - a[1] * b[0]};
        double sgn = (cr[0] * nn[0] + cr[1] * nn[1] + cr[2] * nn[2]) >= 0.0 ? 1.0 : -1.0;
        span += sgn * (atan2(s1, d) - atan2(s0, d));
        // angle psi from the edge normal, substituted tan(psi) = sinh(w): rho = d cosh(w),
        // dpsi = dw / cosh(w); this grades the panels logarithmically along edges that are long
        // compared with their distance d from x_p, where the integrand varies fastest
        const double w0 = asinh(s0 / d), w1 = asinh(s1 / d);
        const int NPAN = 8;
        double hw = 0.5 * (w1 - w0) / NPAN;
        for (int pan = 0; pan < NPAN; ++pan) {
            double mid = w0 + (2 * pan + 1) * hw;
            for (int q = 0; q < 8; ++q) {
                double ww = mid + hw * GL8X[q];
                double ch = cosh(ww);
                double w = sgn * hw * GL8W[q] / ch;
                double rho = d * ch;
                double R = sqrt(rho * rho + h * h);
                double dR = R - ah;
                // z = k dR from its half angle: sin z = 2 s c and 1 - cos z = 2 s^2 (no cancellation
                // at small z); the radial L integral is e^{ik|h|} (sin z + i (1 - cos z)) / k and
                // e^{ikR} = e^{ik|h|} e^{iz}, the common factor e^{ik|h|} taken once at the end
                double s, c;
                sincos_red(0.5 * k * dR, s, c);
                const double sz = 2.0 * s * c, omc = 2.0 * s * s;
                Lacc = cadd(Lacc, cmk(w * sz, w * omc));
                Macc = cadd(Macc, cscale(cmk(1.0 - omc, sz), w / R));
            }
        }
    }
    double sh, ch;
    sincos(k * ah, &sh, &ch);
    double2 eh_ = cmk(ch, sh);
    Lout = cscale(cmul(eh_, Lacc), 1.0 / (4.0 * FMM_PI * k));
    if (h == 0.0) {
        Mout = cmk(0, 0);
    } else {
        double sgh = h > 0 ? 1.0 : -1.0;
        Mout = cadd(cscale(cmul(eh_, Macc), -h / (4.0 * FMM_PI)), cscale(eh_, sgh * span / (4.0 * FMM_PI)));
    }
}

// L' = int_T dG/dn_x dS and M' = d/dn_x int_T dG/dn_y dS for the indirect formulation
// (Eq. ibem3), from the surface divergence theorem on the flat triangle (normal n, edges with
// unit tangent tau running counter-clockwise about n, outward in-plane normal nu = tau x n):
//   grad_x L = -n M - sum_e nu_e int_e G dl,                so L' = -(n_x.n) M - sum_e (n_x.nu_e) I0_e
//   n_x.grad_x M = k^2 (n_x.n) L + sum_e c_e int_e G (ikr - 1)/r^2 dl,  c_e = (f_e - x).(tau_e x n_x)
// with f_e the foot of the perpendicular from x on the edge line; (y - x).(tau x n_x) is constant
// along the edge, which makes the second line integral scalar.  On the element itself
// (n_x = n) this is the Hadamard finite part; L' = 0 there.  The edge integrals use
// s = d sinh(w) (d = distance from x to the edge line, ds = r dw), 8 panels x 8 points.
__device__ void tri_integrals_n(const double *x, const double *nx, const double *v, double k, int self, double2 &L,
                                double2 &M, double2 &Lp, double2 &Mp) {
    tri_integrals(x, v, k, self, L, M);
    double e1[3] = {v[3] - v[0], v[4] - v[1], v[5] - v[2]};
    double e2[3] = {v[6] - v[0], v[7] - v[1], v[8] - v[2]};
    double nn[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2], e1[0] * e2[1] - e1[1] * e2[0]};
    double nl = sqrt(nn[0] * nn[0] + nn[1] * nn[1] + nn[2] * nn[2]);
    for (int q = 0; q < 3; ++q) nn[q] /= nl;
    const double nxn = nx[0] * nn[0] + nx[1] * nn[1] + nx[2] * nn[2];
    double2 lp = cscale(M, -nxn), mp = cscale(L, k * k * nxn);
    for (int e = 0; e < 3; ++e) {
        const int eb = (e + 1) % 3;
        const double a[3] = {v[3 * e], v[3 * e + 1], v[3 * e + 2]}, b[3] = {v[3 * eb], v[3 * eb + 1], v[3 * eb + 2]};
        double tau[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]};
        const double le = sqrt(tau[0] * tau[0] + tau[1] * tau[1] + tau[2] * tau[2]);
        for (int q = 0; q < 3; ++q) tau[q] /= le;
        const double nu[3] = {tau[1] * nn[2] - tau[2] * nn[1], tau[2] * nn[0] - tau[0] * nn[2], tau[0] * nn[1] - tau[1] * nn[0]};
        const double tn[3] = {tau[1] * nx[2] - tau[2] * nx[1], tau[2] * nx[0] - tau[0] * nx[2], tau[0] * nx[1] - tau[1] * nx[0]};
        const double ax[3] = {a[0] - x[0], a[1] - x[1], a[2] - x[2]};
        const double s0 = ax[0] * tau[0] + ax[1] * tau[1] + ax[2] * tau[2], s1 = s0 + le;
        const double fx[3] = {ax[0] - s0 * tau[0], ax[1] - s0 * tau[1], ax[2] - s0 * tau[2]};  // f - x
        const double d = sqrt(fx[0] * fx[0] + fx[1] * fx[1] + fx[2] * fx[2]);
        const double ce = fx[0] * tn[0] + fx[1] * tn[1] + fx[2] * tn[2];
        const double cnu = nx[0] * nu[0] + nx[1] * nu[1] + nx[2] * nu[2];
        double2 I0 = cmk(0, 0), I2 = cmk(0, 0);
        const int NPAN = 8;
        if (d > 1e-9 * le) {
            const double w0 = asinh(s0 / d), w1 = asinh(s1 / d), hw = 0.5 * (w1 - w0) / NPAN;
            for (int pan = 0; pan < NPAN; ++pan) {
                const double mid = w0 + (2 * pan + 1) * hw;
                for (int q = 0; q < 8; ++q) {
                    const double r = d * cosh(mid + hw * GL8X[q]);
                    const double wt = hw * GL8W[q] * r;  // ds = r dw
                    double sn, cs;
                    sincos(k * r, &sn, &cs);
                    const double2 G = cmk(cs / (4.0 * FMM_PI * r), sn / (4.0 * FMM_PI * r));
                    I0 = cadd(I0, cscale(G, wt));
                    I2 = cadd(I2, cscale(cmul(G, cmk(-1.0, k * r)), wt / (r * r)));
                }
            }
        } else {
            // x on the edge's line (outside the segment): c_e = 0; plain panels in s for I0
            const double hs = 0.5 * (s1 - s0) / NPAN;
            for (int pan = 0; pan < NPAN; ++pan) {
                const double mid = s0 + (2 * pan + 1) * hs;
                for (int q = 0; q < 8; ++q) {
                    const double r = fabs(mid + hs * GL8X[q]);
                    double sn, cs;
                    sincos(k * r, &sn, &cs);
                    I0 = cadd(I0, cscale(cmk(cs, sn), hs * GL8W[q] / (4.0 * FMM_PI * r)));
                }
            }
        }
        lp = csub(lp, cscale(I0, cnu));
        mp = cadd(mp, cscale(I2, ce));
    }
    Lp = self ? cmk(0, 0) : lp;
    Mp = mp;
}

__global__ void k_near_quad_n(int64_t nnz, const int32_t *rowv, const int32_t *col, const double4 *ec,
                              const double4 *en, const double *ev, double k, double2 *Lpv, double2 *Mpv) {
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= nnz) return;
    int i = rowv[e], j = col[e];
    double4 ci = ec[i], ni = en[i];
    double x[3] = {ci.x, ci.y, ci.z}, nx[3] = {ni.x, ni.y, ni.z}, v[9];
    for (int q = 0; q < 9; ++q) v[q] = ev[9 * (int64_t)j + q];
    double2 L, M, Lp, Mp;
    tri_integrals_n(x, nx, v, k, i == j, L, M, Lp, Mp);
    Lpv[e] = Lp;
    Mpv[e] = Mp;
}

// ------------------------------------------------------------------ near-field table
__global__ void k_near_count(int64_t n, const int32_t *leaf_of, const int32_t *leaf_start, const int32_t *nbr_start,
                             const int32_t *nbr_list, const double4 *ec, double rc2, int32_t *cnt) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double4 ci = ec[i];
    int b = leaf_of[i], c = 0;
    for (int q = nbr_start[b]; q < nbr_start[b + 1]; ++q) {
        int sb = nbr_list[q];
        for (int j = leaf_start[sb]; j < leaf_start[sb + 1]; ++j) {
            double4 cj = ec[j];
            if (j == i || dist2_exact(ci.x, ci.y, ci.z, cj.x, cj.y, cj.z) < rc2) ++c;
        }
    }
    cnt[i] = c;
}

__global__ void k_near_fill(int64_t n, const int32_t *leaf_of, const int32_t *leaf_start, const int32_t *nbr_start,
                            const int32_t *nbr_list, const double4 *ec, double rc2, const int32_t *start,
                            int32_t *rowv, int32_t *col) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double4 ci = ec[i];
    int b = leaf_of[i], o = start[i];
    for (int q = nbr_start[b]; q < nbr_start[b + 1]; ++q) {
        int sb = nbr_list[q];
        for (int j = leaf_start[sb]; j < leaf_start[sb + 1]; ++j) {
            double4 cj = ec[j];
            if (j == i || dist2_exact(ci.x, ci.y, ci.z, cj.x, cj.y, cj.z) < rc2) {
                rowv[o] = (int32_t)i;
                col[o++] = j;
            }
        }
    }
}

__global__ void k_near_quad(int64_t nnz, const int32_t *rowv, const int32_t *col, const double4 *ec, const double *ev,
                            double k, double2 *Lv, double2 *Mv) {
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= nnz) return;
    int i = rowv[e], j = col[e];
    double4 ci = ec[i];
    double x[3] = {ci.x, ci.y, ci.z}, v[9];
    for (int q = 0; q < 9; ++q) v[q] = ev[9 * (int64_t)j + q];
    double2 L, M;
    tri_integrals(x, v, k, i == j, L, M);
    Lv[e] = L;
    Mv[e] = M;
}

// ------------------------------------------------------------------ densities
// sigma_i = -i k beta_i x_i, mu_i = x_i (sorted order; x in caller order)
// nr right-hand sides: x is nr x N in caller order; sigma/mu interleaved, [i * nr + r] in tree order
__global__ void k_densities(int64_t n, int nr, const int32_t *perm, const double2 *x, const double2 *beta, double k,
                            double2 *sigma, double2 *mu) {
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n * nr) return;
    const int64_t i = e / nr;
    const int r = (int)(e - i * nr);
    double2 xi = x[(int64_t)r * n + perm[i]];
    double2 bx = cmul(beta[i], xi);
    sigma[e] = cmk(k * bx.y, -k * bx.x);  // -i k (beta x)
    mu[e] = xi;
}

// gamma_i = -dpsi_in/dn + i k beta psi_in at centroid i for a monopole of amplitude amp at rs (Eq. sp7)
__global__ void k_gamma(int64_t n, const double4 *ec, const double4 *en, const double2 *beta, double k, double sx,
                        double sy, double sz, double2 amp, double2 *sigma, double2 *mu) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double4 c = ec[i], nv = en[i];
    double dx = c.x - sx, dy = c.y - sy, dz = c.z - sz;
    double r = sqrt(dx * dx + dy * dy + dz * dz);
    double s, co;
    sincos(k * r, &s, &co);
    double2 G = cmul(amp, cmk(co / (4 * FMM_PI * r), s / (4 * FMM_PI * r)));
    double proj = (dx * nv.x + dy * nv.y + dz * nv.z) / (r * r);
    double2 dG = cscale(cmul(G, cmk(-1.0, k * r)), proj);      // G (ikr - 1) (x - rs).n / r^2
    double2 ikb = cmk(-k * beta[i].y, k * beta[i].x);          // i k beta
    sigma[i] = csub(cmul(ikb, G), dG);
    mu[i] = cmk(0, 0);
}

// ------------------------------------------------------------------ pair-kernel helpers
// 1/sqrt(d) for a positive, normal d: hardware estimate and two Newton steps (about an ulp)
__device__ inline double rsq_nr(double d) {
    double y = __builtin_amdgcn_rsq(d);
    double e = fma(-d * y, y, 1.0);
    y = fma(0.5 * y, e, y);
    e = fma(-d * y, y, 1.0);
    return fma(0.5 * y, e, y);
}

// ------------------------------------------------------------------ P2P + near table
// y_i = sum_{j in neighbour leaves, |c_i - c_j| >= r_c} [G q_j + dG/dn_y w_j] + sum_near [L sigma + M mu]
// with q_j = A_j sigma_j, w_j = A_j mu_j.  One workgroup (one wavefront) per target leaf,
// source tiles staged in LDS.  A small leaf splits every source tile over S groups of lanes, one
// target per lane of a group, and adds the groups' sums at the end.
// Source splits S of a leaf of nt targets: lane groups of TP = floor(64 / S) targets, each group
// summing every S-th source, ceil(nt / TP) passes over the sources; S in 1..8 minimises the lane
// work ceil(nt / TP) / S (ties to the smaller S, which adds fewer partial sums).  Lanes past S TP
// (S = 3, 5, 6, 7) stay idle.
__device__ inline int p2p_splits(int nt) {
    int best = 1;
    double bc = 1e30;
    for (int S = 1; S <= 8; ++S) {
        const int TP = 64 / S;
        const double c = (double)((nt + TP - 1) / TP) / S;
        if (c < bc - 1e-12) {
            bc = c;
            best = S;
        }
    }
    return best;
}

template <int NR>
__global__ void __launch_bounds__(64) k_p2p(int nleaf, const int32_t *leaf_start, const int32_t *nbr_start,
                                            const int32_t *nbr_list, int all_leaves, const double4 *ec,
                                            const double4 *en, const double2 *sigma, const double2 *mu, double k,
                                            double rc2, const int32_t *near_start, const int32_t *near_col,
                                            const double2 *nL, const double2 *nM, double2 *y) {
    const int b = blockIdx.x, tid = threadIdx.x;
    __shared__ double sx[64], sy[64], sz[64], snx[64], sny[64], snz[64];
    __shared__ double2 sq[64 * NR], sw[64 * NR];
    __shared__ double2 red[64 * NR];
    const int ts = leaf_start[b], te = leaf_start[b + 1];
    const int nb0 = all_leaves ? 0 : nbr_start[b], nb1 = all_leaves ? nleaf : nbr_start[b + 1];
    const double inv4pi = 1.0 / (4.0 * FMM_PI);
    const int S = p2p_splits(te - ts), TP = 64 / S;  // source splits, targets per pass
    const int h = tid / TP;
    for (int t0 = ts; t0 < te; t0 += TP) {
        const int t = t0 + tid % TP;
        const bool act = t < te && h < S;
        double4 ct = act ? ec[t] : make_double4(0, 0, 0, 0);
        double2 acc[NR];
#pragma unroll
        for (int r = 0; r < NR; ++r) acc[r] = cmk(0, 0);
        for (int q = nb0; q < nb1; ++q) {
            const int sb = all_leaves ? q : nbr_list[q];
            const int ss = leaf_start[sb], se = leaf_start[sb + 1];
            for (int j0 = ss; j0 < se; j0 += 64) {
                __syncthreads();
                int j = j0 + tid;
                if (j < se) {
                    double4 c = ec[j], nv = en[j];
                    sx[tid] = c.x;
                    sy[tid] = c.y;
                    sz[tid] = c.z;
                    snx[tid] = nv.x;
                    sny[tid] = nv.y;
                    snz[tid] = nv.z;
#pragma unroll
                    for (int r = 0; r < NR; ++r) {
                        sq[tid * NR + r] = cscale(sigma[(int64_t)j * NR + r], c.w);
                        sw[tid * NR + r] = cscale(mu[(int64_t)j * NR + r], c.w);
                    }
                }
                __syncthreads();
                const int cnt = min(64, se - j0);
                if (act) {
                    for (int jj = h; jj < cnt; jj += S) {
                        double d2 = dist2_exact(ct.x, ct.y, ct.z, sx[jj], sy[jj], sz[jj]);
                        if (d2 < rc2) continue;
                        double dx = sx[jj] - ct.x, dy = sy[jj] - ct.y, dz = sz[jj] - ct.z;
                        const double ir = rsq_nr(d2), r = d2 * ir;
                        double s, c;
                        sincos_red(k * r, s, c);
                        double2 G = cmk(c * ir * inv4pi, s * ir * inv4pi);
                        double u = (dx * snx[jj] + dy * sny[jj] + dz * snz[jj]) * ir * ir;  // (y-x).n / r^2
                        // G * (q + (ikr - 1) u w)
                        const double2 f = cmk(-u, k * r * u);
#pragma unroll
                        for (int rr = 0; rr < NR; ++rr) {
                            double2 t2 = cmul(f, sw[jj * NR + rr]);
                            acc[rr] = cfma(G, cadd(sq[jj * NR + rr], t2), acc[rr]);
                        }
                    }
                }
            }
        }
        if (act) {
            for (int e = near_start[t] + h; e < near_start[t + 1]; e += S) {
                const int64_t j = near_col[e];
                const double2 l = nL[e], m = nM[e];
#pragma unroll
                for (int rr = 0; rr < NR; ++rr) {
                    acc[rr] = cfma(l, sigma[j * NR + rr], acc[rr]);
                    acc[rr] = cfma(m, mu[j * NR + rr], acc[rr]);
                }
            }
        }
        if (S > 1) {  // add the groups' partial sums (group 0 keeps the result)
            __syncthreads();
#pragma unroll
            for (int rr = 0; rr < NR; ++rr) red[tid * NR + rr] = acc[rr];
            __syncthreads();
            if (h == 0)
                for (int g = 1; g < S; ++g)
#pragma unroll
                    for (int rr = 0; rr < NR; ++rr) acc[rr] = cadd(acc[rr], red[(tid + g * TP) * NR + rr]);
        }
        if (act && h == 0) {
#pragma unroll
            for (int rr = 0; rr < NR; ++rr) y[(int64_t)t * NR + rr] = acc[rr];
        }
    }
}

// ------------------------------------------------------------------ P2P, FP32 arithmetic
// Mixed-precision near field: the near/far classification uses the exact FP64 squared distance
// (so it matches the near table), the kernel evaluation runs in FP32, and the accumulation is
// Kahan-compensated in FP32.  Near-table entries are stored in FP32.
__device__ inline void kahan_add(float &s, float &c, float v) {
    const float y = v - c;
    const float t = s + y;
    c = (t - s) - y;
    s = t;
}

template <int NR>
__global__ void __launch_bounds__(64) k_p2p32(int nleaf, const int32_t *leaf_start, const int32_t *nbr_start,
                                              const int32_t *nbr_list, const double4 *ec, const double4 *en,
                                              const double2 *sigma, const double2 *mu, double k, double rc2,
                                              const int32_t *near_start, const int32_t *near_col, const float2 *nL,
                                              const float2 *nM, double2 *y) {
    const int b = blockIdx.x, tid = threadIdx.x;
    __shared__ double sx[64], sy[64], sz[64];
    __shared__ float snx[64], sny[64], snz[64];
    __shared__ float2 sq[64 * NR], sw[64 * NR];
    __shared__ double2 red[64 * NR];
    const int ts = leaf_start[b], te = leaf_start[b + 1];
    const float kf = (float)k, inv4pi = (float)(1.0 / (4.0 * FMM_PI));
    const int S = p2p_splits(te - ts), TP = 64 / S;  // source splits, targets per pass (as in k_p2p)
    const int h = tid / TP;
    for (int t0 = ts; t0 < te; t0 += TP) {
        const int t = t0 + tid % TP;
        const bool act = t < te && h < S;
        double4 ct = act ? ec[t] : make_double4(0, 0, 0, 0);
        float ar[NR], ai[NR], cr[NR], ci[NR];
#pragma unroll
        for (int r = 0; r < NR; ++r) ar[r] = ai[r] = cr[r] = ci[r] = 0.f;
        for (int q = nbr_start[b]; q < nbr_start[b + 1]; ++q) {
            const int sb = nbr_list[q];
            const int ss = leaf_start[sb], se = leaf_start[sb + 1];
            for (int j0 = ss; j0 < se; j0 += 64) {
                __syncthreads();
                int j = j0 + tid;
                if (j < se) {
                    double4 c = ec[j], nv = en[j];
                    sx[tid] = c.x;
                    sy[tid] = c.y;
                    sz[tid] = c.z;
                    snx[tid] = (float)nv.x;
                    sny[tid] = (float)nv.y;
                    snz[tid] = (float)nv.z;
#pragma unroll
                    for (int r = 0; r < NR; ++r) {
                        const double2 s = sigma[(int64_t)j * NR + r], m = mu[(int64_t)j * NR + r];
                        sq[tid * NR + r] = make_float2((float)(s.x * c.w), (float)(s.y * c.w));
                        sw[tid * NR + r] = make_float2((float)(m.x * c.w), (float)(m.y * c.w));
                    }
                }
                __syncthreads();
                const int cnt = min(64, se - j0);
                if (act) {
                    for (int jj = h; jj < cnt; jj += S) {
                        double d2 = dist2_exact(ct.x, ct.y, ct.z, sx[jj], sy[jj], sz[jj]);
                        if (d2 < rc2) continue;
                        const float dx = (float)(sx[jj] - ct.x), dy = (float)(sy[jj] - ct.y), dz = (float)(sz[jj] - ct.z);
                        const float r2 = (float)d2, ir = rsqrtf(r2), r = r2 * ir;
                        float s, c;
                        sincosf(kf * r, &s, &c);
                        const float gr = c * ir * inv4pi, gi = s * ir * inv4pi;
                        const float u = (dx * snx[jj] + dy * sny[jj] + dz * snz[jj]) * ir * ir;
                        const float kru = kf * r * u;
#pragma unroll
                        for (int rr = 0; rr < NR; ++rr) {
                            // G * (q + (ikr - 1) u w)
                            const float2 w = sw[jj * NR + rr], qq = sq[jj * NR + rr];
                            const float tr = qq.x - u * w.x - kru * w.y;
                            const float ti = qq.y - u * w.y + kru * w.x;
                            kahan_add(ar[rr], cr[rr], gr * tr - gi * ti);
                            kahan_add(ai[rr], ci[rr], gr * ti + gi * tr);
                        }
                    }
                }
            }
        }
        double2 acc[NR];
#pragma unroll
        for (int rr = 0; rr < NR; ++rr) acc[rr] = make_double2((double)ar[rr] - (double)cr[rr], (double)ai[rr] - (double)ci[rr]);
        if (act) {
            for (int e = near_start[t] + h; e < near_start[t + 1]; e += S) {
                const int64_t j = near_col[e];
                const float2 l = nL[e], m = nM[e];
                const double2 ld = make_double2(l.x, l.y), md = make_double2(m.x, m.y);
#pragma unroll
                for (int rr = 0; rr < NR; ++rr) {
                    acc[rr] = cfma(ld, sigma[j * NR + rr], acc[rr]);
                    acc[rr] = cfma(md, mu[j * NR + rr], acc[rr]);
                }
            }
        }
        if (S > 1) {  // add the groups' partial sums (group 0 keeps the result)
            __syncthreads();
#pragma unroll
            for (int rr = 0; rr < NR; ++rr) red[tid * NR + rr] = acc[rr];
            __syncthreads();
            if (h == 0)
                for (int g = 1; g < S; ++g)
#pragma unroll
                    for (int rr = 0; rr < NR; ++rr) acc[rr] = cadd(acc[rr], red[(tid + g * TP) * NR + rr]);
        }
        if (act && h == 0) {
#pragma unroll
            for (int rr = 0; rr < NR; ++rr) y[(int64_t)t * NR + rr] = acc[rr];
        }
    }
}

__global__ void k_zero8(int64_t n, uint64_t *p) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

__global__ void k_cvt_d2f(int64_t n, const double2 *a, float2 *b) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) b[i] = make_float2((float)a[i].x, (float)a[i].y);
}
__global__ void k_cvt_f2d(int64_t n, const float2 *a, double2 *b) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) b[i] = make_double2(a[i].x, a[i].y);
}
__global__ void k_cvt_real_d2f(int64_t n, const double *a, float *b) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) b[i] = (float)a[i];
}

// ------------------------------------------------------------------ regular-basis helpers
// reciprocal of a positive, normal double: hardware estimate and two Newton steps (within an ulp)
__device__ inline double rcp_nr(double d) {
    double y = __builtin_amdgcn_rcp(d);
    double e = fma(-d, y, 1.0);
    y = fma(y, e, y);
    e = fma(-d, y, 1.0);
    return fma(y, e, y);
}

// sum of the power series of x^{-n} (2n+1)!! j_n(x): t_0 = 1, t_k = t_{k-1} h / (k (2n+2k+1)), h = -x^2/2
__device__ inline double jn_series(int n, double h, int kmax) {
    double s = 1.0, t = 1.0;
    for (int q = 1; q <= kmax; ++q) {
        t *= h * rcp_nr((double)q * (double)(2 * n + 2 * q + 1));
        s += t;
        if (fabs(t) <= 1e-17 * fabs(s)) break;
    }
    return s;
}

// j_0(x) .. j_N(x), x >= 0.  Small x: every order from its series (orders that underflow are
// zero to working precision).  x < 4 and N <= 40: j_N and j_{N-1} from their series, then the
// downward recurrence j_{n-1} = (2n+1)/x j_n - j_{n+1}, which is stable for this (minimal)
// solution.  Otherwise Miller's normalised recurrence.
__device__ inline void bessel_j_seq(double x, int N, double *j) {
    const double h = -0.5 * x * x;
    if (x < 1e-2) {
        double pre = 1.0;  // x^n / (2n+1)!!
        for (int n = 0; n <= N; ++n) {
            if (n > 0) pre *= x * rcp_nr(2.0 * n + 1.0);
            j[n] = pre * jn_series(n, h, 6);
        }
        return;
    }
    if (x >= 4.0 || N > 40) {
        sph_jn_seq(x, N, j);
        return;
    }
    if (N == 0) {
        j[0] = jn_series(0, h, 40);
        return;
    }
    double xn = 1.0, df = 1.0;  // x^{N-1} and (2N-1)!!
    for (int n = 1; n < N; ++n) {
        xn *= x;
        df *= 2.0 * n + 1.0;
    }
    const double pre = xn / df;
    double jh = pre * x / (2.0 * N + 1.0) * jn_series(N, h, 40);
    double jl = pre * jn_series(N - 1, h, 40);
    j[N] = jh;
    j[N - 1] = jl;
    const double ix = 1.0 / x;
    for (int n = N - 1; n >= 1; --n) {
        const double jm = fma((2.0 * n + 1.0) * ix, jl, -jh);
        j[n - 1] = jm;
        jh = jl;
        jl = jm;
    }
}

// spherical coordinates of (dx, dy, dz) about the expansion centre: r, cos/sin of the polar
// angle and e^{i phi} (any unit phase where the point lies on the axis: the orders m != 0 vanish)
__device__ inline void sph_frame(double dx, double dy, double dz, double &r, double &ct, double &st, double2 &eph) {
    const double rxy2 = dx * dx + dy * dy;
    r = sqrt(rxy2 + dz * dz);
    const double rxy = sqrt(rxy2);
    if (r > 0) {
        const double ir = 1.0 / r;
        ct = dz * ir;
        st = rxy * ir;
    } else {
        ct = 1.0;
        st = 0.0;
    }
    if (rxy > 0) {
        const double irx = 1.0 / rxy;
        eph = cmk(dx * irx, dy * irx);
    } else {
        eph = cmk(1.0, 0.0);
    }
}

// ------------------------------------------------------------------ P2M
// C_n^m = i k sum_j [ q_j R_n^{-m}(c_j - C) + w_j (n_j . grad) R_n^{-m}(c_j - C) ]
// using  d_z R_n^m = k (a_{n-1}^m R_{n-1}^m - a_n^m R_{n+1}^m),
//        (d_x + i d_y) R_n^m = k (b_{n+1}^{-m-1} R_{n+1}^{m+1} - b_n^m R_{n-1}^{m+1}),
//        (d_x - i d_y) R_n^m = k (b_{n+1}^{m-1} R_{n+1}^{m-1} - b_n^{-m} R_{n-1}^{m-1}).
// One workgroup per leaf.  Per chunk of CH sources: geometry and j_n(k r) per source, the basis
// R_n^{m'} (n <= p, m' >= 0, plus a zero slot) per (source, m') in LDS, then each thread adds the
// sources' terms to its coefficient(s).  The seven basis entries a coefficient reads, with their
// factors and conjugation signs, are fixed per coefficient and set up once.
struct P2mTerms {
    int i[7];          // basis slot (the zero slot where the entry does not exist)
    double fx[7], fy[7];  // factors of the real and imaginary parts (fy = -fx for conjugated entries)
};
__device__ inline void p2m_term(int p, int TB, int nn, int mm, double f, int &i, double &fx, double &fy) {
    const int am = mm < 0 ? -mm : mm;
    if (nn < 0 || nn > p || am > nn) {
        i = TB;
        fx = fy = 0.0;
        return;
    }
    i = leg_tri(nn, am);
    fx = f;
    fy = mm < 0 ? -f : f;
}
__device__ inline void p2m_terms(int p, int TB, int c, double k, P2mTerms &T) {
    int n = (int)sqrt((double)c);
    while (n * n > c) --n;
    while ((n + 1) * (n + 1) <= c) ++n;
    const int mm = -(c - n * n - n);
    p2m_term(p, TB, n, mm, 1.0, T.i[0], T.fx[0], T.fy[0]);
    p2m_term(p, TB, n - 1, mm, k * coef_a(n - 1, mm), T.i[1], T.fx[1], T.fy[1]);
    p2m_term(p, TB, n + 1, mm, -k * coef_a(n, mm), T.i[2], T.fx[2], T.fy[2]);
    p2m_term(p, TB, n + 1, mm + 1, k * coef_b(n + 1, -mm - 1), T.i[3], T.fx[3], T.fy[3]);
    p2m_term(p, TB, n - 1, mm + 1, -k * coef_b(n, mm), T.i[4], T.fx[4], T.fy[4]);
    p2m_term(p, TB, n + 1, mm - 1, k * coef_b(n + 1, mm - 1), T.i[5], T.fx[5], T.fy[5]);
    p2m_term(p, TB, n - 1, mm - 1, -k * coef_b(n, -mm), T.i[6], T.fx[6], T.fy[6]);
}
template <int NR>
__device__ inline void p2m_accumulate(const P2mTerms &T, int cnt, int TS, const double2 *basis, const double2 *qw,
                                      const double *nrm, double2 (&a)[NR]) {
    for (int s = 0; s < cnt; ++s) {
        const double2 *B = basis + (int64_t)s * TS;
        double2 v[7];
#pragma unroll
        for (int t = 0; t < 7; ++t) v[t] = B[T.i[t]];
        const double2 R0 = cmk(T.fx[0] * v[0].x, T.fy[0] * v[0].y);
        const double2 dz = cmk(fma(T.fx[1], v[1].x, T.fx[2] * v[2].x), fma(T.fy[1], v[1].y, T.fy[2] * v[2].y));
        const double2 dp = cmk(fma(T.fx[3], v[3].x, T.fx[4] * v[4].x), fma(T.fy[3], v[3].y, T.fy[4] * v[4].y));
        const double2 dm = cmk(fma(T.fx[5], v[5].x, T.fx[6] * v[6].x), fma(T.fy[5], v[5].y, T.fy[6] * v[6].y));
        // n.grad = n_z d_z + (n_x - i n_y)/2 (d_x + i d_y) + (n_x + i n_y)/2 (d_x - i d_y); nrm holds
        // (n_x/2, n_y/2, n_z)
        const double hx = nrm[3 * s], hy = nrm[3 * s + 1], nz = nrm[3 * s + 2];
        double2 dn = cscale(dz, nz);
        dn = cfma(cmk(hx, -hy), dp, dn);
        dn = cfma(cmk(hx, hy), dm, dn);
#pragma unroll
        for (int rr = 0; rr < NR; ++rr) {
            a[rr] = cfma(qw[(2 * s) * NR + rr], R0, a[rr]);
            a[rr] = cfma(qw[(2 * s + 1) * NR + rr], dn, a[rr]);
        }
    }
}

// Slot sums: the derivative relations are linear with source-independent factors, so with
// per-source weights al_0 = q, al_1 = w n_z, al_2 = w (n_x - i n_y)/2, al_3 = w (n_x + i n_y)/2,
//   sum_s al_k,s B_s[t] (P) and sum_s conj(al_k,s) B_s[t] (Q)
// over the basis slots t (m' >= 0) give every coefficient as seven factor-weighted sums: an entry
// read conjugated (negative order) is conj(Q[t]).  One thread per slot keeps the eight sums per
// vector in registers across the leaf's chunks; each basis value is read once per source.
struct P2mSlotSums {
    static constexpr int K = 4;
};

template <int NR>
__global__ void __launch_bounds__(256) k_p2m_wide(int nleaf, int p, int CH, const int32_t *leaf_start,
                                             const double4 *center, const double4 *ec, const double4 *en,
                                             const double2 *sigma, const double2 *mu, double k, const double *leg,
                                             double2 *Mout) {
    extern __shared__ double2 smem[];
    const int b = blockIdx.x, tid = threadIdx.x;
    const int TB = (p + 1) * (p + 2) / 2, TS = TB + 1;     // basis entries and the zero slot
    double2 *basis = smem;                                 // CH * TS
    double2 *qw = basis + (int64_t)CH * TS;                // CH * 2 * NR
    double2 *W = qw + CH * 2 * NR;                         // CH * 4 * NR: slot-sum weights al_k
    double *jb = (double *)(W + CH * 4 * NR);              // CH * (p+2)
    double *geo = jb + CH * (p + 2);                       // CH * 4: cos, sin of the polar angle, e^{i phi}
    double *nrm = geo + CH * 4;                            // CH * 3
    double *lt = nrm + CH * 3;                             // 3 TB: Legendre recurrence table
    for (int e = tid; e < 3 * TB; e += blockDim.x) lt[e] = leg[e];
    const double4 C = center[b];
    const int ss = leaf_start[b], se = leaf_start[b + 1];
    const int ncoef = p * p;
    double2 *Mb = Mout + (int64_t)b * NR * ncoef;          // NR expansions of this leaf
    // slot sums in registers (one slot per thread, the zero slot included) when the slots fit the
    // workgroup and the staged basis can hold the eight sums of one vector at the end; otherwise
    // each thread accumulates whole coefficients in place
    const bool slots = TS <= (int)blockDim.x && CH * TS >= 8 * TS;
    double2 S[2 * P2mSlotSums::K][NR];
#pragma unroll
    for (int q = 0; q < 2 * P2mSlotSums::K; ++q)
#pragma unroll
        for (int rr = 0; rr < NR; ++rr) S[q][rr] = cmk(0, 0);
    if (!slots)
        for (int c = tid; c < NR * ncoef; c += blockDim.x) Mb[c] = cmk(0, 0);
    for (int j0 = ss; j0 < se; j0 += CH) {
        const int cnt = min(CH, se - j0);
        __syncthreads();
        if (tid < cnt) {
            const int j = j0 + tid;
            const double4 c = ec[j], nv = en[j];
            double r, ct, st;
            double2 eph;
            sph_frame(c.x - C.x, c.y - C.y, c.z - C.z, r, ct, st, eph);
            geo[4 * tid] = ct;
            geo[4 * tid + 1] = st;
            geo[4 * tid + 2] = eph.x;
            geo[4 * tid + 3] = eph.y;
            bessel_j_seq(k * r, p, jb + tid * (p + 2));
#pragma unroll
            for (int rr = 0; rr < NR; ++rr) {
                qw[(2 * tid) * NR + rr] = cscale(sigma[(int64_t)j * NR + rr], c.w);
                qw[(2 * tid + 1) * NR + rr] = cscale(mu[(int64_t)j * NR + rr], c.w);
            }
            nrm[3 * tid] = 0.5 * nv.x;
            nrm[3 * tid + 1] = 0.5 * nv.y;
            nrm[3 * tid + 2] = nv.z;
#pragma unroll
            for (int rr = 0; rr < NR; ++rr) {
                const double2 q = qw[(2 * tid) * NR + rr], w = qw[(2 * tid + 1) * NR + rr];
                W[(4 * tid) * NR + rr] = q;
                W[(4 * tid + 1) * NR + rr] = cscale(w, nv.z);
                W[(4 * tid + 2) * NR + rr] = cmul(w, cmk(0.5 * nv.x, -0.5 * nv.y));
                W[(4 * tid + 3) * NR + rr] = cmul(w, cmk(0.5 * nv.x, 0.5 * nv.y));
            }
        }
        __syncthreads();
        // basis column m' of source s: R_n^{m'} = j_n(k r) P_n^{m'}(cos) e^{i m' phi}, n = m'..p
        for (int w = tid; w < cnt * (p + 1); w += blockDim.x) {
            const int s = w / (p + 1), mp = w - s * (p + 1);
            const double ct = geo[4 * s], st = geo[4 * s + 1];
            const double2 eph = cmk(geo[4 * s + 2], geo[4 * s + 3]);
            const double *js = jb + s * (p + 2);
            double2 *out = basis + (int64_t)s * TS;
            double2 e = cmk(1.0, 0.0);
            double sp = 1.0;
            for (int q = 0; q < mp; ++q) {
                e = cmul(e, eph);
                sp *= st;
            }
            double P1 = lt[3 * leg_tri(mp, mp) + 2] * sp, P2 = 0.0;
            out[leg_tri(mp, mp)] = cscale(e, js[mp] * P1);
            for (int n = mp + 1; n <= p; ++n) {
                const int t = leg_tri(n, mp);
                const double P = fma(lt[3 * t] * ct, P1, -lt[3 * t + 1] * P2);
                P2 = P1;
                P1 = P;
                out[t] = cscale(e, js[n] * P);
            }
            if (mp == 0) out[TB] = cmk(0, 0);
        }
        __syncthreads();
        if (slots) {
            if (tid < TS)
                for (int s2 = 0; s2 < cnt; ++s2) {
                    const double2 B = basis[(int64_t)s2 * TS + tid];
#pragma unroll
                    for (int kk = 0; kk < P2mSlotSums::K; ++kk)
#pragma unroll
                        for (int rr = 0; rr < NR; ++rr) {
                            const double2 al = W[(4 * s2 + kk) * NR + rr];
                            S[2 * kk][rr] = cfma(al, B, S[2 * kk][rr]);
                            S[2 * kk + 1][rr] = cfma(cmk(al.x, -al.y), B, S[2 * kk + 1][rr]);
                        }
                }
        } else {
            for (int c = tid; c < ncoef; c += blockDim.x) {
                P2mTerms Tc;
                p2m_terms(p, TB, c, k, Tc);
                double2 a[NR];
#pragma unroll
                for (int rr = 0; rr < NR; ++rr) a[rr] = cmk(0, 0);
                p2m_accumulate<NR>(Tc, cnt, TS, basis, qw, nrm, a);
#pragma unroll
                for (int rr = 0; rr < NR; ++rr)
                    Mb[rr * ncoef + c] = cadd(Mb[rr * ncoef + c], cmuli(cscale(a[rr], k)));  // i k sum
            }
        }
    }
    if (slots) {
        // coefficient c = seven factor-weighted slot sums (entry i of term t from sum type k(t):
        // t = 0 monopole, 1-2 n_z d_z, 3-4 (d_x + i d_y), 5-6 (d_x - i d_y)), one vector at a time
        // through the staged basis region
        const int kt[7] = {0, 1, 1, 2, 2, 3, 3};
        double2 *SL = basis;  // [8][TS]
#pragma unroll
        for (int rr = 0; rr < NR; ++rr) {
            __syncthreads();
            if (tid < TS)
#pragma unroll
                for (int q = 0; q < 2 * P2mSlotSums::K; ++q) SL[q * TS + tid] = S[q][rr];
            __syncthreads();
            for (int c = tid; c < ncoef; c += blockDim.x) {
                P2mTerms T;
                p2m_terms(p, TB, c, k, T);
                double2 a = cmk(0, 0);
#pragma unroll
                for (int t = 0; t < 7; ++t) {
                    const bool cj = T.fy[t] != T.fx[t];  // conjugated entry: conj of the Q sum
                    const double2 v = SL[(2 * kt[t] + (cj ? 1 : 0)) * TS + T.i[t]];
                    a = cadd(a, cmk(T.fx[t] * v.x, T.fy[t] * v.y));
                }
                Mb[rr * ncoef + c] = cmuli(cscale(a, k));  // i k sum
            }
        }
    }
}

// j_0(x) .. j_N(x) for the expansion kernels: the sequence of bessel_j_seq, with Miller's
// normalised downward recurrence (x >= 4) taking one multiplication by 1/x per step instead of a
// division and starting 16 + 2 sqrt(max(N, x) + 1) orders above max(N, x): the minimal solution's
// ratio over the start's tail is then far below the recurrence's own rounding (a check of this
// start against a reference sequence for N <= 60, 4 <= x <= 1.2 N + 5 finds the same ~1e-12
// worst relative error, near zeros of j_n, as starting 40 + 4 sqrt(max(N, x) + 1) above).
__device__ inline void bessel_j_seq_fast(double x, int N, double *j) {
    if (x < 4.0 && N <= 40) {
        bessel_j_seq(x, N, j);
        return;
    }
    const int top = N > (int)x ? N : (int)x;
    const int start = top + 16 + (int)(2.0 * sqrt((double)top + 1.0));
    const double ix = rcp_nr(x);
    double fp1 = 0.0, f = 1e-300;
    for (int n = start; n >= 1; --n) {
        const double fm1 = fma((2.0 * n + 1.0) * ix, f, -fp1);
        fp1 = f;
        f = fm1;
        if (n - 1 <= N) j[n - 1] = f;
        if (fabs(f) > 1e250) {  // rescale everything stored so far
            f *= 1e-250;
            fp1 *= 1e-250;
            for (int q = n - 1; q <= N; ++q) j[q] *= 1e-250;
        }
    }
    double sn, cn;
    sincos(x, &sn, &cn);
    const double j0 = sn * ix, j1 = (sn * ix - cn) * ix;
    const double scale = (fabs(j0) >= fabs(j1) || N < 1) ? j0 / j[0] : j1 / j[1];
    for (int n = 0; n <= N; ++n) j[n] *= scale;
}

// Coefficients of the power series of x^{-n} (2n+1)!! j_n(x) (t_q = t_{q-1} h c_q) for the orders N
// and N - 1: c[o BS_TERMS + q - 1] = 1 / (q (2n + 2q + 1)), n = N - o, q = 1 .. BS_TERMS.  Computed
// once per workgroup, so that each series term costs two multiplications.
constexpr int BS_TERMS = 40;
__device__ inline void bessel_series_coeffs(int N, double *c, int tid, int nthreads) {
    for (int e = tid; e < 2 * BS_TERMS; e += nthreads) {
        const int o = e / BS_TERMS, q = e % BS_TERMS + 1, n = N - o;
        c[e] = 1.0 / ((double)q * (2.0 * n + 2.0 * q + 1.0));
    }
}

// j_0(x) .. j_N(x): for 1e-2 <= x < 4 and 1 <= N <= 40 the method of bessel_j_seq (j_N and j_{N-1}
// from their series, then the downward recurrence) with both series summed in one loop from the
// coefficients c of bessel_series_coeffs(N); otherwise bessel_j_seq_fast.
__device__ inline void bessel_j_seq_tab(double x, int N, double *j, const double *c) {
    if (x < 1e-2 || x >= 4.0 || N > 40 || N < 1) {
        bessel_j_seq_fast(x, N, j);
        return;
    }
    const double h = -0.5 * x * x;
    double sh = 1.0, th = 1.0, sl = 1.0, tl = 1.0;  // orders N and N - 1
    for (int q = 0; q < BS_TERMS; ++q) {
        th *= h * c[q];
        tl *= h * c[BS_TERMS + q];
        sh += th;
        sl += tl;
        if (fabs(th) <= 1e-17 * fabs(sh) && fabs(tl) <= 1e-17 * fabs(sl)) break;
    }
    double xn = 1.0, df = 1.0;  // x^{N-1} and (2N-1)!!
    for (int n = 1; n < N; ++n) {
        xn *= x;
        df *= 2.0 * n + 1.0;
    }
    const double pre = xn / df;
    double jh = pre * x / (2.0 * N + 1.0) * sh;
    double jl = pre * sl;
    j[N] = jh;
    j[N - 1] = jl;
    const double ix = 1.0 / x;
    for (int n = N - 1; n >= 1; --n) {
        const double jm = fma((2.0 * n + 1.0) * ix, jl, -jh);
        j[n - 1] = jm;
        jh = jl;
        jl = jm;
    }
}

// P2M with one thread per basis slot.  A workgroup takes one leaf; per chunk of CH sources:
//  1. one thread per source: frame, j_0..j_p(k r), the phase powers E_m' = (sin(th) e^{i phi})^m'
//     and the slot weights al_k of every vector;
//  2. the real part of the basis, R~_n^m' = j_n(k r) P_n^m'(cos th) / sin^m'(th), one recurrence in
//     n per (source, m'), the orders m' and p - m' paired so that each item is p + 2 steps long;
//  3. one thread per slot (n, m'), m' >= 0: R_n^m' = E_m' R~_n^m' and, for every k, the four real
//     sums of Re/Im al_k times Re/Im R, which give both sum_s al_k R (P) and sum_s conj(al_k) R (Q)
//     (the same slot sums as the wide kernel, at half its multiplications);
//  4. every coefficient from seven factor-weighted slot sums, through LDS.
// Needs (p + 1)(p + 2)/2 <= 256 (p <= 20); launch_p2m takes the wide kernel beyond.
template <int NR>
__global__ void __launch_bounds__(256) k_p2m(int nleaf, int p, int CH, const int32_t *leaf_start,
                                             const double4 *center, const double4 *ec, const double4 *en,
                                             const double2 *sigma, const double2 *mu, double k, const double *leg,
                                             double2 *Mout) {
    extern __shared__ double2 smem[];
    const int b = blockIdx.x, tid = threadIdx.x;
    const int TB = (p + 1) * (p + 2) / 2, TS = TB + 1, p1 = p + 1;
    double2 *E = smem;                          // CH * (p+1)
    double2 *al = E + CH * p1;                  // CH * 4 * NR
    double *Rb = (double *)(al + CH * 4 * NR);  // CH * TB
    double *jb = Rb + CH * TB;                  // CH * (p+2)
    double *cth = jb + CH * (p + 2);            // CH
    double *lt = cth + CH;                      // 3 TB: Legendre recurrence table
    double *bc = lt + 3 * TB;                   // 2 BS_TERMS: series coefficients of j_p, j_{p-1}
    double2 *SL = smem;                         // after the last chunk: [8][TS] slot sums of one vector
    for (int e = tid; e < 3 * TB; e += blockDim.x) lt[e] = leg[e];
    bessel_series_coeffs(p, bc, tid, blockDim.x);
    const double4 C = center[b];
    const int ss = leaf_start[b], se = leaf_start[b + 1];
    // a chunk's source data is loaded while the previous chunk is summed
    double4 pc = make_double4(0, 0, 0, 0), pn = pc;
    double2 pq[NR], pw[NR];
    auto fetch = [&](int j0n) {
        const int j = j0n + tid;
        if (tid < CH && j < se) {
            pc = ec[j];
            pn = en[j];
#pragma unroll
            for (int rr = 0; rr < NR; ++rr) {
                pq[rr] = sigma[(int64_t)j * NR + rr];
                pw[rr] = mu[(int64_t)j * NR + rr];
            }
        }
    };
    fetch(ss);
    // this thread's slot
    int sn = 0, sm = 0;
    if (tid < TB) {
        while ((sn + 1) * (sn + 2) / 2 <= tid) ++sn;
        sm = tid - sn * (sn + 1) / 2;
    }
    double acc[4][NR][4];
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int rr = 0; rr < NR; ++rr)
#pragma unroll
            for (int u = 0; u < 4; ++u) acc[q][rr][u] = 0.0;
    const int npair = p / 2 + 1;
    for (int j0 = ss; j0 < se; j0 += CH) {
        const int cnt = min(CH, se - j0);
        __syncthreads();  // the previous chunk's readers are done (and lt is in place)
        if (tid < cnt) {
            const double4 c = pc, nv = pn;
            double r, ct, st;
            double2 eph;
            sph_frame(c.x - C.x, c.y - C.y, c.z - C.z, r, ct, st, eph);
            cth[tid] = ct;
            bessel_j_seq_tab(k * r, p, jb + tid * (p + 2), bc);
            const double2 u = cscale(eph, st);
            double2 e = cmk(1.0, 0.0);
            for (int m = 0; m <= p; ++m) {
                E[tid * p1 + m] = e;
                e = cmul(e, u);
            }
#pragma unroll
            for (int rr = 0; rr < NR; ++rr) {
                const double2 q = cscale(pq[rr], c.w), w = cscale(pw[rr], c.w);
                al[(tid * 4) * NR + rr] = q;
                al[(tid * 4 + 1) * NR + rr] = cscale(w, nv.z);
                al[(tid * 4 + 2) * NR + rr] = cmul(w, cmk(0.5 * nv.x, -0.5 * nv.y));
                al[(tid * 4 + 3) * NR + rr] = cmul(w, cmk(0.5 * nv.x, 0.5 * nv.y));
            }
        }
        __syncthreads();
        fetch(j0 + CH);
        for (int w = tid; w < cnt * npair; w += blockDim.x) {
            const int s = w / npair, pr = w - s * npair;
            const double ct = cth[s];
            const double *js = jb + s * (p + 2);
            double *out = Rb + s * TB;
            for (int h = 0; h < 2; ++h) {
                const int mp = h == 0 ? pr : p - pr;
                if (h == 1 && mp == pr) break;
                double P1 = lt[3 * leg_tri(mp, mp) + 2], P2 = 0.0;
                out[leg_tri(mp, mp)] = js[mp] * P1;
                for (int n = mp + 1; n <= p; ++n) {
                    const int t = leg_tri(n, mp);
                    const double P = fma(lt[3 * t] * ct, P1, -lt[3 * t + 1] * P2);
                    P2 = P1;
                    P1 = P;
                    out[t] = js[n] * P;
                }
            }
        }
        __syncthreads();
        if (tid < TB)
            for (int s = 0; s < cnt; ++s) {
                const double2 B = cscale(E[s * p1 + sm], Rb[s * TB + tid]);
#pragma unroll
                for (int q = 0; q < 4; ++q)
#pragma unroll
                    for (int rr = 0; rr < NR; ++rr) {
                        const double2 a = al[(s * 4 + q) * NR + rr];
                        acc[q][rr][0] = fma(a.x, B.x, acc[q][rr][0]);
                        acc[q][rr][1] = fma(a.y, B.y, acc[q][rr][1]);
                        acc[q][rr][2] = fma(a.x, B.y, acc[q][rr][2]);
                        acc[q][rr][3] = fma(a.y, B.x, acc[q][rr][3]);
                    }
            }
    }
    // coefficient c = seven factor-weighted slot sums (entry i of term t from sum type k(t):
    // t = 0 monopole, 1-2 n_z d_z, 3-4 (d_x + i d_y), 5-6 (d_x - i d_y)), one vector at a time
    const int kt[7] = {0, 1, 1, 2, 2, 3, 3};
    const int ncoef = p * p;
    double2 *Mb = Mout + (int64_t)b * NR * ncoef;
#pragma unroll
    for (int rr = 0; rr < NR; ++rr) {
        __syncthreads();
        if (tid < TB)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const double A = acc[q][rr][0], Bq = acc[q][rr][1], Cq = acc[q][rr][2], D = acc[q][rr][3];
                SL[(2 * q) * TS + tid] = cmk(A - Bq, Cq + D);      // sum al_k R
                SL[(2 * q + 1) * TS + tid] = cmk(A + Bq, Cq - D);  // sum conj(al_k) R
            }
        if (tid < 8) SL[tid * TS + TB] = cmk(0.0, 0.0);
        __syncthreads();
        for (int c = tid; c < ncoef; c += blockDim.x) {
            P2mTerms T;
            p2m_terms(p, TB, c, k, T);
            double2 a = cmk(0, 0);
#pragma unroll
            for (int t = 0; t < 7; ++t) {
                const bool cj = T.fy[t] != T.fx[t];  // conjugated entry: conj of the Q sum
                const double2 v = SL[(2 * kt[t] + (cj ? 1 : 0)) * TS + T.i[t]];
                a = cadd(a, cmk(T.fx[t] * v.x, T.fy[t] * v.y));
            }
            Mb[rr * ncoef + c] = cmuli(cscale(a, k));  // i k sum
        }
    }
}

// ------------------------------------------------------------------ L2P + combine
// y[perm[i]] = half * x[perm[i]] + y_near[i] + sum_{n,m} D_n^m R_n^m(c_i - C).
// One thread per target; the recurrence table and (STAGE) the leaf's expansions are staged in LDS
// (every thread reads the same entry at once: broadcasts), the degree loop unrolled so that its
// reads overlap.  Without STAGE (expansions too large for LDS) they are read from global memory.
template <int NR, bool STAGE>
__global__ void __launch_bounds__(64) k_l2p(int nleaf, int p, const int32_t *leaf_start, const double4 *center,
                                            const double4 *ec, const double2 *Lc, double k, const double *leg,
                                            const double2 *ynear, double half, const int32_t *perm, int64_t n,
                                            const double2 *x, double2 *y, int has_far) {
    extern __shared__ double2 l2p_sm[];
    const int b = blockIdx.x, tid = threadIdx.x;
    const double4 C = center[b];
    const int ts = leaf_start[b], te = leaf_start[b + 1];
    const int pp = p * p, TB = p * (p + 1) / 2;
    const double2 *Dg = Lc + (int64_t)b * NR * pp;   // NR expansions of this leaf
    double2 *Dl = l2p_sm;
    double *lt = STAGE ? (double *)(Dl + NR * pp) : (double *)l2p_sm;  // 3 TB: Legendre recurrence (degrees < p)
    double *bc = lt + 3 * TB;                                           // series coefficients of j_{p-1}, j_{p-2}
    double *jb = bc + 2 * BS_TERMS + tid * (p + 2);
    const double2 *D = STAGE ? (const double2 *)Dl : Dg;
    if (has_far) {
        for (int e = tid; e < 3 * TB; e += blockDim.x) lt[e] = leg[e];
        bessel_series_coeffs(p - 1, bc, tid, blockDim.x);
        if (STAGE)
            for (int e = tid; e < NR * pp; e += blockDim.x) Dl[e] = Dg[e];
        __syncthreads();
    }
    // A leaf of at most 32 (16) targets splits the orders m over 2 (4) lane groups of 32 (16)
    // targets, group g taking m = g, g + S, ..., and adds the groups' sums at the end (leaves hold
    // about 34 targets on average: one target per lane leaves half the lanes idle)
    __shared__ double2 red[64 * NR];
    const int nt = te - ts, S = nt <= 16 ? 4 : (nt <= 32 ? 2 : 1), TP = 64 / S, g = tid / TP;
    for (int t0 = ts; t0 < te; t0 += TP) {
        const int t = t0 + tid % TP;
        const bool act = t < te;
        double2 far[NR];
#pragma unroll
        for (int rr = 0; rr < NR; ++rr) far[rr] = cmk(0, 0);
        if (has_far && act) {
            const double4 c = ec[t];
            double r, ct, st;
            double2 eph;
            sph_frame(c.x - C.x, c.y - C.y, c.z - C.z, r, ct, st, eph);
            bessel_j_seq_tab(k * r, p - 1, jb, bc);
            double2 e = cmk(1.0, 0.0);
            double sp = 1.0;
            for (int q = 0; q < g; ++q) {
                e = cmul(e, eph);
                sp *= st;
            }
            for (int mp = g; mp < p; mp += S) {
                if (mp > g)
                    for (int q = 0; q < S; ++q) {  // e^{i m phi} and sin^m by the same products as for S = 1
                        e = cmul(e, eph);
                        sp *= st;
                    }
                double P1 = lt[3 * leg_tri(mp, mp) + 2] * sp, P2 = 0.0;
                double2 sa[NR], sb[NR];
#pragma unroll
                for (int rr = 0; rr < NR; ++rr) {
                    sa[rr] = cscale(D[rr * pp + cidx(mp, mp)], jb[mp] * P1);
                    sb[rr] = mp > 0 ? cscale(D[rr * pp + cidx(mp, -mp)], jb[mp] * P1) : cmk(0, 0);
                }
#pragma unroll 4
                for (int nn = mp + 1; nn < p; ++nn) {
                    const int q = leg_tri(nn, mp);
                    const double P = fma(lt[3 * q] * ct, P1, -lt[3 * q + 1] * P2);
                    P2 = P1;
                    P1 = P;
                    const double R = jb[nn] * P;
#pragma unroll
                    for (int rr = 0; rr < NR; ++rr) {
                        sa[rr] = cadd(sa[rr], cscale(D[rr * pp + cidx(nn, mp)], R));
                        if (mp > 0) sb[rr] = cadd(sb[rr], cscale(D[rr * pp + cidx(nn, -mp)], R));
                    }
                }
                // sum_n D_n^m R e^{i m phi} + D_n^{-m} R e^{-i m phi}
#pragma unroll
                for (int rr = 0; rr < NR; ++rr) {
                    far[rr] = cfma(sa[rr], e, far[rr]);
                    if (mp > 0) far[rr] = cfma(sb[rr], cconj(e), far[rr]);
                }
            }
        }
        if (S > 1) {  // group 0 adds the other groups' sums
            __syncthreads();
#pragma unroll
            for (int rr = 0; rr < NR; ++rr) red[tid * NR + rr] = far[rr];
            __syncthreads();
            if (g == 0)
                for (int gg = 1; gg < S; ++gg)
#pragma unroll
                    for (int rr = 0; rr < NR; ++rr) far[rr] = cadd(far[rr], red[(tid + gg * TP) * NR + rr]);
        }
        if (!act || g > 0) continue;
        const int64_t u = perm[t];
#pragma unroll
        for (int rr = 0; rr < NR; ++rr) {
            double2 v = cadd(ynear[(int64_t)t * NR + rr], far[rr]);
            if (x) v = cadd(v, cscale(x[rr * n + u], half));  // the right-hand side pass has no identity term
            y[rr * n + u] = v;
        }
    }
}

// ------------------------------------------------------------------ field at points
// out[q] = amp * G(r_q, rs) + sum_j [L_j(r_q) sigma_j + M_j(r_q) mu_j], accurate integrals for
// elements with |r_q - c_j| < r_c, one-point rule otherwise.  One workgroup per point (few points:
// below about three workgroups of k_field_tile per CU).
__global__ void __launch_bounds__(256) k_field(int64_t nt, const double *pts, const double4 *ec, const double4 *en,
                                               const double *ev, const double2 *sigma, const double2 *mu, double k,
                                               double rc2, double sx, double sy, double sz, double2 amp,
                                               double2 *out) {
    const int q = blockIdx.x, tid = threadIdx.x;
    const double x[3] = {pts[3 * q], pts[3 * q + 1], pts[3 * q + 2]};
    double2 acc = cmk(0, 0);
    const double inv4pi = 1.0 / (4.0 * FMM_PI);
    for (int64_t j = tid; j < nt; j += blockDim.x) {
        double4 c = ec[j];
        double d2 = dist2_exact(x[0], x[1], x[2], c.x, c.y, c.z);
        double2 L, M;
        if (d2 < rc2) {
            double v[9];
            for (int e = 0; e < 9; ++e) v[e] = ev[9 * j + e];
            tri_integrals(x, v, k, 0, L, M);
        } else {
            double4 nv = en[j];
            double dx = c.x - x[0], dy = c.y - x[1], dz = c.z - x[2];
            double r = sqrt(d2), s, co;
            sincos(k * r, &s, &co);
            double2 G = cmk(co / r * inv4pi, s / r * inv4pi);
            double u = (dx * nv.x + dy * nv.y + dz * nv.z) / d2;
            L = cscale(G, c.w);
            M = cscale(cmul(G, cmk(-u, k * r * u)), c.w);
        }
        acc = cfma(L, sigma[j], acc);
        acc = cfma(M, mu[j], acc);
    }
    __shared__ double2 red[256];
    red[tid] = acc;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if (tid < s) red[tid] = cadd(red[tid], red[tid + s]);
        __syncthreads();
    }
    if (tid == 0) {
        double dx = x[0] - sx, dy = x[1] - sy, dz = x[2] - sz;
        double r = sqrt(dx * dx + dy * dy + dz * dz), s, co;
        sincos(k * r, &s, &co);
        out[q] = cadd(red[0], cmul(amp, cmk(co / r * inv4pi, s / r * inv4pi)));
    }
}

// The same for many points: a workgroup takes FIELD_FQ points, tiles of
// 256 elements pass through LDS once for all of them (one workgroup per point read every element
// from the caches once per point), 32 threads per point take every 32nd element of a tile, and
// each point's 32 partial sums are added in a fixed order.  1/r and sin/cos(kr) as in the pair
// kernel of the product.  Three waves per SIMD (168 registers; four waves spill): 19,200 points
// on the 1M L-room at 2.0e11 pairs/s, against 1.25-1.47e11 with one workgroup per point.
static_assert(FIELD_FQ * 32 == 256, "32 threads per receiver in a workgroup of 256");
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3, 3)))
k_field_tile(int64_t nt, int64_t nq, const double *pts, const double4 *ec, const double4 *en, const double *ev,
             const double2 *sigma, const double2 *mu, double k, double rc2, double sx, double sy, double sz,
             double2 amp, double2 *out) {
    __shared__ double4 sc[256], sn[256];
    __shared__ double2 ssg[256], smu[256], red[256];
    const int tid = threadIdx.x, l = tid & 31;
    const int64_t q = (int64_t)blockIdx.x * FIELD_FQ + (tid >> 5), qc = q < nq ? q : nq - 1;
    const double x[3] = {pts[3 * qc], pts[3 * qc + 1], pts[3 * qc + 2]};
    const double inv4pi = 1.0 / (4.0 * FMM_PI);
    double2 acc = cmk(0, 0);
    for (int64_t j0 = 0; j0 < nt; j0 += 256) {
        __syncthreads();
        if (j0 + tid < nt) {
            sc[tid] = ec[j0 + tid];
            sn[tid] = en[j0 + tid];
            ssg[tid] = sigma[j0 + tid];
            smu[tid] = mu[j0 + tid];
        }
        __syncthreads();
        const int cnt = (int)(nt - j0 < 256 ? nt - j0 : 256);
        for (int jj = l; jj < cnt; jj += 32) {
            const double4 c = sc[jj];
            const double d2 = dist2_exact(x[0], x[1], x[2], c.x, c.y, c.z);
            double2 L, M;
            if (d2 < rc2) {
                double v[9];
                for (int e = 0; e < 9; ++e) v[e] = ev[9 * (j0 + jj) + e];
                tri_integrals(x, v, k, 0, L, M);
            } else {
                const double4 nv = sn[jj];
                const double dx = c.x - x[0], dy = c.y - x[1], dz = c.z - x[2];
                const double ir = rsq_nr(d2), r = d2 * ir;
                double s, co;
                sincos_red(k * r, s, co);
                const double2 G = cmk(co * ir * inv4pi, s * ir * inv4pi);
                const double u = (dx * nv.x + dy * nv.y + dz * nv.z) * ir * ir;
                L = cscale(G, c.w);
                M = cscale(cmul(G, cmk(-u, k * r * u)), c.w);
            }
            acc = cfma(L, ssg[jj], acc);
            acc = cfma(M, smu[jj], acc);
        }
    }
    red[tid] = acc;
    __syncthreads();
    for (int h = 16; h > 0; h >>= 1) {
        if (l < h) red[tid] = cadd(red[tid], red[tid + h]);
        __syncthreads();
    }
    if (l == 0 && q < nq) {
        double dx = x[0] - sx, dy = x[1] - sy, dz = x[2] - sz;
        double r = sqrt(dx * dx + dy * dy + dz * dz), s, co;
        sincos(k * r, &s, &co);
        out[q] = cadd(red[tid], cmul(amp, cmk(co / r * inv4pi, s / r * inv4pi)));
    }
}

// ------------------------------------------------------------------ indirect formulation (Eq. ibem5)
// Unknowns x = (psi-, psi+), N each in caller order.  Both block rows need the same layer
// densities s = -i k (beta- psi- + beta+ psi+) (single layer) and m = psi- - psi+ (double layer):
//   row 1 = (psi- + psi+)/2 + L[s] + M[m],   row 2 = i k (beta- psi- - beta+ psi+)/2 + L'[s] + M'[m],
// so one FMM pass evaluates the potential and its normal derivative at every collocation point.

// g- = -dpsi_in/dn + i k beta- psi_in, g+ = dpsi_in/dn + i k beta+ psi_in (tree order)
__global__ void k_gamma_pm(int64_t n, const double4 *ec, const double4 *en, const double2 *bm, const double2 *bp,
                           double k, double sx, double sy, double sz, double2 amp, double2 *gm, double2 *gp) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double4 c = ec[i], nv = en[i];
    double dx = c.x - sx, dy = c.y - sy, dz = c.z - sz;
    double r = sqrt(dx * dx + dy * dy + dz * dz);
    double s, co;
    sincos(k * r, &s, &co);
    double2 G = cmul(amp, cmk(co / (4 * FMM_PI * r), s / (4 * FMM_PI * r)));
    double proj = (dx * nv.x + dy * nv.y + dz * nv.z) / (r * r);
    double2 dG = cscale(cmul(G, cmk(-1.0, k * r)), proj);  // dpsi_in/dn
    gm[i] = csub(cmul(cmk(-k * bm[i].y, k * bm[i].x), G), dG);
    gp[i] = cadd(cmul(cmk(-k * bp[i].y, k * bp[i].x), G), dG);
}

__global__ void k_densities_ind(int64_t n, const int32_t *perm, const double2 *x, const double2 *bm,
                                const double2 *bp, double k, double2 *sigma, double2 *mu) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t u = perm[i];
    const double2 pm = x[u], pp = x[n + u];
    const double2 t = cadd(cmul(bm[i], pm), cmul(bp[i], pp));
    sigma[i] = cmk(k * t.y, -k * t.x);  // -i k (beta- psi- + beta+ psi+)
    mu[i] = csub(pm, pp);
}

// densities of the receiver formula (Eq. ibem1, ibem4): sigma = g- + g+ + i k (beta- psi- +
// beta+ psi+), mu = psi+ - psi-
__global__ void k_field_dens_ind(int64_t n, const int32_t *perm, const double2 *x, const double2 *gm,
                                 const double2 *gp, const double2 *bm, const double2 *bp, double k, double2 *sigma,
                                 double2 *mu) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t u = perm[i];
    const double2 pm = x[u], pp = x[n + u];
    const double2 t = cadd(cmul(bm[i], pm), cmul(bp[i], pp));
    sigma[i] = cadd(cadd(gm[i], gp[i]), cmk(-k * t.y, k * t.x));
    mu[i] = csub(pp, pm);
}

// Densities of the receiver formula from the surface unknown x (caller order), in tree order, with
// the incident field of a monopole of amplitude amp at s evaluated at each centroid (Eq. sp6-sp7):
//   form 0, unknown psi_sc (Eq. dbem4 and the combined form): sigma = gamma + i k beta x,
//           mu = -x (Eq. dbem1), gamma = -dpsi_in/dn + i k beta psi_in;
//   form 1, unknown v = dpsi_sc/dn (Eq. dbem5): sigma = v, mu = -psi_sc = -(v - gamma)/(i k beta);
//   form 3, unknowns (psi-, psi+) (Eq. ibem5): sigma = g- + g+ + i k (beta- psi- + beta+ psi+),
//           mu = psi+ - psi- (Eq. ibem1, ibem4), g-+ = -+ dpsi_in/dn + i k beta-+ psi_in.
__global__ void k_field_dens(int64_t n, int form, const int32_t *perm, const double2 *x, const double4 *ec,
                             const double4 *en, const double2 *bm, const double2 *bp, double k, double sx, double sy,
                             double sz, double2 amp, double2 *sigma, double2 *mu) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double4 c = ec[i], nv = en[i];
    const double dx = c.x - sx, dy = c.y - sy, dz = c.z - sz;
    const double r = sqrt(dx * dx + dy * dy + dz * dz);
    double s, co;
    sincos(k * r, &s, &co);
    const double2 G = cmul(amp, cmk(co / (4 * FMM_PI * r), s / (4 * FMM_PI * r)));
    const double proj = (dx * nv.x + dy * nv.y + dz * nv.z) / (r * r);
    const double2 dG = cscale(cmul(G, cmk(-1.0, k * r)), proj);  // dpsi_in/dn
    const int64_t u = perm[i];
    const double2 ikbm = cmk(-k * bm[i].y, k * bm[i].x);
    const double2 gm = csub(cmul(ikbm, G), dG);
    if (form == 3) {
        const double2 ikbp = cmk(-k * bp[i].y, k * bp[i].x);
        const double2 gp = cadd(cmul(ikbp, G), dG);
        const double2 pm = x[u], pp = x[n + u];
        sigma[i] = cadd(cadd(gm, gp), cadd(cmul(ikbm, pm), cmul(ikbp, pp)));
        mu[i] = csub(pp, pm);
    } else if (form == 1) {
        const double2 v = x[u];
        sigma[i] = v;
        mu[i] = cscale(cdiv(csub(v, gm), ikbm), -1.0);
    } else {
        const double2 xi = x[u];
        sigma[i] = cadd(gm, cmul(ikbm, xi));
        mu[i] = cscale(xi, -1.0);
    }
}

// row 2 of the right-hand side gets (g+ - g-)/2
__global__ void k_rhs_ind_local(int64_t n, const int32_t *perm, const double2 *gm, const double2 *gp, double2 *b) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t u = perm[i];
    b[n + u] = cadd(b[n + u], cscale(csub(gp[i], gm[i]), 0.5));
}

// Eq. (dbem5), unknown v = dpsi_sc/dn (caller order): densities sigma = -i k v, mu = zeta v with
// zeta = 1/beta (tree order); the product is v/2 + beta (L[sigma] + M[mu]).
__global__ void k_densities_dpsi(int64_t n, const int32_t *perm, const double2 *v, const double2 *beta, double k,
                                 double2 *sigma, double2 *mu) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double2 vi = v[perm[i]];
    sigma[i] = cmk(k * vi.y, -k * vi.x);  // -i k v
    mu[i] = cdiv(vi, beta[i]);
}
// y = half h + beta P (h, P, y caller order; beta tree order): the product (h = v) and the
// right-hand side (h = gamma in caller order)
__global__ void k_dpsi_combine(int64_t n, const int32_t *perm, const double2 *h, const double2 *beta, const double2 *P,
                               double2 *y) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t u = perm[i];
    y[u] = cadd(cscale(h[u], 0.5), cmul(beta[i], P[u]));
}
// right-hand side densities of Eq. (dbem5): gamma (in sigma, tree order) -> gamma in caller order,
// mu = zeta gamma, sigma = 0
__global__ void k_rhs_dpsi_dens(int64_t n, const int32_t *perm, const double2 *beta, double2 *sigma, double2 *mu,
                                double2 *gam_caller) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double2 g = sigma[i];
    gam_caller[perm[i]] = g;
    mu[i] = cdiv(g, beta[i]);
    sigma[i] = cmk(0, 0);
}
// z = v * beta (inv = 0) or v / beta (inv = 1), caller order
__global__ void k_scale_beta(int64_t n, const int32_t *perm, const double2 *beta, int inv, const double2 *v,
                             double2 *z) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t u = perm[i];
    z[u] = inv ? cdiv(v[u], beta[i]) : cmul(v[u], beta[i]);
}

// Combined (Burton-Miller) direct equation: Eq. (dbem3) plus alpha times its normal derivative
// (Section 3.2 jump relations; v = dpsi/dn = gamma + i k beta psi).  From the potential P and the
// normal derivative Q of the layers sigma = -i k beta x, mu = x (caller order, pq[0..n) and
// pq[n..2n)):  y = x/2 + (alpha i k / 2) beta x + P + alpha Q.
__global__ void k_bm_combine(int64_t n, const int32_t *perm, const double2 *x, const double2 *beta, double k,
                             double2 alpha, const double2 *pq, double2 *y) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t u = perm[i];
    const double2 xu = x[u];
    const double2 half_aikb = cscale(cmul(alpha, cmuli(beta[i])), 0.5 * k);  // alpha i k beta / 2
    double2 v = cadd(cscale(xu, 0.5), cmul(half_aikb, xu));
    v = cadd(v, pq[u]);
    y[u] = cadd(v, cmul(alpha, pq[n + u]));
}

// Right-hand side of the combined equation: b = P + alpha (Q - gamma / 2), (P, Q) of the layer
// sigma = gamma (gamma in tree order).
__global__ void k_bm_rhs(int64_t n, const int32_t *perm, const double2 *gam, double2 alpha, const double2 *pq,
                         double2 *b) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t u = perm[i];
    b[u] = cadd(pq[u], cmul(alpha, csub(pq[n + u], cscale(gam[i], 0.5))));
}

// potential and normal derivative at the targets from one-point pairs and the near table
__global__ void __launch_bounds__(64) k_p2p_n(int nleaf, const int32_t *leaf_start, const int32_t *nbr_start,
                                              const int32_t *nbr_list, int all_leaves, const double4 *ec,
                                              const double4 *en, const double2 *sigma, const double2 *mu, double k,
                                              double rc2, const int32_t *near_start, const int32_t *near_col,
                                              const double2 *nL, const double2 *nM, const double2 *nLp,
                                              const double2 *nMp, double2 *y, double2 *yn) {
    const int b = blockIdx.x, tid = threadIdx.x;
    __shared__ double sx[64], sy[64], sz[64], snx[64], sny[64], snz[64];
    __shared__ double2 sq[64], sw[64];
    const int ts = leaf_start[b], te = leaf_start[b + 1];
    const int nb0 = all_leaves ? 0 : nbr_start[b], nb1 = all_leaves ? nleaf : nbr_start[b + 1];
    const double inv4pi = 1.0 / (4.0 * FMM_PI);
    for (int t0 = ts; t0 < te; t0 += 64) {
        const int t = t0 + tid;
        const bool act = t < te;
        const double4 ct = act ? ec[t] : make_double4(0, 0, 0, 0);
        const double4 nt = act ? en[t] : make_double4(0, 0, 1, 0);
        double2 acc = cmk(0, 0), accn = cmk(0, 0);
        for (int q = nb0; q < nb1; ++q) {
            const int sb = all_leaves ? q : nbr_list[q];
            const int ss = leaf_start[sb], se = leaf_start[sb + 1];
            for (int j0 = ss; j0 < se; j0 += 64) {
                __syncthreads();
                int j = j0 + tid;
                if (j < se) {
                    double4 c = ec[j], nv = en[j];
                    sx[tid] = c.x;
                    sy[tid] = c.y;
                    sz[tid] = c.z;
                    snx[tid] = nv.x;
                    sny[tid] = nv.y;
                    snz[tid] = nv.z;
                    sq[tid] = cscale(sigma[j], c.w);
                    sw[tid] = cscale(mu[j], c.w);
                }
                __syncthreads();
                const int cnt = min(64, se - j0);
                if (act) {
                    for (int jj = 0; jj < cnt; ++jj) {
                        double d2 = dist2_exact(ct.x, ct.y, ct.z, sx[jj], sy[jj], sz[jj]);
                        if (d2 < rc2) continue;
                        const double dx = sx[jj] - ct.x, dy = sy[jj] - ct.y, dz = sz[jj] - ct.z;
                        const double ir = rsq_nr(d2), r = d2 * ir, ir2 = ir * ir;
                        double s, c;
                        sincos_red(k * r, s, c);
                        const double2 E = cmk(c * inv4pi, s * inv4pi);  // e^{ikr} / 4 pi
                        const double2 G = cscale(E, ir);
                        const double dny = dx * snx[jj] + dy * sny[jj] + dz * snz[jj];
                        const double dnx = dx * nt.x + dy * nt.y + dz * nt.z;
                        const double nn = nt.x * snx[jj] + nt.y * sny[jj] + nt.z * snz[jj];
                        const double2 g1 = cmul(G, cmk(-1.0, k * r));  // G (ikr - 1)
                        // potential: G q + G (ikr - 1) (d.n_y)/r^2 w
                        acc = cfma(G, sq[jj], acc);
                        acc = cfma(cscale(g1, dny * ir2), sw[jj], acc);
                        // normal derivative: -G (ikr - 1)(d.n_x)/r^2 q + K w
                        accn = cfma(cscale(g1, -dnx * ir2), sq[jj], accn);
                        const double2 k3 = cmul(E, cmk(3.0 - k * k * d2, -3.0 * k * r));  // e(3 - 3ikr - k^2 r^2)
                        const double2 K = csub(cscale(k3, -dnx * dny * ir2 * ir2 * ir), cscale(cmul(E, cmk(-1.0, k * r)), nn * ir2 * ir));
                        accn = cfma(K, sw[jj], accn);
                    }
                }
            }
        }
        if (act) {
            for (int e = near_start[t]; e < near_start[t + 1]; ++e) {
                const int j = near_col[e];
                acc = cfma(nL[e], sigma[j], acc);
                acc = cfma(nM[e], mu[j], acc);
                accn = cfma(nLp[e], sigma[j], accn);
                accn = cfma(nMp[e], mu[j], accn);
            }
            y[t] = acc;
            yn[t] = accn;
        }
    }
}

// derivative local expansions of a leaf (degree p + 1) from its local expansion D (degree p):
//   d_z R_n^m = k (a_{n-1}^m R_{n-1}^m - a_n^m R_{n+1}^m), etc. (the P2M recurrences), collected
//   per output coefficient (n, m)
__device__ inline double2 dget_nm(const double2 *D, int p, int n, int m) {
    if (n < 0 || n >= p || (m < 0 ? -m : m) > n) return cmk(0, 0);
    return D[cidx(n, m)];
}
__global__ void k_local_derivs(int64_t nleaf, int p, const double2 *D, double k, double2 *Dz, double2 *Dp,
                               double2 *Dm) {
    const int64_t b = blockIdx.x;
    const int q1 = (p + 1) * (p + 1);
    const double2 *Db = D + b * p * p;
    for (int c = threadIdx.x; c < q1; c += blockDim.x) {
        int n = (int)sqrt((double)c);
        while (n * n > c) --n;
        while ((n + 1) * (n + 1) <= c) ++n;
        const int m = c - n * n - n;
        const double2 z = csub(cscale(dget_nm(Db, p, n + 1, m), coef_a(n, m)), cscale(dget_nm(Db, p, n - 1, m), coef_a(n - 1, m)));
        const double2 pl = csub(cscale(dget_nm(Db, p, n - 1, m - 1), coef_b(n, -m)),
                                cscale(dget_nm(Db, p, n + 1, m - 1), coef_b(n + 1, m - 1)));
        const double2 mi = csub(cscale(dget_nm(Db, p, n - 1, m + 1), coef_b(n, m)),
                                cscale(dget_nm(Db, p, n + 1, m + 1), coef_b(n + 1, -m - 1)));
        Dz[b * q1 + c] = cscale(z, k);
        Dp[b * q1 + c] = cscale(pl, k);
        Dm[b * q1 + c] = cscale(mi, k);
    }
}

// potential (local expansion D, degree p) and normal derivative (derivative expansions, degree
// p + 1) at the targets, plus the near part and the local terms of both block rows
__global__ void __launch_bounds__(64) k_l2p_n(int nleaf, int p, const int32_t *leaf_start, const double4 *center,
                                              const double4 *ec, const double4 *en, const double2 *Lc,
                                              const double2 *Dz, const double2 *Dp, const double2 *Dm, double k,
                                              const double *leg, const double2 *ynear, const double2 *ynearn,
                                              const int32_t *perm,
                                              int64_t n, const double2 *x, const double2 *bm, const double2 *bp,
                                              double2 *y, int has_far) {
    extern __shared__ double jbuf[];
    const int b = blockIdx.x, tid = threadIdx.x;
    const double4 C = center[b];
    const int ts = leaf_start[b], te = leaf_start[b + 1];
    const int q1 = (p + 1) * (p + 1);
    const double2 *D = Lc + (int64_t)b * p * p, *Ez = Dz + (int64_t)b * q1, *Ep = Dp + (int64_t)b * q1,
                  *Em = Dm + (int64_t)b * q1;
    const int TB = (p + 1) * (p + 2) / 2;
    double *lt = jbuf;  // 3 TB: Legendre recurrence table (degrees <= p)
    double *jb = jbuf + 3 * TB + tid * (p + 3);
    if (has_far) {
        for (int e = tid; e < 3 * TB; e += blockDim.x) lt[e] = leg[e];
        __syncthreads();
    }
    for (int t = ts + tid; t < te; t += 64) {
        double2 far = cmk(0, 0), fz = cmk(0, 0), fp = cmk(0, 0), fm = cmk(0, 0);
        if (has_far) {
            const double4 c = ec[t];
            double r, ct, st;
            double2 eph;
            sph_frame(c.x - C.x, c.y - C.y, c.z - C.z, r, ct, st, eph);
            bessel_j_seq(k * r, p, jb);
            double2 e = cmk(1.0, 0.0);
            double spw = 1.0;
            for (int mp = 0; mp <= p; ++mp) {
                if (mp > 0) {
                    e = cmul(e, eph);
                    spw *= st;
                }
                double pm1 = lt[3 * leg_tri(mp, mp) + 2] * spw, pm2 = 0.0;
                double2 sv[2] = {cmk(0, 0), cmk(0, 0)}, sz_[2] = {cmk(0, 0), cmk(0, 0)},
                        sp_[2] = {cmk(0, 0), cmk(0, 0)}, sm_[2] = {cmk(0, 0), cmk(0, 0)};
                for (int nn = mp; nn <= p; ++nn) {
                    if (nn > mp) {
                        const int q = leg_tri(nn, mp);
                        const double P = fma(lt[3 * q] * ct, pm1, -lt[3 * q + 1] * pm2);
                        pm2 = pm1;
                        pm1 = P;
                    }
                    const double R = jb[nn] * pm1;
                    if (nn < p) {
                        sv[0] = cadd(sv[0], cscale(D[cidx(nn, mp)], R));
                        if (mp > 0) sv[1] = cadd(sv[1], cscale(D[cidx(nn, -mp)], R));
                    }
                    sz_[0] = cadd(sz_[0], cscale(Ez[cidx(nn, mp)], R));
                    sp_[0] = cadd(sp_[0], cscale(Ep[cidx(nn, mp)], R));
                    sm_[0] = cadd(sm_[0], cscale(Em[cidx(nn, mp)], R));
                    if (mp > 0) {
                        sz_[1] = cadd(sz_[1], cscale(Ez[cidx(nn, -mp)], R));
                        sp_[1] = cadd(sp_[1], cscale(Ep[cidx(nn, -mp)], R));
                        sm_[1] = cadd(sm_[1], cscale(Em[cidx(nn, -mp)], R));
                    }
                }
                const double2 ep = e, em = cconj(e);
                far = cadd(far, cmul(sv[0], ep));
                fz = cadd(fz, cmul(sz_[0], ep));
                fp = cadd(fp, cmul(sp_[0], ep));
                fm = cadd(fm, cmul(sm_[0], ep));
                if (mp > 0) {
                    far = cadd(far, cmul(sv[1], em));
                    fz = cadd(fz, cmul(sz_[1], em));
                    fp = cadd(fp, cmul(sp_[1], em));
                    fm = cadd(fm, cmul(sm_[1], em));
                }
            }
        }
        const double4 nt = en[t];
        // n.grad = n_z d_z + (n_x - i n_y)/2 (d_x + i d_y) + (n_x + i n_y)/2 (d_x - i d_y)
        double2 farn = cscale(fz, nt.z);
        farn = cadd(farn, cmul(cmk(0.5 * nt.x, -0.5 * nt.y), fp));
        farn = cadd(farn, cmul(cmk(0.5 * nt.x, 0.5 * nt.y), fm));
        const int64_t u = perm[t];
        double2 v1 = cadd(ynear[t], far), v2 = cadd(ynearn[t], farn);
        if (x) {
            const double2 pm = x[u], pp = x[n + u];
            v1 = cadd(v1, cscale(cadd(pm, pp), 0.5));
            // i k (beta- psi- - beta+ psi+) / 2
            const double2 t2 = csub(cmul(bm[t], pm), cmul(bp[t], pp));
            v2 = cadd(v2, cmk(-0.5 * k * t2.y, 0.5 * k * t2.x));
        }
        y[u] = v1;
        y[n + u] = v2;
    }
}

// 2x2 diagonal blocks of the indirect operator (local terms and self entries) and their inverses:
//   [ 1/2 - i k beta- L_ii          1/2 - i k beta+ L_ii  ]
//   [ i k beta-/2 + M'_ii          -i k beta+/2 - M'_ii   ]      (M_ii = L'_ii = 0)
__global__ void k_diag2_inv(int64_t n, const int32_t *near_start, const int32_t *near_col, const double2 *nL,
                            const double2 *nMp, const double2 *bm, const double2 *bp, double k, double shift,
                            double2 *inv) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double2 L = cmk(0, 0), Mp = cmk(0, 0);
    for (int e = near_start[i]; e < near_start[i + 1]; ++e)
        if (near_col[e] == i) {
            L = nL[e];
            Mp = nMp[e];
        }
    const double2 ik = cmk(0, k);
    const double2 a = cadd(cmk(0.5 + shift, 0), cscale(cmul(cmul(ik, bm[i]), L), -1.0));
    const double2 b = csub(cmk(0.5, 0), cmul(cmul(ik, bp[i]), L));
    const double2 c = cadd(cscale(cmul(ik, bm[i]), 0.5), Mp);
    const double2 d = csub(cadd(cscale(cmul(ik, bp[i]), -0.5), cmk(shift, 0)), Mp);
    const double2 det = csub(cmul(a, d), cmul(b, c));
    inv[4 * i] = cdiv(d, det);
    inv[4 * i + 1] = cdiv(cscale(b, -1.0), det);
    inv[4 * i + 2] = cdiv(cscale(c, -1.0), det);
    inv[4 * i + 3] = cdiv(a, det);
}

// z = blockdiag(inv) v on (psi-, psi+) pairs (caller order; inv in tree order)
__global__ void k_mul_diag2(int64_t n, const int32_t *perm, const double2 *inv, const double2 *v, double2 *z) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t u = perm[i];
    const double2 a = v[u], b = v[n + u];
    z[u] = cadd(cmul(inv[4 * i], a), cmul(inv[4 * i + 1], b));
    z[n + u] = cadd(cmul(inv[4 * i + 2], a), cmul(inv[4 * i + 3], b));
}

// ------------------------------------------------------------------ launchers (RHS count 1, 2, 4)
#define FMM_NR_DISPATCH(nr, CALL)                                             \
    switch (nr) {                                                             \
    case 1: CALL(1); break;                                                   \
    case 2: CALL(2); break;                                                   \
    case 4: CALL(4); break;                                                   \
    default: throw FmmError(-1, "right-hand-side chunk must be 1, 2 or 4");  \
    }

void launch_p2p(int nr, bool fp32, int nleaf, const int32_t *leaf_start, const int32_t *nbr_start,
                const int32_t *nbr_list, int all_leaves, const double4 *ec, const double4 *en, const double2 *sigma,
                const double2 *mu, double k, double rc2, const int32_t *near_start, const int32_t *near_col,
                const void *nL, const void *nM, double2 *y, hipStream_t st) {
    if (fp32 && all_leaves) throw FmmError(-1, "the all-pairs near field is an FP64 product");
#define P2P_CALL(R)                                                                                                   \
    if (fp32)                                                                                                         \
        k_p2p32<R><<<nleaf, 64, 0, st>>>(nleaf, leaf_start, nbr_start, nbr_list, ec, en, sigma, mu, k, rc2,          \
                                         near_start, near_col, (const float2 *)nL, (const float2 *)nM, y);           \
    else                                                                                                              \
        k_p2p<R><<<nleaf, 64, 0, st>>>(nleaf, leaf_start, nbr_start, nbr_list, all_leaves, ec, en, sigma, mu, k, rc2, \
                                       near_start, near_col, (const double2 *)nL, (const double2 *)nM, y)
    FMM_NR_DISPATCH(nr, P2P_CALL)
#undef P2P_CALL
    LAUNCH_OK();
}

size_t p2m_stage_bytes(int nr, int p) {
    const int TB = (p + 1) * (p + 2) / 2;
    return (size_t)(TB + 1) * 16 + (size_t)nr * 96 + (size_t)(p + 2) * 8 + 56;  // per staged source
}
size_t p2m_fixed_bytes(int p) { return (size_t)3 * (p + 1) * (p + 2) / 2 * sizeof(double); }

// LDS of the slot-owner kernel: per staged source E (p+1 complex), the weights (4 NR complex), the
// real basis (TB), j_n (p+2) and cos(th); the recurrence table; the slot sums of one vector
// ([8][TB+1] complex) reuse the staging area after the last chunk.
static size_t p2m_slot_stage(int nr, int p) {
    const int TB = (p + 1) * (p + 2) / 2;
    return (size_t)(p + 1) * 16 + (size_t)nr * 64 + (size_t)TB * 8 + (size_t)(p + 2) * 8 + 8;
}
static bool p2m_slot_ok(int p) { return (p + 1) * (p + 2) / 2 <= 256; }
static int p2m_slot_chunk(int nr, int p, size_t &sh) {
    const int TB = (p + 1) * (p + 2) / 2;
    const size_t per = p2m_slot_stage(nr, p), fixed = (size_t)(3 * TB + 2 * BS_TERMS) * 8, sums = (size_t)8 * (TB + 1) * 16;
    // about 40 KB per workgroup (four resident per CU), at least the slot sums' area
    int CH = (int)std::max<size_t>(1, std::min<size_t>(64, (40000 - std::min<size_t>(fixed, 39000)) / per));
    while ((size_t)CH * per < sums) ++CH;
    sh = (size_t)CH * per + fixed;
    return CH;
}

bool p2m_fits(int nr, int p) {
    if (p2m_slot_ok(p)) {
        size_t sh;
        p2m_slot_chunk(nr, p, sh);
        return sh <= 65536;
    }
    return p2m_stage_bytes(nr, p) + p2m_fixed_bytes(p) <= 60000;
}

void launch_p2m(int nr, int nleaf, int p, const int32_t *leaf_start, const double4 *center, const double4 *ec,
                const double4 *en, const double2 *sigma, const double2 *mu, double k, const double *leg,
                double2 *Mout, hipStream_t st) {
    if (nleaf <= 0) return;
    if (p2m_slot_ok(p)) {
        size_t sh;
        const int CH = p2m_slot_chunk(nr, p, sh);
#define P2M_CALL(R) \
    k_p2m<R><<<nleaf, 256, sh, st>>>(nleaf, p, CH, leaf_start, center, ec, en, sigma, mu, k, leg, Mout)
        FMM_NR_DISPATCH(nr, P2M_CALL)
#undef P2M_CALL
    } else {
        const size_t per = p2m_stage_bytes(nr, p), fixed = p2m_fixed_bytes(p);
        const int CH = (int)std::max<size_t>(1, std::min<size_t>(32, (60000 - fixed) / per));
        const size_t sh = (size_t)CH * per + fixed;
#define P2M_CALL(R) \
    k_p2m_wide<R><<<nleaf, 256, sh, st>>>(nleaf, p, CH, leaf_start, center, ec, en, sigma, mu, k, leg, Mout)
        FMM_NR_DISPATCH(nr, P2M_CALL)
#undef P2M_CALL
    }
    LAUNCH_OK();
}

void launch_l2p(int nr, int nleaf, int p, const int32_t *leaf_start, const double4 *center, const double4 *ec,
                const double2 *Lc, double k, const double *leg, const double2 *ynear, double half,
                const int32_t *perm, int64_t n, const double2 *x, double2 *y, int has_far, hipStream_t st) {
    if (nleaf <= 0) return;
    const size_t base = ((size_t)64 * (p + 2) + (size_t)3 * p * (p + 1) / 2 + 2 * BS_TERMS) * sizeof(double);
    const size_t staged = base + (size_t)nr * p * p * 16;
    if (staged <= 48 * 1024) {
#define L2P_CALL(R)                                                                                                   \
    k_l2p<R, true><<<nleaf, 64, staged, st>>>(nleaf, p, leaf_start, center, ec, Lc, k, leg, ynear, half, perm, n, x, y, \
                                              has_far)
        FMM_NR_DISPATCH(nr, L2P_CALL)
#undef L2P_CALL
    } else {
#define L2P_CALL(R)                                                                                                  \
    k_l2p<R, false><<<nleaf, 64, base, st>>>(nleaf, p, leaf_start, center, ec, Lc, k, leg, ynear, half, perm, n, x, y, \
                                             has_far)
        FMM_NR_DISPATCH(nr, L2P_CALL)
#undef L2P_CALL
    }
    LAUNCH_OK();
}

}  // namespace fmm
