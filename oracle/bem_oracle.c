/*
 * CPU oracle for the collocation boundary-element operator -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow, FP64 C written from the paper's definitions.  Only the test suite, the
 * smoke check and the benchmark's CPU-baseline leg may load this library; the product
 * path never does.  It shares no code with the HIP library.
 *
 * What it computes (all with a complex wavenumber k so that damped-k checks are possible):
 *   G(x,y)        = exp(ik|x-y|) / (4 pi |x-y|)                     (Eq. sp6)
 *   L_j(x)        = int_{T_j} G(x,y) dS_y                           (single layer, Eq. dbem2)
 *   M_j(x)        = int_{T_j} dG(x,y)/dn_y dS_y                      (double layer, Eq. dbem2)
 * on flat triangles with constant elements collocated at centroids.  The near/far split
 * follows Section 3.3 (entries of close elements are integrated accurately, far ones by a
 * cheap rule): a pair is "near" iff |c_i - c_j|^2 < rc^2; far pairs use the one-point
 * (centroid) rule; near pairs use recursive 4-way subdivision of T_j with a conical-product
 * Gauss rule on each piece; the self pair uses three sub-triangles with apex at the centroid
 * and a Duffy map, which removes the 1/r singularity.  M_ii is zero (flat element,
 * in-plane collocation point: the principal value of Eq. dbem3 vanishes).
 *
 * For the indirect formulation (Eq. ibem3, ibem5) it also computes, with the normal n_x of the
 * collocation element,
 *   L'_j(x)       = int_{T_j} dG(x,y)/dn_x dS_y                      (zero on the element itself)
 *   M'_j(x)       = d/dn_x int_{T_j} dG(x,y)/dn_y dS_y                (hypersingular)
 * where for the element's own centroid M' is the Hadamard finite part: the in-plane kernel is
 * (1 - ikr) e^{ikr} / (4 pi r^3) = 1/(4 pi r^3) + k^2/(8 pi r) + a bounded rest; the first two
 * parts are integrated in closed form edge by edge, the rest by the same Duffy rule as L.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;

#define PI 3.14159265358979323846

/* ---------------------------------------------------------------- Gauss-Legendre on [0,1] */
static void gauss01(int n, double *x, double *w) {
    for (int i = 0; i < n; ++i) {
        double z = cos(PI * (i + 0.75) / (n + 0.5)), pp = 0.0;
        for (int it = 0; it < 100; ++it) {
            double p1 = 1.0, p2 = 0.0;
            for (int j = 1; j <= n; ++j) {
                double p3 = p2;
                p2 = p1;
                p1 = ((2.0 * j - 1.0) * z * p2 - (j - 1.0) * p3) / j;
            }
            pp = n * (z * p1 - p2) / (z * z - 1.0);
            double z1 = z;
            z = z1 - p1 / pp;
            if (fabs(z - z1) < 1e-15) break;
        }
        x[i] = 0.5 * (1.0 - z);
        w[i] = 1.0 / ((1.0 - z * z) * pp * pp);
    }
}

#define QN 8      /* conical product rule order for regular near pieces */
#define QS 20     /* Duffy rule order for the self integral */
static double gx8[QN], gw8[QN], gxs[QS], gws[QS];
static int rules_ready = 0;
static void init_rules(void) {
    if (rules_ready) return;
    gauss01(QN, gx8, gw8);
    gauss01(QS, gxs, gws);
    rules_ready = 1;
}

/* ---------------------------------------------------------------- small vector helpers */
static inline void sub3(const double *a, const double *b, double *o) { o[0] = a[0] - b[0]; o[1] = a[1] - b[1]; o[2] = a[2] - b[2]; }
static inline double dot3(const double *a, const double *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
static inline void cross3(const double *a, const double *b, double *o) {
    o[0] = a[1] * b[2] - a[2] * b[1];
    o[1] = a[2] * b[0] - a[0] * b[2];
    o[2] = a[0] * b[1] - a[1] * b[0];
}
static inline double norm3(const double *a) { return sqrt(dot3(a, a)); }

/* kernels at a single point: G and dG/dn_y */
static inline void kern(const double *x, const double *y, const double *ny, cplx k, cplx *g, cplx *dgdny) {
    double d[3];
    sub3(y, x, d);
    double r = norm3(d);
    cplx G = cexp(I * k * r) / (4.0 * PI * r);
    *g = G;
    *dgdny = G * (I * k * r - 1.0) * dot3(d, ny) / (r * r);
}

/* the two normal-derivative kernels: dG/dn_x and d^2 G / dn_x dn_y (with d = y - x):
 *   dG/dn_x        = G (ikr - 1) ((x - y).n_x) / r^2
 *   d2G/dn_x dn_y  = -e^{ikr} (3 - 3ikr - k^2 r^2) (d.n_x)(d.n_y) / (4 pi r^5)
 *                    - e^{ikr} (ikr - 1) (n_x.n_y) / (4 pi r^3)                              */
static inline void kern_n(const double *x, const double *nx, const double *y, const double *ny, cplx k, cplx *g,
                          cplx *dgdny, cplx *dgdnx, cplx *d2g) {
    double d[3];
    sub3(y, x, d);
    double r = norm3(d), r2 = r * r;
    cplx e = cexp(I * k * r) / (4.0 * PI);
    cplx G = e / r;
    double dnx = dot3(d, nx), dny = dot3(d, ny);
    *g = G;
    *dgdny = G * (I * k * r - 1.0) * dny / r2;
    *dgdnx = -G * (I * k * r - 1.0) * dnx / r2;
    *d2g = -e * (3.0 - 3.0 * I * k * r - k * k * r2) * dnx * dny / (r2 * r2 * r) - e * (I * k * r - 1.0) * dot3(nx, ny) / (r2 * r);
}

/* ---------------------------------------------------------------- geometry */
void oracle_geometry(int64_t nt, const double *V, const int64_t *T, double *c, double *nrm, double *area) {
    for (int64_t j = 0; j < nt; ++j) {
        const double *a = V + 3 * T[3 * j], *b = V + 3 * T[3 * j + 1], *e = V + 3 * T[3 * j + 2];
        double u[3], v[3], w[3];
        sub3(b, a, u);
        sub3(e, a, v);
        cross3(u, v, w);
        double l = norm3(w);
        for (int q = 0; q < 3; ++q) {
            c[3 * j + q] = (a[q] + b[q] + e[q]) / 3.0;
            nrm[3 * j + q] = w[q] / l;
        }
        area[j] = 0.5 * l;
    }
}

/* ---------------------------------------------------------------- triangle integrals */
/* conical-product rule on triangle (a,b,e): y = a + s(b-a) + s t (e-b), dS = 2A s ds dt */
static void rule_tri(const double *x, const double *a, const double *b, const double *e, const double *ny, cplx k,
                     cplx *L, cplx *M) {
    double u[3], v[3], w[3];
    sub3(b, a, u);
    sub3(e, b, v);
    cross3(u, v, w);
    double twoA = norm3(w);
    cplx sl = 0, sm = 0;
    for (int i = 0; i < QN; ++i) {
        double s = gx8[i];
        for (int j = 0; j < QN; ++j) {
            double t = gx8[j], y[3];
            for (int q = 0; q < 3; ++q) y[q] = a[q] + s * u[q] + s * t * v[q];
            cplx g, dg;
            kern(x, y, ny, k, &g, &dg);
            double wt = gw8[i] * gw8[j] * twoA * s;
            sl += wt * g;
            sm += wt * dg;
        }
    }
    *L += sl;
    *M += sm;
}

static void adapt_tri(const double *x, const double *a, const double *b, const double *e, const double *ny, cplx k,
                      double eta, int depth, cplx *L, cplx *M) {
    double cen[3], d[3], ab[3], be[3], ea[3];
    for (int q = 0; q < 3; ++q) cen[q] = (a[q] + b[q] + e[q]) / 3.0;
    sub3(cen, x, d);
    sub3(b, a, ab);
    sub3(e, b, be);
    sub3(a, e, ea);
    double diam = fmax(norm3(ab), fmax(norm3(be), norm3(ea)));
    if (diam < eta * norm3(d) || depth >= 14) {
        rule_tri(x, a, b, e, ny, k, L, M);
        return;
    }
    double mab[3], mbe[3], mea[3];
    for (int q = 0; q < 3; ++q) {
        mab[q] = 0.5 * (a[q] + b[q]);
        mbe[q] = 0.5 * (b[q] + e[q]);
        mea[q] = 0.5 * (e[q] + a[q]);
    }
    adapt_tri(x, a, mab, mea, ny, k, eta, depth + 1, L, M);
    adapt_tri(x, mab, b, mbe, ny, k, eta, depth + 1, L, M);
    adapt_tri(x, mea, mbe, e, ny, k, eta, depth + 1, L, M);
    adapt_tri(x, mab, mbe, mea, ny, k, eta, depth + 1, L, M);
}

/* the same conical rule and subdivision for the four kernels (L, M, L', M') */
static void rule_tri4(const double *x, const double *nx, const double *a, const double *b, const double *e,
                      const double *ny, cplx k, cplx *out) {
    double u[3], v[3], w[3];
    sub3(b, a, u);
    sub3(e, b, v);
    cross3(u, v, w);
    double twoA = norm3(w);
    cplx s[4] = {0, 0, 0, 0};
    for (int i = 0; i < QN; ++i) {
        double sp = gx8[i];
        for (int j = 0; j < QN; ++j) {
            double t = gx8[j], y[3];
            for (int q = 0; q < 3; ++q) y[q] = a[q] + sp * u[q] + sp * t * v[q];
            cplx g, dg, dgx, d2;
            kern_n(x, nx, y, ny, k, &g, &dg, &dgx, &d2);
            double wt = gw8[i] * gw8[j] * twoA * sp;
            s[0] += wt * g;
            s[1] += wt * dg;
            s[2] += wt * dgx;
            s[3] += wt * d2;
        }
    }
    for (int q = 0; q < 4; ++q) out[q] += s[q];
}

static void adapt_tri4(const double *x, const double *nx, const double *a, const double *b, const double *e,
                       const double *ny, cplx k, double eta, int depth, cplx *out) {
    double cen[3], d[3], ab[3], be[3], ea[3];
    for (int q = 0; q < 3; ++q) cen[q] = (a[q] + b[q] + e[q]) / 3.0;
    sub3(cen, x, d);
    sub3(b, a, ab);
    sub3(e, b, be);
    sub3(a, e, ea);
    double diam = fmax(norm3(ab), fmax(norm3(be), norm3(ea)));
    if (diam < eta * norm3(d) || depth >= 16) {
        rule_tri4(x, nx, a, b, e, ny, k, out);
        return;
    }
    double mab[3], mbe[3], mea[3];
    for (int q = 0; q < 3; ++q) {
        mab[q] = 0.5 * (a[q] + b[q]);
        mbe[q] = 0.5 * (b[q] + e[q]);
        mea[q] = 0.5 * (e[q] + a[q]);
    }
    adapt_tri4(x, nx, a, mab, mea, ny, k, eta, depth + 1, out);
    adapt_tri4(x, nx, mab, b, mbe, ny, k, eta, depth + 1, out);
    adapt_tri4(x, nx, mea, mbe, e, ny, k, eta, depth + 1, out);
    adapt_tri4(x, nx, mab, mbe, mea, ny, k, eta, depth + 1, out);
}

/* Finite part of M' over the collocation element itself (x in the plane of T).
 *   f.p. int_T dS / (4 pi r^3) = -(1/4pi) oint dtheta / R(theta): for the edge (va, vb) seen
 *   from x at perpendicular distance h, with signed positions s_a, s_b of va, vb along the
 *   edge from the foot of the perpendicular, the angular integral is (s_b/|x-vb| - s_a/|x-va|)/h;
 *   int_T dS / r = sum over edges h (asinh(s_b/h) - asinh(s_a/h));
 *   the rest [e^{ikr}(1 - ikr) - 1 - k^2 r^2/2] / (4 pi r^3) is bounded and integrated with
 *   the Duffy rule of self_L (series in ikr for small |kr|, where the difference cancels). */
static cplx rest_mp(cplx k, double r) {
    cplx z = I * k * r;
    if (cabs(z) < 0.5) {
        /* e^z (1 - z) - 1 + z^2/2 = sum_{n>=3} (1 - n) z^n / n! */
        cplx term = z * z / 2.0, s = 0;
        for (int n = 3; n < 30; ++n) {
            term *= z / n;
            s += (1.0 - n) * term;
        }
        return s / (4.0 * PI * r * r * r);
    }
    return (cexp(z) * (1.0 - z) - 1.0 + z * z / 2.0) / (4.0 * PI * r * r * r);
}

static cplx self_Mp(const double *x, const double *p0, const double *p1, const double *p2, cplx k) {
    enum { NPT = 8 };
    const double *P[3] = {p0, p1, p2};
    double fp_inv_r3 = 0.0, int_inv_r = 0.0;
    cplx rest = 0;
    for (int e = 0; e < 3; ++e) {
        const double *va = P[e], *vb = P[(e + 1) % 3];
        double ev[3], xa[3];
        sub3(vb, va, ev);
        double len = norm3(ev);
        for (int q = 0; q < 3; ++q) ev[q] /= len;
        sub3(va, x, xa);
        double sa = dot3(xa, ev), sb = sa + len, perp[3];
        for (int q = 0; q < 3; ++q) perp[q] = xa[q] - sa * ev[q];
        double h = norm3(perp);
        double ra = sqrt(sa * sa + h * h), rb = sqrt(sb * sb + h * h);
        fp_inv_r3 += (sb / rb - sa / ra) / h;
        int_inv_r += h * (asinh(sb / h) - asinh(sa / h));
        /* Duffy rule for the bounded rest on the sub-triangle (x, va, vb) */
        double u[3], v[3], w[3];
        sub3(va, x, u);
        sub3(vb, va, v);
        cross3(u, v, w);
        double twoA = norm3(w);
        for (int pt = 0; pt < NPT; ++pt) {
            for (int j = 0; j < QS; ++j) {
                double t = (pt + gxs[j]) / NPT, wt = gws[j] / NPT, d[3];
                for (int q = 0; q < 3; ++q) d[q] = u[q] + t * v[q];
                double rho = norm3(d);
                for (int i = 0; i < QS; ++i) {
                    double r = gxs[i] * rho;
                    rest += gws[i] * wt * twoA * gxs[i] * rest_mp(k, r);  /* dS = twoA s ds dt */
                }
            }
        }
    }
    return -fp_inv_r3 / (4.0 * PI) + k * k * int_inv_r / (8.0 * PI) + rest;
}

/* self integral of G over T with the collocation point x = centroid: three sub-triangles
 * (x, v_a, v_b) with a Duffy map y = x + s(v_a - x) + s t (v_b - v_a); the Jacobian 2A_sub*s
 * cancels the 1/r singularity. */
static cplx self_L(const double *x, const double *p0, const double *p1, const double *p2, cplx k) {
    /* the t-integrand 1/rho(t) has complex poles at distance (edge height / edge length)
     * from [0,1]; NPT panels in t keep the Gauss rule far from them */
    enum { NPT = 8 };
    const double *P[3] = {p0, p1, p2};
    cplx sum = 0;
    for (int e = 0; e < 3; ++e) {
        const double *va = P[e], *vb = P[(e + 1) % 3];
        double u[3], v[3], w[3];
        sub3(va, x, u);
        sub3(vb, va, v);
        cross3(u, v, w);
        double twoA = norm3(w);
        for (int pt = 0; pt < NPT; ++pt) {
            for (int j = 0; j < QS; ++j) {
                double t = (pt + gxs[j]) / NPT, wt = gws[j] / NPT, d[3];
                for (int q = 0; q < 3; ++q) d[q] = u[q] + t * v[q];
                double rho = norm3(d); /* r = s*rho */
                for (int i = 0; i < QS; ++i)
                    sum += gws[i] * wt * twoA * cexp(I * k * gxs[i] * rho) / (4.0 * PI * rho);
            }
        }
    }
    return sum;
}

/* accurate L_j(x), M_j(x) for an arbitrary point x (not on T_j unless it is T_j's centroid,
 * which the caller flags with self=1) */
static void accurate_LM(const double *x, const double *V, const int64_t *tri, const double *ny, cplx k, int self,
                        double eta, cplx *L, cplx *M) {
    const double *a = V + 3 * tri[0], *b = V + 3 * tri[1], *e = V + 3 * tri[2];
    if (self) {
        *L = self_L(x, a, b, e, k);
        *M = 0.0;
        return;
    }
    cplx l = 0, m = 0;
    adapt_tri(x, a, b, e, ny, k, eta, 0, &l, &m);
    *L = l;
    *M = m;
}

/* L_ij, M_ij for collocation point i (centroid c_i) and element j */
static void pair_LM(int64_t i, int64_t j, const double *V, const int64_t *T, const double *c, const double *nrm,
                    const double *area, cplx k, double rc2, double eta, cplx *L, cplx *M) {
    const double *x = c + 3 * i, *y = c + 3 * j;
    double d[3];
    sub3(y, x, d);
    double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
    if (i == j) {
        accurate_LM(x, V, T + 3 * j, nrm + 3 * j, k, 1, eta, L, M);
    } else if (r2 < rc2) {
        accurate_LM(x, V, T + 3 * j, nrm + 3 * j, k, 0, eta, L, M);
    } else {
        cplx g, dg;
        kern(x, y, nrm + 3 * j, k, &g, &dg);
        *L = g * area[j];
        *M = dg * area[j];
    }
}

/* ---------------------------------------------------------------- exported entry points */
/* Dense L and M (row-major, N x N, complex interleaved). */
void oracle_dense_LM(int64_t nv, const double *V, int64_t nt, const int64_t *T, double kr, double ki, double rc,
                     double eta, double *Lout, double *Mout) {
    (void)nv;
    init_rules();
    cplx k = kr + I * ki;
    double *c = malloc(sizeof(double) * 3 * nt), *nrm = malloc(sizeof(double) * 3 * nt), *area = malloc(sizeof(double) * nt);
    oracle_geometry(nt, V, T, c, nrm, area);
    double rc2 = rc * rc;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < nt; ++i) {
        for (int64_t j = 0; j < nt; ++j) {
            cplx L, M;
            pair_LM(i, j, V, T, c, nrm, area, k, rc2, eta, &L, &M);
            Lout[2 * (i * nt + j)] = creal(L);
            Lout[2 * (i * nt + j) + 1] = cimag(L);
            Mout[2 * (i * nt + j)] = creal(M);
            Mout[2 * (i * nt + j) + 1] = cimag(M);
        }
    }
    free(c);
    free(nrm);
    free(area);
}

/* Matrix-free rows of  y_i = sum_j [ L_ij sigma_j + M_ij mu_j ]  for the listed rows. */
void oracle_layer_rows(int64_t nv, const double *V, int64_t nt, const int64_t *T, double kr, double ki, double rc,
                       double eta, int64_t nrows, const int64_t *rows, const double *sigma, const double *mu,
                       double *yout) {
    (void)nv;
    init_rules();
    cplx k = kr + I * ki;
    double *c = malloc(sizeof(double) * 3 * nt), *nrm = malloc(sizeof(double) * 3 * nt), *area = malloc(sizeof(double) * nt);
    oracle_geometry(nt, V, T, c, nrm, area);
    double rc2 = rc * rc;
    const cplx *sg = (const cplx *)sigma, *m = (const cplx *)mu;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t r = 0; r < nrows; ++r) {
        int64_t i = rows[r];
        cplx acc = 0;
        for (int64_t j = 0; j < nt; ++j) {
            cplx L, M;
            pair_LM(i, j, V, T, c, nrm, area, k, rc2, eta, &L, &M);
            acc += L * sg[j] + M * m[j];
        }
        yout[2 * r] = creal(acc);
        yout[2 * r + 1] = cimag(acc);
    }
    free(c);
    free(nrm);
    free(area);
}

/* Layer potentials at off-surface points: out_p = sum_j [ L_j(r_p) sigma_j + M_j(r_p) mu_j ].
 * An element is integrated accurately when |r_p - c_j|^2 < rc^2, else by the centroid rule. */
void oracle_field(int64_t nv, const double *V, int64_t nt, const int64_t *T, double kr, double ki, double rc,
                  double eta, int64_t np, const double *pts, const double *sigma, const double *mu, double *out) {
    (void)nv;
    init_rules();
    cplx k = kr + I * ki;
    double *c = malloc(sizeof(double) * 3 * nt), *nrm = malloc(sizeof(double) * 3 * nt), *area = malloc(sizeof(double) * nt);
    oracle_geometry(nt, V, T, c, nrm, area);
    double rc2 = rc * rc;
    const cplx *sg = (const cplx *)sigma, *m = (const cplx *)mu;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t p = 0; p < np; ++p) {
        const double *x = pts + 3 * p;
        cplx acc = 0;
        for (int64_t j = 0; j < nt; ++j) {
            double d[3];
            sub3(c + 3 * j, x, d);
            double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
            cplx L, M;
            if (r2 < rc2) {
                accurate_LM(x, V, T + 3 * j, nrm + 3 * j, k, 0, eta, &L, &M);
            } else {
                cplx g, dg;
                kern(x, c + 3 * j, nrm + 3 * j, k, &g, &dg);
                L = g * area[j];
                M = dg * area[j];
            }
            acc += L * sg[j] + M * m[j];
        }
        out[2 * p] = creal(acc);
        out[2 * p + 1] = cimag(acc);
    }
    free(c);
    free(nrm);
    free(area);
}

/* One accurate pair integral (for pinning the quadrature against brute force). */
void oracle_pair(const double *x, const double *tri_xyz, double kr, double ki, int self, double eta, double *LM) {
    init_rules();
    int64_t t3[3] = {0, 1, 2};
    double u[3], v[3], w[3];
    sub3(tri_xyz + 3, tri_xyz, u);
    sub3(tri_xyz + 6, tri_xyz, v);
    cross3(u, v, w);
    double l = norm3(w), ny[3] = {w[0] / l, w[1] / l, w[2] / l};
    cplx L, M;
    accurate_LM(x, tri_xyz, t3, ny, kr + I * ki, self, eta, &L, &M);
    LM[0] = creal(L);
    LM[1] = cimag(L);
    LM[2] = creal(M);
    LM[3] = cimag(M);
}

/* ---------------------------------------------------------------- indirect formulation */
/* L, M, L', M' of element j at the centroid of element i (normal n_i), with the same near/far
 * classification as pair_LM */
static void pair_4(int64_t i, int64_t j, const double *V, const int64_t *T, const double *c, const double *nrm,
                   const double *area, cplx k, double rc2, double eta, cplx *out) {
    const double *x = c + 3 * i, *y = c + 3 * j, *nx = nrm + 3 * i, *ny = nrm + 3 * j;
    double d[3];
    sub3(y, x, d);
    double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
    const int64_t *tri = T + 3 * j;
    const double *a = V + 3 * tri[0], *b = V + 3 * tri[1], *e = V + 3 * tri[2];
    if (i == j) {
        out[0] = self_L(x, a, b, e, k);
        out[1] = 0.0;
        out[2] = 0.0;
        out[3] = self_Mp(x, a, b, e, k);
    } else if (r2 < rc2) {
        for (int q = 0; q < 4; ++q) out[q] = 0;
        adapt_tri4(x, nx, a, b, e, ny, k, eta, 0, out);
    } else {
        cplx g, dg, dgx, d2;
        kern_n(x, nx, y, ny, k, &g, &dg, &dgx, &d2);
        out[0] = g * area[j];
        out[1] = dg * area[j];
        out[2] = dgx * area[j];
        out[3] = d2 * area[j];
    }
}

/* Dense L, M, L', M' (row-major N x N complex interleaved each). */
void oracle_dense_LMn(int64_t nv, const double *V, int64_t nt, const int64_t *T, double kr, double ki, double rc,
                      double eta, double *Lout, double *Mout, double *Lpout, double *Mpout) {
    (void)nv;
    init_rules();
    cplx k = kr + I * ki;
    double *c = malloc(sizeof(double) * 3 * nt), *nrm = malloc(sizeof(double) * 3 * nt), *area = malloc(sizeof(double) * nt);
    oracle_geometry(nt, V, T, c, nrm, area);
    double rc2 = rc * rc;
    double *outs[4] = {Lout, Mout, Lpout, Mpout};
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < nt; ++i) {
        for (int64_t j = 0; j < nt; ++j) {
            cplx v[4];
            pair_4(i, j, V, T, c, nrm, area, k, rc2, eta, v);
            for (int q = 0; q < 4; ++q) {
                outs[q][2 * (i * nt + j)] = creal(v[q]);
                outs[q][2 * (i * nt + j) + 1] = cimag(v[q]);
            }
        }
    }
    free(c);
    free(nrm);
    free(area);
}

/* Matrix-free rows of y_i = sum_j [L_ij s_j + M_ij m_j] and yn_i = sum_j [L'_ij s_j + M'_ij m_j]. */
void oracle_layer_rows_n(int64_t nv, const double *V, int64_t nt, const int64_t *T, double kr, double ki, double rc,
                         double eta, int64_t nrows, const int64_t *rows, const double *sigma, const double *mu,
                         double *yout, double *ynout) {
    (void)nv;
    init_rules();
    cplx k = kr + I * ki;
    double *c = malloc(sizeof(double) * 3 * nt), *nrm = malloc(sizeof(double) * 3 * nt), *area = malloc(sizeof(double) * nt);
    oracle_geometry(nt, V, T, c, nrm, area);
    double rc2 = rc * rc;
    const cplx *sg = (const cplx *)sigma, *m = (const cplx *)mu;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t r = 0; r < nrows; ++r) {
        int64_t i = rows[r];
        cplx acc = 0, accn = 0;
        for (int64_t j = 0; j < nt; ++j) {
            cplx v[4];
            pair_4(i, j, V, T, c, nrm, area, k, rc2, eta, v);
            acc += v[0] * sg[j] + v[1] * m[j];
            accn += v[2] * sg[j] + v[3] * m[j];
        }
        yout[2 * r] = creal(acc);
        yout[2 * r + 1] = cimag(acc);
        ynout[2 * r] = creal(accn);
        ynout[2 * r + 1] = cimag(accn);
    }
    free(c);
    free(nrm);
    free(area);
}

/* One accurate pair of all four integrals at x with normal nx (self=1: x is T's centroid and
 * nx its normal); out = L, M, L', M' interleaved. */
void oracle_pair4(const double *x, const double *nx, const double *tri_xyz, double kr, double ki, int self,
                  double eta, double *out) {
    init_rules();
    double u[3], v[3], w[3];
    sub3(tri_xyz + 3, tri_xyz, u);
    sub3(tri_xyz + 6, tri_xyz, v);
    cross3(u, v, w);
    double l = norm3(w), ny[3] = {w[0] / l, w[1] / l, w[2] / l};
    cplx k = kr + I * ki, r[4] = {0, 0, 0, 0};
    const double *a = tri_xyz, *b = tri_xyz + 3, *e = tri_xyz + 6;
    if (self) {
        r[0] = self_L(x, a, b, e, k);
        r[3] = self_Mp(x, a, b, e, k);
    } else {
        adapt_tri4(x, nx, a, b, e, ny, k, eta, 0, r);
    }
    for (int q = 0; q < 4; ++q) {
        out[2 * q] = creal(r[q]);
        out[2 * q + 1] = cimag(r[q]);
    }
}
