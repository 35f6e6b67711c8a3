// FP64 device generation of the FMM operator tables.
//
//  * spherical Bessel sequences j_n(x), y_n(x), n = 0..N: y_n by forward recurrence (stable,
//    growing), j_n by Miller's backward recurrence normalised against j_0 or j_1.
//  * coaxial translation coefficients (E|F)^m_{n'n}(tau) of Eq. (shft0.1), E|F = S|R or R|R,
//    by the recursions of Section 3.3.1:
//      step 1  zonal seed (Eq. shft1),
//      step 2  sectorial coefficients, propagation in m (Eq. shft2),
//      original step 3: tesseral coefficients by propagation in n (Eq. shft5, range shft4),
//      stabilised scheme (k tau >= switch): zonal block by propagation in n (step 3.1, Eq. shft7),
//        diagonal and the two sub-diagonals by propagation in m (step 3.2, Eq. shft8), then the
//        interior by propagation in n' (Eq. shift6), and step 4 symmetry for n' < n.
//    In the third line of Eq. (shft8) the coefficient multiplying (E|F)^m_{n+1,n-1} is taken as
//    b_n^{-m-1}: this is what the m-recurrence that gives the first two lines yields, and the
//    printed b_{n+1}^{-m-1} does not reproduce the coefficients.
//  * rotation matrices Delta^n = T^n(R_y(pi/2)) (real), used to factor every rotation about the
//    y axis as R_y(beta) = R_x(-pi/2) R_z(beta) R_x(pi/2): the z rotations are diagonal phases,
//    so one table of quarter-turn matrices serves all directions.  G = eps_m eps_m' Delta
//    (eps_m = (-1)^m for m < 0, else 1) satisfies
//      sqrt((n-m')(n+m'+1)) G_{m,m'+1} + sqrt((n+m')(n-m'+1)) G_{m,m'-1} + 2 m G_{m,m'} = 0,
//    with edge column G_{m,n} = sqrt(C(2n, n+m)) 2^-n and G_{m,-m'} = (-1)^(n+m) G_{m,m'}.
//    The recurrence is run downward in m' from the edge to 0, where the wanted solution grows
//    or oscillates, never decays, so it is stable to high degree (the quarter-turn factorisation
//    is a Fourier-series evaluation of Wigner matrices, e.g. Risbo 1996).
#include "common.h"
#include "internal.h"

namespace fmm {

// ------------------------------------------------------------------ coaxial tables
// Workspace layout per table (complex): seq[2P], S[P][2P] sectorial, Z[2P][P+2] zonal,
// D0/D1/D2[P+2][P+2] diagonals, with P = p + 2.
struct CoaxWS {
    int p, W;  // W = 2p + 4 row stride
    double2 *base;
    __device__ double2 *seq() const { return base; }
    __device__ double2 &S(int m, int nn) const { return base[W + (int64_t)m * W + nn]; }
    __device__ double2 &Z(int nn, int n) const { return base[W + (int64_t)(p + 2) * W + (int64_t)nn * (p + 4) + n]; }
    __device__ double2 &D(int which, int m, int n) const {
        return base[W + (int64_t)(p + 2) * W + (int64_t)W * (p + 4) + (int64_t)which * (p + 4) * (p + 4) +
                    (int64_t)m * (p + 4) + n];
    }
};
int64_t coax_ws_size(int p) {
    int64_t W = 2 * p + 4;
    return W + (p + 2) * W + W * (p + 4) + 3 * (int64_t)(p + 4) * (p + 4);
}

// kernel 1: one workgroup per table.  seq, sectorial, zonal and diagonal coefficients.
__global__ void __launch_bounds__(256) k_coax_prepare(const CoaxJob *jobs, double2 *ws_base, int64_t ws_stride) {
    const CoaxJob J = jobs[blockIdx.x];
    const int p = J.p;
    CoaxWS ws{p, 2 * p + 4, ws_base + ws_stride * blockIdx.x};
    const int N = 2 * p;  // orders 0..2p-1
    __shared__ double jb[2 * 1024 + 8];
    __shared__ double yb[2 * 1024 + 8];
    if (threadIdx.x == 0) {
        sph_jn_seq(J.ktau, N, jb);
        if (J.kind == 0) sph_yn_seq(J.ktau, N, yb);
    }
    __syncthreads();
    // step 1, Eq. (shft1): (E|F)^0_{n'0} = (-1)^n' sqrt(2n'+1) f_n'(k tau)
    for (int nn = threadIdx.x; nn <= 2 * p - 2; nn += blockDim.x) {
        double sg = (nn & 1) ? -1.0 : 1.0;
        double r = sg * sqrt(2.0 * nn + 1.0);
        ws.S(0, nn) = cmk(r * jb[nn], J.kind == 0 ? r * yb[nn] : 0.0);
    }
    __syncthreads();
    // step 2, Eq. (shft2): sectorial, propagation in m
    for (int m = 0; m <= p - 2; ++m) {
        double bden = coef_b(m + 1, -m - 1);
        for (int nn = m + 1 + threadIdx.x; nn <= 2 * p - 3 - m; nn += blockDim.x) {
            double2 v = csub(cscale(ws.S(m, nn - 1), coef_b(nn, -m - 1)), cscale(ws.S(m, nn + 1), coef_b(nn + 1, m)));
            ws.S(m + 1, nn) = cscale(v, 1.0 / bden);
        }
        __syncthreads();
    }
    if (J.method == 0) return;
    // step 3.1, Eq. (shft7): zonal block by propagation in n
    for (int nn = threadIdx.x; nn <= 2 * p - 2; nn += blockDim.x) ws.Z(nn, 0) = ws.S(0, nn);
    __syncthreads();
    for (int n = 0; n <= p - 2; ++n) {
        double an = coef_a(n, 0), an1 = (n >= 1) ? coef_a(n - 1, 0) : 0.0;
        for (int nn = n + 1 + threadIdx.x; nn <= 2 * p - n - 3; nn += blockDim.x) {
            double2 v = cscale(ws.Z(nn + 1, n), -coef_a(nn, 0));
            v = cadd(v, cscale(ws.Z(nn - 1, n), coef_a(nn - 1, 0)));
            if (n >= 1) v = cadd(v, cscale(ws.Z(nn, n - 1), an1));
            ws.Z(nn, n + 1) = cscale(v, 1.0 / an);
        }
        __syncthreads();
    }
    // step 3.2, Eq. (shft8): diagonals by propagation in m (sequential chain)
    if (threadIdx.x == 0) {
        for (int n = 0; n <= p - 1; ++n) {
            ws.D(0, 0, n) = ws.Z(n, n);
            ws.D(1, 0, n) = ws.Z(n + 1, n);
            ws.D(2, 0, n) = ws.Z(n + 2, n);
        }
        for (int m = 0; m <= p - 3; ++m) {
            const int M = m + 1;
            ws.D(0, M, M) = ws.S(M, M);
            ws.D(1, M, M) = ws.S(M, M + 1);
            ws.D(2, M, M) = ws.S(M, M + 2);
            for (int n = m + 1; n <= p - 2; ++n) {
                const double bnp1 = coef_b(n + 1, -m - 1);
                // (E|F)^{m+1}_{n+1,n+1}
                double2 v = cscale(ws.D(0, m, n), bnp1);
                v = csub(v, cscale(ws.D(2, m, n), coef_b(n + 2, m)));
                if (n - 1 >= M) v = cadd(v, cscale(ws.D(2, M, n - 1), coef_b(n, m)));
                ws.D(0, M, n + 1) = cscale(v, 1.0 / bnp1);
                if (n >= m + 2) {
                    // (E|F)^{m+1}_{n+1,n}
                    double2 w = cscale(ws.D(1, m, n), coef_b(n + 1, m));
                    w = cadd(w, cscale(ws.D(1, m, n - 1), coef_b(n, -m - 1)));
                    w = csub(w, cscale(ws.D(1, M, n - 1), coef_b(n, m)));
                    ws.D(1, M, n) = cscale(w, 1.0 / bnp1);
                    // (E|F)^{m+1}_{n+2,n}  (coefficient of (E|F)^m_{n+1,n-1} read as b_n^{-m-1})
                    double2 u = cscale(ws.D(0, M, n), coef_b(n + 1, m));
                    u = csub(u, cscale(ws.D(0, m, n + 1), coef_b(n + 1, m)));
                    u = cadd(u, cscale(ws.D(2, m, n - 1), coef_b(n, -m - 1)));
                    ws.D(2, M, n) = cscale(u, 1.0 / coef_b(n + 2, -m - 1));
                }
            }
        }
    }
}

// kernel 2: one workgroup per (table, m).  Fills block m of the output table.
__global__ void __launch_bounds__(256) k_coax_fill(const CoaxJob *jobs, double2 *ws_base, int64_t ws_stride) {
    const CoaxJob J = jobs[blockIdx.y];
    const int p = J.p;
    const int m = blockIdx.x;
    if (m >= p) return;
    CoaxWS ws{p, 2 * p + 4, ws_base + ws_stride * blockIdx.y};
    double2 *out = J.out + coax_block_off(p, m);
    const int B = p - m;  // block edge
    auto put = [&](int nn, int n, double2 v) { out[(int64_t)(nn - m) * B + (n - m)] = v; };
    __shared__ double2 rows[3][1024 + 8];

    if (J.method == 0) {
        // original scheme, Eq. (shft5) over the range (shft4): propagate columns in n
        double2 *c0 = rows[0], *c1 = rows[1], *c2 = rows[2];  // columns n-1, n, n+1 indexed by n'
        const int top = 2 * p - 2 - m;
        for (int nn = m + threadIdx.x; nn <= top; nn += blockDim.x) {
            c1[nn] = ws.S(m, nn);
            c0[nn] = cmk(0, 0);
            if (nn < p) put(nn, m, c1[nn]);
        }
        __syncthreads();
        for (int n = m; n <= p - 2; ++n) {
            const double an = coef_a(n, m), anm1 = coef_a(n - 1, m);
            const int hi = 2 * p - 3 - n;
            for (int nn = m + threadIdx.x; nn <= hi; nn += blockDim.x) {
                double2 v = csub(cscale(c0[nn], anm1), cscale(c1[nn + 1], coef_a(nn, m)));
                if (nn - 1 >= m) v = cadd(v, cscale(c1[nn - 1], coef_a(nn - 1, m)));
                v = cscale(v, 1.0 / an);
                c2[nn] = v;
                if (nn < p) put(nn, n + 1, v);
            }
            __syncthreads();
            double2 *t = c0;
            c0 = c1;
            c1 = c2;
            c2 = t;
        }
        return;
    }

    if (m == 0) {
        for (int e = threadIdx.x; e < p * p; e += blockDim.x) {
            int nn = e / p, n = e % p;
            double2 v = (nn >= n) ? ws.Z(nn, n) : cscale(ws.Z(n, nn), ((n + nn) & 1) ? -1.0 : 1.0);
            put(nn, n, v);
        }
        return;
    }
    auto put_sym = [&](int nn, int n, double2 v) {  // lower entry and its step-4 mirror
        put(nn, n, v);
        if (nn != n) put(n, nn, cscale(v, ((n + nn) & 1) ? -1.0 : 1.0));
    };
    // rows n' are built in a 3-row window: r[n' % 3][n]
    for (int nn = m + threadIdx.x; nn < p; nn += blockDim.x) {
        // sectorial column and the three diagonals
        put_sym(nn, m, ws.S(m, nn));
    }
    for (int n = m + 1 + threadIdx.x; n < p; n += blockDim.x) {
        put_sym(n, n, ws.D(0, m, n));
        if (n + 1 < p) put_sym(n + 1, n, ws.D(1, m, n));
        if (n + 2 < p) put_sym(n + 2, n, ws.D(2, m, n));
    }
    // window init with rows m+2 and m+3 (lower-triangle entries only; cols m..row)
    auto row_val = [&](int nn, int n) -> double2 {  // only valid for n' - n <= 2 or n == m
        if (n == m) return ws.S(m, nn);
        int d = nn - n;
        return ws.D(d, m, n);
    };
    for (int n = m + threadIdx.x; n <= m + 3 && n < p; n += blockDim.x) {
        if (m + 2 < p && n <= m + 2) rows[(m + 2) % 3][n] = row_val(m + 2, n);
        if (m + 3 < p) rows[(m + 3) % 3][n] = row_val(m + 3, n);
    }
    __syncthreads();
    // Eq. (shift6): propagation in n' for n' = m+3..p-2, n = m+1..n'-2
    for (int nn = m + 3; nn <= p - 2; ++nn) {
        double2 *rp = rows[nn % 3], *rm = rows[(nn - 1) % 3], *rn = rows[(nn + 1) % 3];
        const double inv = 1.0 / coef_a(nn, m), amm = coef_a(nn - 1, m);
        for (int n = m + threadIdx.x; n <= nn + 1; n += blockDim.x) {
            double2 v;
            if (n == m || nn + 1 - n <= 2) {
                v = row_val(nn + 1, n);
            } else {
                v = cscale(rp[n - 1], coef_a(n - 1, m));
                v = csub(v, cscale(rp[n + 1], coef_a(n, m)));
                v = cadd(v, cscale(rm[n], amm));
                v = cscale(v, inv);
                put_sym(nn + 1, n, v);
            }
            rn[n] = v;
        }
        __syncthreads();
    }
}

void build_coax_tables(const std::vector<CoaxJob> &jobs, DeviceBuffers &scratch, hipStream_t st) {
    if (jobs.empty()) return;
    int pmax = 0;
    for (auto &j : jobs) pmax = std::max(pmax, j.p);
    if (pmax > 1000) throw FmmError(-1, "truncation number above 1000 is not supported");
    for (auto &j : jobs)  // the original scheme keeps columns of length 2p-1 in LDS
        if (j.method == 0 && j.p > 512) throw FmmError(-1, "original coaxial recursion limited to p <= 512");
    int64_t wsz = coax_ws_size(pmax);
    // process in groups so the workspace stays bounded (~1 GiB)
    int64_t per = std::max<int64_t>(1, (int64_t(1) << 26) / wsz);
    CoaxJob *djobs = (CoaxJob *)scratch.get("coax_jobs", sizeof(CoaxJob) * jobs.size());
    h2d_now(djobs, jobs.data(), sizeof(CoaxJob) * jobs.size(), st);
    for (size_t s = 0; s < jobs.size(); s += per) {
        int cnt = (int)std::min<int64_t>(per, jobs.size() - s);
        double2 *ws = (double2 *)scratch.get("coax_ws", sizeof(double2) * wsz * cnt);
        k_coax_prepare<<<cnt, 256, 0, st>>>(djobs + s, ws, wsz);
        LAUNCH_OK();
        k_coax_fill<<<dim3(pmax, cnt), 256, 0, st>>>(djobs + s, ws, wsz);
        LAUNCH_OK();
    }
}

// ------------------------------------------------------------------ rotation (Delta) tables
// one thread per (n, row m): G row by the downward m' recurrence, then Delta = eps G eps;
// writes Delta (rows m, cols m') and its transpose.
__global__ void k_delta(int p, double *D, double *DT) {
    int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    // map gid -> (n, m): rows of degree n are 2n+1; prefix n^2
    int n = (int)floor(sqrt((double)gid));
    while ((int64_t)n * n > gid) --n;
    while ((int64_t)(n + 1) * (n + 1) <= gid) ++n;
    if (n >= p) return;
    int m = (int)(gid - (int64_t)n * n) - n;
    double *row = D + rot_block_off(n) + (int64_t)(m + n) * (2 * n + 1);
    // edge value e_|m| = sqrt(C(2n, n+|m|)) 2^-n
    double e0 = 1.0;
    for (int q = 1; q <= n; ++q) e0 *= (2.0 * q - 1.0) / (2.0 * q);
    double e = sqrt(e0);
    int am = m < 0 ? -m : m;
    for (int q = 0; q < am; ++q) e *= sqrt((double)(n - q) / (double)(n + q + 1));
    // G_{m, m'} for m' = n..0, stored into row[m' + n]
    row[2 * n] = e;
    double up = 0.0, cur = e;
    for (int mp = n; mp >= 1; --mp) {
        double nxt = -(2.0 * m * cur + sqrt((double)(n - mp) * (double)(n + mp + 1)) * up) /
                     sqrt((double)(n + mp) * (double)(n - mp + 1));
        row[mp - 1 + n] = nxt;
        up = cur;
        cur = nxt;
    }
    const double sym = ((n + m) & 1) ? -1.0 : 1.0;
    for (int mp = 1; mp <= n; ++mp) row[-mp + n] = sym * row[mp + n];
    // eps factors
    const double em = (m < 0 && (m & 1)) ? -1.0 : 1.0;
    for (int mp = -n; mp <= n; ++mp) {
        double emp = (mp < 0 && (mp & 1)) ? -1.0 : 1.0;
        double v = row[mp + n] * em * emp;
        row[mp + n] = v;
        DT[rot_block_off(n) + (int64_t)(mp + n) * (2 * n + 1) + (m + n)] = v;
    }
}

// Rotation matrices for polar angle b from the quarter-turn matrices (Fourier-series form of the
// Wigner matrices): H_n(b)[m'][m] = sum_k Delta_{m'k} Delta_{mk} cos(k b + (m'-m) pi/2), which is
// the real matrix i^{m'-m} sum_k Delta_{m'k} Delta_{mk} e^{i k b}.  One thread per (b, n, m'),
// writing row m' of H and column m' of H^T.
__global__ void k_rot_tables(int nb, const double *betas, int P, const double *D, double *H, double *HT) {
    int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t per = (int64_t)P * P;  // rows over all degrees < P
    if (gid >= per * nb) return;
    const int ib = (int)(gid / per);
    const int64_t r = gid - (int64_t)ib * per;
    int n = (int)floor(sqrt((double)r));
    while ((int64_t)n * n > r) --n;
    while ((int64_t)(n + 1) * (n + 1) <= r) ++n;
    const int w = 2 * n + 1;
    const int mpi = (int)(r - (int64_t)n * n);  // row index m' + n
    const double b = betas[ib];
    const double *Dn = D + rot_block_off(n);
    double *Hn = H + (int64_t)ib * rot_table_size(P) + rot_block_off(n);
    double *HTn = HT + (int64_t)ib * rot_table_size(P) + rot_block_off(n);
    double sb, cb, s0, c0;
    sincos(b, &sb, &cb);
    sincos(-n * b, &s0, &c0);
    for (int mi = 0; mi < w; ++mi) {
        const int d = (((mpi - mi) % 4) + 4) % 4;
        double s = 0.0, cs = c0, sn = s0;  // e^{i k b}, advanced by angle addition
        for (int ki = 0; ki < w; ++ki) {
            const double f = d == 0 ? cs : d == 1 ? -sn : d == 2 ? -cs : sn;
            s = fma(Dn[(int64_t)mpi * w + ki] * Dn[(int64_t)mi * w + ki], f, s);
            const double nc = cs * cb - sn * sb;
            sn = cs * sb + sn * cb;
            cs = nc;
        }
        Hn[(int64_t)mpi * w + mi] = s;
        HTn[(int64_t)mi * w + mpi] = s;
    }
}

void build_rot_tables(const std::vector<double> &betas, int P, const double *D, double *H, double *HT,
                      DeviceBuffers &scratch, hipStream_t st) {
    if (betas.empty()) return;
    double *db = (double *)scratch.get("rot_betas", sizeof(double) * betas.size());
    HIP_OK(hipMemcpyAsync(db, betas.data(), sizeof(double) * betas.size(), hipMemcpyHostToDevice, st));
    const int64_t nthr = (int64_t)P * P * betas.size();
    k_rot_tables<<<ceil_div(nthr, 128), 128, 0, st>>>((int)betas.size(), db, P, D, H, HT);
    LAUNCH_OK();
    HIP_OK(hipStreamSynchronize(st));  // betas buffer reuse
}

void build_delta_table(int p, double *D, double *DT, hipStream_t st) {
    int64_t nthreads = (int64_t)p * p;
    k_delta<<<ceil_div(nthreads, 128), 128, 0, st>>>(p, D, DT);
    LAUNCH_OK();
}

}  // namespace fmm
