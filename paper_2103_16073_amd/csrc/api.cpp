// C ABI of the fmmbem library: context, setup orchestration, the FMM matrix-vector product
// driver, right-hand side, flexible GMRES solve and field evaluation.
#include <chrono>
#include <cmath>
#include <cstring>
#include <functional>
#include <numeric>

#include "internal.h"

#include <atomic>
#include <mutex>
#include <set>
#include <thread>

namespace fmm {
// kernels (fmm.hip / solver.hip)
__global__ void k_near_count(int64_t, const int32_t *, const int32_t *, const int32_t *, const int32_t *,
                             const double4 *, double, int32_t *);
__global__ void k_near_fill(int64_t, const int32_t *, const int32_t *, const int32_t *, const int32_t *,
                            const double4 *, double, const int32_t *, int32_t *, int32_t *);
__global__ void k_near_quad(int64_t, const int32_t *, const int32_t *, const double4 *, const double *, double,
                            double2 *, double2 *);
__global__ void k_densities(int64_t, int, const int32_t *, const double2 *, const double2 *, double, double2 *,
                            double2 *);
__global__ void k_gamma(int64_t, const double4 *, const double4 *, const double2 *, double, double, double, double,
                        double2, double2 *, double2 *);
__global__ void k_zero8(int64_t, uint64_t *);
__global__ void k_near_quad_n(int64_t, const int32_t *, const int32_t *, const double4 *, const double4 *,
                              const double *, double, double2 *, double2 *);
__global__ void k_gamma_pm(int64_t, const double4 *, const double4 *, const double2 *, const double2 *, double, double,
                           double, double, double2, double2 *, double2 *);
__global__ void k_densities_ind(int64_t, const int32_t *, const double2 *, const double2 *, const double2 *, double,
                                double2 *, double2 *);
__global__ void k_field_dens_ind(int64_t, const int32_t *, const double2 *, const double2 *, const double2 *,
                                 const double2 *, const double2 *, double, double2 *, double2 *);
__global__ void k_field_dens(int64_t, int, const int32_t *, const double2 *, const double4 *, const double4 *,
                             const double2 *, const double2 *, double, double, double, double, double2, double2 *,
                             double2 *);
__global__ void k_rhs_ind_local(int64_t, const int32_t *, const double2 *, const double2 *, double2 *);
__global__ void k_bm_combine(int64_t, const int32_t *, const double2 *, const double2 *, double, double2,
                             const double2 *, double2 *);
__global__ void k_bm_rhs(int64_t, const int32_t *, const double2 *, double2, const double2 *, double2 *);
__global__ void k_densities_dpsi(int64_t, const int32_t *, const double2 *, const double2 *, double, double2 *,
                                 double2 *);
__global__ void k_dpsi_combine(int64_t, const int32_t *, const double2 *, const double2 *, const double2 *, double2 *);
__global__ void k_rhs_dpsi_dens(int64_t, const int32_t *, const double2 *, double2 *, double2 *, double2 *);
__global__ void k_scale_beta(int64_t, const int32_t *, const double2 *, int, const double2 *, double2 *);
__global__ void k_diag_bm_inv(int64_t, const int32_t *, const int32_t *, const int32_t *, const double2 *,
                              const double2 *, const double2 *, const double2 *, const double2 *, double, double2,
                              double, double2 *);
__global__ void k_p2p_n(int, const int32_t *, const int32_t *, const int32_t *, int, const double4 *, const double4 *,
                        const double2 *, const double2 *, double, double, const int32_t *, const int32_t *,
                        const double2 *, const double2 *, const double2 *, const double2 *, double2 *, double2 *);
__global__ void k_local_derivs(int64_t, int, const double2 *, double, double2 *, double2 *, double2 *);
__global__ void k_l2p_n(int, int, const int32_t *, const double4 *, const double4 *, const double4 *, const double2 *,
                        const double2 *, const double2 *, const double2 *, double, const double *, const double2 *,
                        const double2 *, const int32_t *, int64_t, const double2 *, const double2 *, const double2 *,
                        double2 *, int);
__global__ void k_diag2_inv(int64_t, const int32_t *, const int32_t *, const double2 *, const double2 *,
                            const double2 *, const double2 *, double, double, double2 *);
__global__ void k_mul_diag2(int64_t, const int32_t *, const double2 *, const double2 *, double2 *);
void launch_p2p(int nr, bool fp32, int nleaf, const int32_t *leaf_start, const int32_t *nbr_start,
                const int32_t *nbr_list, int all_leaves, const double4 *ec, const double4 *en, const double2 *sigma,
                const double2 *mu, double k, double rc2, const int32_t *near_start, const int32_t *near_col,
                const void *nL, const void *nM, double2 *y, hipStream_t st);
bool p2m_fits(int nr, int p);
void launch_p2m(int nr, int nleaf, int p, const int32_t *leaf_start, const double4 *center, const double4 *ec,
                const double4 *en, const double2 *sigma, const double2 *mu, double k, const double *leg,
                double2 *Mout, hipStream_t st);
void launch_l2p(int nr, int nleaf, int p, const int32_t *leaf_start, const double4 *center, const double4 *ec,
                const double2 *Lc, double k, const double *leg, const double2 *ynear, double half,
                const int32_t *perm, int64_t n, const double2 *x, double2 *y, int has_far, hipStream_t st);
__global__ void k_cvt_d2f(int64_t, const double2 *, float2 *);
__global__ void k_cvt_f2d(int64_t, const float2 *, double2 *);
__global__ void k_cvt_real_d2f(int64_t, const double *, float *);
__global__ void k_field(int64_t, const double *, const double4 *, const double4 *, const double *, const double2 *,
                        const double2 *, double, double, double, double, double, double2, double2 *);
__global__ void k_field_tile(int64_t, int64_t, const double *, const double4 *, const double4 *, const double *,
                             const double2 *, const double2 *, double, double, double, double, double, double2,
                             double2 *);
__global__ void k_diag_inv(int64_t, const int32_t *, const int32_t *, const int32_t *, const double2 *,
                           const double2 *, const double2 *, double, double, double2 *);
__global__ void k_mul_diag(int64_t, const double2 *, const double2 *, double2 *);
__global__ void k_leaf_blocks(int, const int32_t *, const int64_t *, const double4 *, const double4 *,
                              const double2 *, double, double, const int32_t *, const int32_t *, const double2 *,
                              const double2 *, double2 *);
__global__ void k_leaf_blocks_ind(int, const int32_t *, const int64_t *, const double4 *, const double4 *,
                                  const double2 *, const double2 *, double, double, const int32_t *, const int32_t *,
                                  const double2 *, const double2 *, const double2 *, const double2 *, double2 *);
__global__ void k_leaf_blocks_bm(int, const int32_t *, const int64_t *, const double4 *, const double4 *,
                                 const double2 *, double, double2, double, const int32_t *, const int32_t *,
                                 const double2 *, const double2 *, const double2 *, const double2 *, double2 *);
__global__ void k_leaf_invert(int, const int32_t *, const int64_t *, double2 *, int32_t *, int *, int);
__global__ void k_leaf_apply(int, const int32_t *, const int64_t *, const double2 *, const int32_t *,
                             const double2 *, double2 *, int, int64_t);
void box_center(const TreeHost &T, int l, uint64_t code, double *c);
int fgmres_batch(int64_t n, hipStream_t st, DeviceBuffers &scr, int nv,
                 const std::function<void(int, const double2 *, double2 *)> &matvec,
                 const std::function<void(int, const double2 *, double2 *)> &matvec_check,
                 const std::function<void(const double2 *, double2 *)> &precond, const double2 *B, double2 *X,
                 double tol, int m, int maxit, bool x0_given, std::vector<int> &iters, std::vector<int> &restarts,
                 std::vector<double> &rel_res, std::vector<int> &status, bool basis32 = false, int reorth = 1);
int fgmres(int64_t n, hipStream_t st, DeviceBuffers &scr, const char *tag,
           const std::function<void(const double2 *, double2 *)> &matvec,
           const std::function<void(const double2 *, double2 *)> &matvec_check,
           const std::function<void(const double2 *, double2 *)> &precond, const double2 *b, double2 *x, double tol,
           int m, int maxit, bool x0_given, bool final_residual, std::vector<double> *history, int &iters,
           int &restarts, double &rel_res, const FgmresHooks *hooks, bool basis32 = false, int reorth = 1);

void drop_graphs(fmmbem_ctx *c);
static void autotune_batches(fmmbem_ctx *c);
static void record_shapes(fmmbem_ctx *c);

// ------------------------------------------------------------------ setup pieces
static int level_p(const fmmbem_options &o, double k, double side) {
    double kd = k * side;
    double p = kd + o.p_excess * std::cbrt(kd);
    return std::max(o.p_min, (int)std::ceil(p));
}

template <class T>
static T *upload(DeviceBuffers &b, const std::string &name, const std::vector<T> &v, hipStream_t st) {
    T *d = dget<T>(b, name, std::max<size_t>(v.size(), 1));
    h2d_now(d, v.data(), sizeof(T) * v.size(), st);  // v is usually a temporary of the caller
    return d;
}

// Legendre recurrence table (built with the rotation tables, degrees up to the largest p + 1)
static const double *leg_table(fmmbem_ctx *c) { return (const double *)c->buf.find("legtab"); }

// P2M stages a chunk of sources and the leaf's basis in LDS
static void check_p2m(int nr, int p) {
    if (!p2m_fits(nr, p)) throw FmmError(FMMBEM_EINVAL, "leaf truncation number too large for P2M staging");
}

static void setup_mesh(fmmbem_ctx *c) {
    const int64_t n = c->nt;
    c->batch_p.clear();  // a new octree: every level's batches are rebuilt
    std::vector<double> cen(3 * n), nrm(3 * n), area(n);
    double vlo[3] = {1e300, 1e300, 1e300}, vhi[3] = {-1e300, -1e300, -1e300};
    for (int64_t v = 0; v < c->nv; ++v)
        for (int d = 0; d < 3; ++d) {
            vlo[d] = std::min(vlo[d], c->xyz[3 * v + d]);
            vhi[d] = std::max(vhi[d], c->xyz[3 * v + d]);
        }
    // mean area by a compensated (Neumaier) sum: correct to about an ulp at any N, so the cutoff
    // does not depend on the order of the triangles
    double asum = 0.0, acomp = 0.0;
    for (int64_t j = 0; j < n; ++j) {
        const double *a = &c->xyz[3 * c->tri[3 * j]], *b = &c->xyz[3 * c->tri[3 * j + 1]], *e = &c->xyz[3 * c->tri[3 * j + 2]];
        double u[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]}, v[3] = {e[0] - a[0], e[1] - a[1], e[2] - a[2]};
        double w[3] = {u[1] * v[2] - u[2] * v[1], u[2] * v[0] - u[0] * v[2], u[0] * v[1] - u[1] * v[0]};
        double l = std::sqrt(w[0] * w[0] + w[1] * w[1] + w[2] * w[2]);
        for (int d = 0; d < 3; ++d) {
            cen[3 * j + d] = (a[d] + b[d] + e[d]) / 3.0;
            nrm[3 * j + d] = w[d] / l;
        }
        area[j] = 0.5 * l;
        const double t = asum + area[j];
        acomp += std::fabs(asum) >= area[j] ? (asum - t) + area[j] : (area[j] - t) + asum;
        asum = t;
    }
    asum += acomp;
    c->rc = c->opt.rc > 0 ? c->opt.rc : c->opt.rc_factor * std::sqrt(2.0 * asum / (double)n);
    TreeHost &T = c->tree;
    c->tree_min_leaf = c->opt.kd_leaf_min > 0 ? c->opt.kd_leaf_min / c->k : 0.0;
    build_tree(cen.data(), n, vlo, vhi, c->rc, c->opt.leaf_max, c->opt.max_depth, c->tree_min_leaf, T);
    const int L = T.depth;
    hipStream_t st = c->stream;
    // sorted element arrays
    std::vector<double4> ec(n), en(n);
    std::vector<double> ev(9 * n);
    std::vector<int32_t> leaf_of(n);
    for (int64_t i = 0; i < n; ++i) {
        int64_t j = T.perm[i];
        ec[i] = make_double4(cen[3 * j], cen[3 * j + 1], cen[3 * j + 2], area[j]);
        en[i] = make_double4(nrm[3 * j], nrm[3 * j + 1], nrm[3 * j + 2], 0.0);
        for (int q = 0; q < 3; ++q)
            for (int d = 0; d < 3; ++d) ev[9 * i + 3 * q + d] = c->xyz[3 * c->tri[3 * j + q] + d];
    }
    const int64_t nleaf = (int64_t)T.leaf_start.size() - 1;
    for (int64_t b = 0; b < nleaf; ++b)
        for (int32_t i = T.leaf_start[b]; i < T.leaf_start[b + 1]; ++i) leaf_of[i] = (int32_t)b;
    upload(c->buf, "ec", ec, st);
    upload(c->buf, "en", en, st);
    upload(c->buf, "ev", ev, st);
    upload(c->buf, "perm", T.perm, st);
    upload(c->buf, "leaf_of", leaf_of, st);
    upload(c->buf, "leaf_start", T.leaf_start, st);
    upload(c->buf, "nbr_start", T.nbr_start, st);
    upload(c->buf, "nbr_list", T.nbr_list, st);
    // P2P pairs (one-point rule candidates) for reporting
    int64_t pairs = 0;
    for (int64_t b = 0; b < nleaf; ++b) {
        int64_t nt_ = T.leaf_start[b + 1] - T.leaf_start[b], ns = 0;
        for (int q = T.nbr_start[b]; q < T.nbr_start[b + 1]; ++q)
            ns += T.leaf_start[T.nbr_list[q] + 1] - T.leaf_start[T.nbr_list[q]];
        pairs += nt_ * ns;
    }
    c->p2p_pairs = pairs;
    // levels: centres, parents, M2L lists, child ranges
    c->lev.assign(L + 1, LevelDev());
    c->iota_h.assign(L + 1, std::vector<int32_t>());
    for (int l = 0; l <= L; ++l) {
        LevelHost &H = T.lv[l];
        LevelDev &D = c->lev[l];
        D.nbox = (int64_t)H.code.size();
        D.side = H.side;
        std::vector<double4> cc(D.nbox);
        for (int64_t b = 0; b < D.nbox; ++b) {
            double x[3];
            box_center(T, l, H.code[b], x);
            cc[b] = make_double4(x[0], x[1], x[2], 0.0);
        }
        std::string s = "L" + std::to_string(l) + "_";
        D.center = upload(c->buf, s + "center", cc, st);
        if (l >= 1) {
            D.parent = upload(c->buf, s + "parent", H.parent, st);
            D.octant = upload(c->buf, s + "octant", H.octant, st);
            // M2M / L2L directions per child
            std::vector<int16_t> up(D.nbox), dn(D.nbox);
            for (int64_t b = 0; b < D.nbox; ++b) {
                up[b] = (int16_t)(343 + H.octant[b]);
                dn[b] = (int16_t)(351 + H.octant[b]);
            }
            upload(c->buf, s + "dir_up", up, st);
            upload(c->buf, s + "dir_dn", dn, st);
            std::vector<int32_t> iota_(D.nbox + 1);
            std::iota(iota_.begin(), iota_.end(), 0);
            upload(c->buf, s + "iota", iota_, st);
            c->iota_h[l] = iota_;
        }
        if (l < L) D.child_start = upload(c->buf, s + "child_start", H.child_start, st);
        if (l >= 2) {
            D.njob_m2l = (int64_t)H.m2l_src.size();
            D.m2l_start = upload(c->buf, s + "m2l_start", H.m2l_start, st);
            D.m2l_src = upload(c->buf, s + "m2l_src", H.m2l_src, st);
            D.m2l_dir = upload(c->buf, s + "m2l_dir", H.m2l_dir, st);
            std::vector<int8_t> tau(H.m2l_dir.size());
            for (size_t q = 0; q < tau.size(); ++q) tau[q] = (int8_t)H.m2l_tau_of_dir[H.m2l_dir[q]];
            D.m2l_tau = upload(c->buf, s + "m2l_tau", tau, st);
            D.ntau = (int)H.m2l_taus.size();
        }
    }
    HIP_OK(hipStreamSynchronize(st));
}

static void direction_vector(int d, double *t) {
    if (d < 343) {
        t[0] = d / 49 - 3;
        t[1] = (d / 7) % 7 - 3;
        t[2] = d % 7 - 3;
    } else {
        int o = (d - 343) % 8;
        double sgn = d < 351 ? -1.0 : 1.0;  // M2M: parent - child; L2L: child - parent
        t[0] = sgn * ((o & 1) ? 1.0 : -1.0);
        t[1] = sgn * ((o & 2) ? 1.0 : -1.0);
        t[2] = sgn * ((o & 4) ? 1.0 : -1.0);
    }
}

static double direction_cos_beta(int d) {
    double t[3];
    direction_vector(d, t);
    return t[2] / std::sqrt(t[0] * t[0] + t[1] * t[1] + t[2] * t[2]);
}

// e^{i m alpha} per direction (alpha = azimuth of t), m = -PH..PH
static void direction_phases(int PH, std::vector<double2> &A) {
    A.assign((size_t)NDIR * (2 * PH + 1), cmk(0, 0));
    for (int d = 0; d < NDIR; ++d) {
        double t[3];
        direction_vector(d, t);
        double tn = std::sqrt(t[0] * t[0] + t[1] * t[1] + t[2] * t[2]);
        if (tn == 0) continue;
        double alpha = (t[0] == 0 && t[1] == 0) ? 0.0 : std::atan2(t[1], t[0]);
        for (int m = -PH; m <= PH; ++m)
            A[(size_t)d * (2 * PH + 1) + m + PH] = cmk(std::cos(m * alpha), std::sin(m * alpha));
    }
}


// the fused translation kernel takes lane batches with p_src = p_tgt = p (coaxial tables of that
// p) up to the p whose 32-job vectors fit the LDS
static bool fused_ok(const TransBatch &b) {
    return b.psrc == b.ptgt && b.PT == b.P && b.P <= trans_fused_pmax();
}
// the p = 16 fused tiles (mode 3: FP64 products of one vector in registers, other products of such
// a batch in LDS; mode 4: every product, the vectors in LDS)
static bool rcr_ok(const TransBatch &b) { return fused_ok(b) && b.P == trans_rcr_p(); }

// Tile layout of a sorted job list for the batch's shape (JT, whole, lane): classes padded to
// whole tiles, per-tile table indices, per-target CSR of the (padded) job order.
static void layout_batch(fmmbem_ctx *c, const std::string &name, const std::vector<JobH> &jobs, TransBatch &b) {
    hipStream_t st = c->stream;
    const int64_t ntgt = b.ntgt;
    std::vector<int32_t> s, t, tc, tr;
    std::vector<int16_t> d;
    size_t q = 0;
    while (q < jobs.size()) {
        size_t e = q;
        while (e < jobs.size() && jobs[e].tab == jobs[q].tab && jobs[e].rot == jobs[q].rot) ++e;
        for (size_t r = q; r < e; ++r) {
            s.push_back(jobs[r].src);
            t.push_back(jobs[r].tgt);
            d.push_back(jobs[r].dir);
        }
        while (s.size() % b.JT) {  // pad the class to whole tiles
            s.push_back(jobs[q].src);
            t.push_back(-1);
            d.push_back(jobs[q].dir);
        }
        const size_t tiles = (e - q + b.JT - 1) / b.JT;
        for (size_t k = 0; k < tiles; ++k) {
            tc.push_back(jobs[q].tab);
            tr.push_back(jobs[q].rot);
        }
        q = e;
    }
    b.njob = (int64_t)s.size();
    // lane batches: runs of one target within SEG_ALIGN-job blocks (jobs of a class are sorted
    // by target); the back rotation sums each run into its first job's row
    std::vector<int8_t> seg;
    if (b.lane) {
        seg.assign(t.size(), 0);
        for (size_t q2 = 0; q2 < t.size();) {
            size_t e = q2 + 1;
            if (t[q2] >= 0)
                while (e < t.size() && e % SEG_ALIGN != 0 && t[e] == t[q2]) ++e;
            if (t[q2] >= 0) seg[q2] = (int8_t)(e - q2);
            q2 = e;
        }
        b.seg = upload(c->buf, name + "_seg", seg, st);
        b.nout = 0;
        for (int8_t v : seg) b.nout += v > 0;
    } else {
        b.seg = nullptr;
        b.nout = (int64_t)jobs.size();
    }
    // rows of every target (CSR over the padded order): every job, or the first job of each run
    {
        std::vector<int32_t> ts(ntgt + 1, 0), tj;
        auto listed = [&](size_t q2) { return t[q2] >= 0 && (!b.lane || seg[q2] > 0); };
        for (size_t q2 = 0; q2 < t.size(); ++q2)
            if (listed(q2)) ts[t[q2] + 1]++;
        for (int64_t q2 = 0; q2 < ntgt; ++q2) ts[q2 + 1] += ts[q2];
        tj.resize(ts[ntgt]);
        std::vector<int32_t> fill(ts.begin(), ts.end() - 1);
        for (size_t q2 = 0; q2 < t.size(); ++q2)
            if (listed(q2)) tj[fill[t[q2]]++] = (int32_t)q2;
        b.tgt_start = upload(c->buf, name + "_tstart", ts, st);
        b.tgt_jobs = upload(c->buf, name + "_tjobs", tj, st);
    }
    b.src = upload(c->buf, name + "_src", s, st);
    b.tgt = upload(c->buf, name + "_tgt", t, st);
    b.dir = upload(c->buf, name + "_dir", d, st);
    b.tile_coax = upload(c->buf, name + "_tcoax", tc, st);
    b.tile_rot = upload(c->buf, name + "_trot", tr, st);
}

// Sort jobs by (coaxial table, polar angle, target), pad every class to whole tiles, build the
// rotation tables of the batch's distinct polar angles.
static void make_batch(fmmbem_ctx *c, const std::string &name, std::vector<JobH> jobs, int psrc, int ptgt, int PT,
                       int64_t ntgt, TransBatch &b) {
    hipStream_t st = c->stream;
    b = TransBatch();
    b.psrc = psrc;
    b.ptgt = ptgt;
    b.PT = PT;
    b.P = std::max(psrc, ptgt);
    b.nreal = (int64_t)jobs.size();
    {
        std::vector<int32_t> srcs;
        srcs.reserve(jobs.size());
        for (auto &j : jobs) srcs.push_back(j.src);
        std::sort(srcs.begin(), srcs.end());
        b.nsrc = std::unique(srcs.begin(), srcs.end()) - srcs.begin();
        int tmax = 0;
        for (auto &j : jobs) tmax = std::max(tmax, j.tab);
        b.ncoax = tmax + 1;
    }
    size_t budget = c->opt.lds_budget > 0 ? (size_t)c->opt.lds_budget : (size_t)32768;
    budget = std::min(budget, c->lds_max - 1024);
    b.ntgt = ntgt;
    // polar-angle classes
    std::vector<double> cb;
    for (auto &j : jobs) cb.push_back(direction_cos_beta(j.dir));
    std::vector<double> uniq = cb;
    std::sort(uniq.begin(), uniq.end());
    std::vector<double> classes;
    for (double v : uniq)
        if (classes.empty() || v - classes.back() > 1e-12) classes.push_back(v);
    for (size_t q = 0; q < jobs.size(); ++q)
        jobs[q].rot = (int)(std::lower_bound(classes.begin(), classes.end(), cb[q] - 1e-12) - classes.begin());
    std::stable_sort(jobs.begin(), jobs.end(), [](const JobH &x, const JobH &y) {
        if (x.tab != y.tab) return x.tab < y.tab;
        if (x.rot != y.rot) return x.rot < y.rot;
        return x.tgt < y.tgt;
    });
    // Tile shape: one job per lane (64-job tiles) when the classes are large enough that padding
    // them to 64 wastes at most a quarter of the work, or, for matrix-core tiles (p >= 24, several
    // times faster than the LDS tiles there), at most half of it (32-job tiles where the 64-job
    // padding would exceed a third); otherwise whole-vector tiles while at least 8 jobs fit the
    // LDS budget, per-degree slices beyond.
    int64_t pad64 = 0, pad32 = 0;
    for (size_t q = 0; q < jobs.size();) {
        size_t e = q;
        while (e < jobs.size() && jobs[e].tab == jobs[q].tab && jobs[e].rot == jobs[q].rot) ++e;
        pad64 += (int64_t)((e - q + 63) / 64) * 64;
        pad32 += (int64_t)((e - q + 31) / 32) * 32;
        q = e;
    }
    const int64_t nj = (int64_t)jobs.size();
    const bool mf = c->opt.mfma == 2 || (c->opt.mfma == 1 && b.P >= 24);
    b.lane = !jobs.empty() && (c->opt.lane_tiles == 2 ||
                               (c->opt.lane_tiles == 1 && (pad64 * 4 <= nj * 5 || (mf && pad32 <= 2 * nj))));
    if (b.lane) {
        b.whole = 0;
        b.JT = 64;
        b.mfma = mf;
        if (mf && pad64 * 2 > nj * 3) b.JT = 32;
        if (c->opt.fused && fused_ok(b)) {
            b.JT = 64;
            b.mfma = rcr_ok(b) ? 4 : 2;
        }
    } else {
        b.whole = trans_pick_jt(b.P, budget, 1) >= 8 && (size_t)8 * 16 * b.P * b.P <= budget;
        b.JT = trans_pick_jt(b.P, budget, b.whole);
    }
    c->batch_jobs[name] = jobs;  // kept for re-layout by the autotuner
    layout_batch(c, name, jobs, b);
    b.nbeta = (int)classes.size();
    std::vector<double> betas;
    for (double v : classes) betas.push_back(std::acos(std::max(-1.0, std::min(1.0, v))));
    b.H = dget<double>(c->buf, name + "_H", std::max<size_t>(1, betas.size()) * rot_table_size(b.P) + TABLE_PAD);
    b.HT = dget<double>(c->buf, name + "_HT", std::max<size_t>(1, betas.size()) * rot_table_size(b.P) + TABLE_PAD);
    {
        const size_t nt_ = std::max<size_t>(1, betas.size()) * rot_table_size(b.P);
        HIP_OK(hipMemsetAsync(b.H + nt_, 0, sizeof(double) * TABLE_PAD, st));
        HIP_OK(hipMemsetAsync(b.HT + nt_, 0, sizeof(double) * TABLE_PAD, st));
    }
    build_rot_tables(betas, b.P, (double *)c->buf.find("delta"), b.H, b.HT, c->scratch, st);
}

// the batch's tables in the fused tiles' fragment order (coax: its ncoax coaxial tables)
static void fused_tables(fmmbem_ctx *c, const std::string &name, TransBatch &b, const double2 *coax, int ncoax) {
    if (b.njob == 0 || !fused_ok(b)) return;
    const size_t nr = (size_t)std::max(1, b.nbeta) * TF_FR_ROT, nc = (size_t)std::max(1, ncoax) * TF_FR_COAX;
    b.frH = dget<double>(c->buf, name + "_frH", nr);
    b.frHT = dget<double>(c->buf, name + "_frHT", nr);
    b.frC = dget<double>(c->buf, name + "_frC", nc);
    b.nfrc = std::max(1, ncoax);
    build_fused_tables(b.P, b.PT, b.nbeta, b.H, b.HT, ncoax, coax, b.frH, b.frHT, b.frC, c->stream);
}

// Batches of every level.  A level whose octree and truncation numbers (its own and the next
// level's) are those its batches were built with keeps them -- job order, tiles, rotation tables
// and tile shapes do not depend on k -- and only the fused tiles' coaxial fragments follow the new
// coaxial tables (a frequency sweep on one mesh rebuilds only the levels whose p moved).
static void build_batches(fmmbem_ctx *c) {
    TreeHost &T = c->tree;
    const int L = T.depth;
    for (int l = 2; l <= L; ++l) {
        LevelHost &H = T.lv[l];
        LevelDev &D = c->lev[l];
        std::string s = "L" + std::to_string(l) + "_";
        const std::pair<int, int> key(D.p, l < L ? c->lev[l + 1].p : -1);
        auto kept = c->batch_p.find(l);
        if (kept != c->batch_p.end() && kept->second == key) {
            fused_tables(c, s + "m2l", D.m2l, D.coax_m2l, D.ntau);
            if (l < L) {
                fused_tables(c, s + "up", D.up, D.coax_up, 1);
                fused_tables(c, s + "down", D.down, D.coax_up, 1);
            }
            continue;
        }
        c->batch_p.erase(l);
        std::vector<JobH> jobs;
        for (int64_t b = 0; b < D.nbox; ++b)
            for (int q = H.m2l_start[b]; q < H.m2l_start[b + 1]; ++q)
                jobs.push_back({H.m2l_src[q], (int32_t)b, H.m2l_dir[q], H.m2l_tau_of_dir[H.m2l_dir[q]], 0});
        make_batch(c, s + "m2l", jobs, D.p, D.p, D.p, D.nbox, D.m2l);
        fused_tables(c, s + "m2l", D.m2l, D.coax_m2l, D.ntau);
        if (l < L) {
            LevelHost &Hc = T.lv[l + 1];
            LevelDev &C = c->lev[l + 1];
            const int PT = std::max(D.p, C.p);
            std::vector<JobH> up, dn;
            for (int64_t ch = 0; ch < C.nbox; ++ch) {
                up.push_back({(int32_t)ch, Hc.parent[ch], (int16_t)(343 + Hc.octant[ch]), 0, 0});
                dn.push_back({Hc.parent[ch], (int32_t)ch, (int16_t)(351 + Hc.octant[ch]), 0, 0});
            }
            make_batch(c, s + "up", up, C.p, D.p, PT, D.nbox, D.up);
            make_batch(c, s + "down", dn, D.p, C.p, PT, C.nbox, D.down);
            fused_tables(c, s + "up", D.up, D.coax_up, 1);
            fused_tables(c, s + "down", D.down, D.coax_up, 1);
        }
        c->batch_p[l] = key;
    }
    HIP_OK(hipStreamSynchronize(c->stream));
}

static void setup_k(fmmbem_ctx *c) {
    TreeHost &T = c->tree;
    const int L = T.depth;
    hipStream_t st = c->stream;
    // truncation numbers
    c->pmax = 0;
    for (int l = 2; l <= L; ++l) {
        c->lev[l].p = level_p(c->opt, c->k, c->lev[l].side);
        T.lv[l].p = c->lev[l].p;
        c->pmax = std::max(c->pmax, c->lev[l].p);
    }
    if (c->pmax > 1000) throw FmmError(FMMBEM_EINVAL, "truncation number above 1000: octree too shallow for this k");
    // rotation tables (frequency independent; rebuilt only when p grows)
    if (c->pmax > c->delta_p) {
        double *D = dget<double>(c->buf, "delta", rot_table_size(c->pmax));
        double *DT = dget<double>(c->buf, "deltaT", rot_table_size(c->pmax));
        build_delta_table(c->pmax, D, DT, st);
        std::vector<double2> A;
        direction_phases(c->pmax, A);
        upload(c->buf, "phA", A, st);
        // recurrence table of the normalised Legendre functions, degrees up to pmax + 1
        const int pl = c->pmax + 1;
        std::vector<double> lt((size_t)leg_table_len(pl), 0.0);
        for (int n = 0; n <= pl; ++n)
            for (int m = 0; m <= n; ++m) {
                double *e = &lt[3 * (size_t)leg_tri(n, m)];
                if (n > m) e[0] = std::sqrt((4.0 * n * n - 1.0) / ((double)n * n - (double)m * m));
                if (n > m + 1)
                    e[1] = std::sqrt((((double)n - 1) * (n - 1) - (double)m * m) * (2.0 * n + 1.0) /
                                     ((2.0 * n - 3.0) * ((double)n * n - (double)m * m)));
                double g = 1.0 / std::sqrt(4.0 * FMM_PI);
                for (int q = 1; q <= m; ++q) g *= std::sqrt((2.0 * q + 1.0) / (2.0 * q));
                e[2] = g;
            }
        upload(c->buf, "legtab", lt, st);
        c->delta_p = c->pmax;
    }
    // coaxial tables
    std::vector<CoaxJob> jobs;
    for (int l = 2; l <= L; ++l) {
        LevelDev &D = c->lev[l];
        const int p = D.p;
        std::string s = "L" + std::to_string(l) + "_";
        D.coax_m2l = dget<double2>(c->buf, s + "coax_m2l", (size_t)coax_table_size(p) * std::max(D.ntau, 1) + TABLE_PAD);
        HIP_OK(hipMemsetAsync(D.coax_m2l + (size_t)coax_table_size(p) * std::max(D.ntau, 1), 0,
                              sizeof(double2) * TABLE_PAD, st));
        for (int q = 0; q < D.ntau; ++q) {
            double kt = c->k * T.lv[l].m2l_taus[q];
            jobs.push_back({0, kt < c->opt.ktau_switch ? 0 : 1, p, kt, D.coax_m2l + (size_t)q * coax_table_size(p)});
        }
        if (l < L) {
            const int PT = std::max(p, c->lev[l + 1].p);
            D.coax_up = dget<double2>(c->buf, s + "coax_up", coax_table_size(PT) + TABLE_PAD);
            HIP_OK(hipMemsetAsync(D.coax_up + coax_table_size(PT), 0, sizeof(double2) * TABLE_PAD, st));
            double kt = c->k * std::sqrt(3.0) * 0.5 * c->lev[l + 1].side;
            jobs.push_back({1, kt < c->opt.ktau_switch ? 0 : 1, PT, kt, D.coax_up});
        }
        D.M = dget<double2>(c->buf, s + "M", (size_t)D.nbox * p * p);
        D.L = dget<double2>(c->buf, s + "L", (size_t)D.nbox * p * p);
    }
    c->nr_cap = 1;
    c->nr_cap32 = 0;
    build_coax_tables(jobs, c->scratch, st);
    build_batches(c);
    // near-field table
    const int64_t n = c->nt;
    const int nleaf = (int)T.leaf_start.size() - 1;
    int32_t *cnt = dget<int32_t>(c->scratch, "near_cnt", n);
    const double rc2 = c->rc * c->rc;
    auto ec = (const double4 *)c->buf.find("ec");
    k_near_count<<<ceil_div(n, 128), 128, 0, st>>>(n, (int32_t *)c->buf.find("leaf_of"), (int32_t *)c->buf.find("leaf_start"),
                                                   (int32_t *)c->buf.find("nbr_start"), (int32_t *)c->buf.find("nbr_list"),
                                                   ec, rc2, cnt);
    LAUNCH_OK();
    std::vector<int32_t> hc(n), start(n + 1, 0);
    HIP_OK(hipMemcpyAsync(hc.data(), cnt, sizeof(int32_t) * n, hipMemcpyDeviceToHost, st));
    HIP_OK(hipStreamSynchronize(st));
    for (int64_t i = 0; i < n; ++i) start[i + 1] = start[i] + hc[i];
    c->near_nnz = start[n];
    int32_t *dstart = upload(c->buf, "near_start", start, st);
    int32_t *drow = dget<int32_t>(c->buf, "near_row", c->near_nnz);
    int32_t *dcol = dget<int32_t>(c->buf, "near_col", c->near_nnz);
    k_near_fill<<<ceil_div(n, 128), 128, 0, st>>>(n, (int32_t *)c->buf.find("leaf_of"), (int32_t *)c->buf.find("leaf_start"),
                                                  (int32_t *)c->buf.find("nbr_start"), (int32_t *)c->buf.find("nbr_list"),
                                                  ec, rc2, dstart, drow, dcol);
    LAUNCH_OK();
    double2 *nL = dget<double2>(c->buf, "near_L", c->near_nnz), *nM = dget<double2>(c->buf, "near_M", c->near_nnz);
    k_near_quad<<<ceil_div(c->near_nnz, 128), 128, 0, st>>>(c->near_nnz, drow, dcol, ec, (double *)c->buf.find("ev"),
                                                            c->k, nL, nM);
    LAUNCH_OK();
    (void)nleaf;
    HIP_OK(hipStreamSynchronize(st));
}

static void ensure_setup(fmmbem_ctx *c) {
    if (!c->have_mesh) throw FmmError(FMMBEM_ENOTREADY, "mesh not set");
    if (!c->have_k) throw FmmError(FMMBEM_ENOTREADY, "wavenumber not set");
    auto t0 = std::chrono::steady_clock::now();
    bool any = c->mesh_dirty || c->k_dirty || c->beta_dirty;
    if (any) {
        drop_graphs(c);
        c->chunks_ready = false;
    }
    if (c->mesh_dirty || c->k_dirty) c->indirect_ready = false;
    if (!c->mesh_dirty && c->k_dirty && c->opt.kd_leaf_min > 0) {
        // the leaf-size bound follows k: rebuild the octree when it would now allow a different depth
        const double nb = c->opt.kd_leaf_min / c->k, side = c->tree.side;
        auto cap = [&](double ml) {  // deepest level whose boxes are not smaller than ml
            int L = 2;
            while (L < 21 && side / (double)(1u << (L + 1)) >= ml) ++L;
            return L;
        };
        const int d = c->tree.depth, c_old = cap(c->tree_min_leaf), c_new = cap(nb);
        if (c_old != c_new && (d >= std::min(c_old, c_new))) c->mesh_dirty = true;
    }
    if (c->mesh_dirty) {
        setup_mesh(c);
        c->k_dirty = true;
        c->beta_dirty = true;
        c->mesh_dirty = false;
    }
    if (c->k_dirty) {
        c->mixed_ready = false;
        setup_k(c);
        if (c->opt.autotune) autotune_batches(c);
        else record_shapes(c);
        c->k_dirty = false;
        c->precond_ready_nb = c->precond_ready_diag = false;
    }
    if (c->beta_dirty) {
        if (!c->have_beta) c->beta.assign(c->nt, cmk(0, 0));
        std::vector<double2> bs(c->nt), bp(c->nt);
        for (int64_t i = 0; i < c->nt; ++i) {
            bs[i] = c->beta[c->tree.perm[i]];
            bp[i] = c->beta_plus.empty() ? bs[i] : c->beta_plus[c->tree.perm[i]];
        }
        upload(c->buf, "beta", bs, c->stream);
        upload(c->buf, "betap", bp, c->stream);
        HIP_OK(hipStreamSynchronize(c->stream));
        c->beta_dirty = false;
        c->precond_ready_nb = c->precond_ready_diag = false;
    }
    if (any) c->t_setup_last = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

// ------------------------------------------------------------------ kernel profiling
static void prof_flush(fmmbem_ctx *c) {
    if (c->prof_pend.empty()) return;
    // the pairs sit on either stream of the product (a flush may come mid-product)
    HIP_OK(hipStreamSynchronize(c->stream));
    HIP_OK(hipStreamSynchronize(c->side));
    for (auto &r : c->prof_pend) {
        float ms = 0;
        HIP_OK(hipEventElapsedTime(&ms, c->prof_ev[r.a], c->prof_ev[r.b]));
        auto &s = c->prof_stats[r.cls];
        s.launches += 1;
        s.ms += ms;
        s.flops += r.flops;
        s.bytes += r.bytes;
    }
    c->prof_pend.clear();
    c->prof_used = 0;
}
static int prof_begin(fmmbem_ctx *c) {
    if (!c->prof_on) return -1;
    if (c->prof_used + 2 > (int)c->prof_ev.size()) prof_flush(c);
    while ((int)c->prof_ev.size() < c->prof_used + 2) {
        hipEvent_t e;
        HIP_OK(hipEventCreate(&e));
        c->prof_ev.push_back(e);
    }
    int a = c->prof_used;
    c->prof_used += 2;
    HIP_OK(hipEventRecord(c->prof_ev[a], c->cur));
    return a;
}
static void prof_end(fmmbem_ctx *c, int a, const char *name, double flops, double bytes) {
    if (a < 0) return;
    HIP_OK(hipEventRecord(c->prof_ev[a + 1], c->cur));
    int cls = -1;
    for (size_t q = 0; q < c->prof_stats.size(); ++q)
        if (!strcmp(c->prof_stats[q].name, name)) cls = (int)q;
    if (cls < 0) {
        fmmbem_kstat s{};
        std::snprintf(s.name, sizeof(s.name), "%s", name);
        c->prof_stats.push_back(s);
        cls = (int)c->prof_stats.size() - 1;
    }
    c->prof_pend.push_back({cls, a, a + 1, flops, bytes});
}
static double rot_flops(int p) {  // one real (2n+1)^2 rotation per degree applied to a complex vector
    double s = 0;
    for (int n = 0; n < p; ++n) s += 4.0 * (2.0 * n + 1) * (2.0 * n + 1);
    return s;
}
static double coax_flops(int ps, int pt) {
    double s = 0;
    int pm = std::min(ps, pt);
    for (int m = -(pm - 1); m <= pm - 1; ++m) s += 8.0 * (pt - std::abs(m)) * (ps - std::abs(m));
    return s;
}

// ------------------------------------------------------------------ the FMM pass
// Staged translation of a batch of jobs (grouped by target) from `src` (psrc) into `dst` (ptgt).
// In FP32 the fused tiles beat the three lane passes at every batch that may use them (they are
// issue-bound there, not bound by the LDS-limited occupancy of FP64), so mixed products run such
// batches fused whatever the FP64 shape chosen for them, unless `fused` is off.
static void zero_dev(fmmbem_ctx *c, void *ptr, size_t bytes);

// accumulate: add into dst; otherwise the batch overwrites every target of dst (an empty batch
// clears it)
template <class R>
static void run_batch(fmmbem_ctx *c, int nrv, const TransBatch &b0, const typename Cx<R>::T *src,
                      typename Cx<R>::T *dst, const TransTables<R> &tb, const typename Cx<R>::T *ph,
                      bool accumulate = true) {
    using C = typename Cx<R>::T;
    if (b0.njob == 0) {
        if (!accumulate) zero_dev(c, dst, sizeof(C) * (size_t)b0.ntgt * nrv * b0.ptgt * b0.ptgt);
        return;
    }
    TransBatch b32;
    if (sizeof(R) == 4 && c->opt.fused && b0.lane && b0.mfma == 0 && fused_ok(b0) && tb.frH) {
        b32 = b0;
        b32.mfma = rcr_ok(b0) ? 4 : 2;  // p = 16: the FP32 register-resident shape (one vector)
    }
    const TransBatch &b = b32.njob ? b32 : b0;
    hipStream_t st = c->cur;
    // work rows per stream, so that batches on the two streams never share them
    const bool side = st == c->side;
    C *W1 = (C *)c->scratch.get(side ? "W1s" : "W1", sizeof(C) * (size_t)b.njob * nrv * b.P * b.P);
    // the fused kernels keep the intermediate rows on chip: no second work array
    const bool fused = b.lane && b.mfma >= 2;
    C *W2 = fused ? nullptr : (C *)c->scratch.get(side ? "W2s" : "W2", sizeof(C) * (size_t)b.njob * nrv * b.P * b.P);
    const double nr = (double)b.nreal * nrv, P2 = (double)b.P * b.P, cs = (double)sizeof(C);
    // Algorithmic work per stage, the method's own: flops of the matrices applied (rotation,
    // coaxial step, rotation; the reduction's additions) and compulsory HBM bytes -- every distinct
    // source expansion read once, the tables the stage applies read once, the target expansions
    // read and written once by the reduction.  The work rows between the stages and the run rows
    // into the reduction exist only because the method is split into kernels; the bench reports
    // them as the difference between the measured traffic and these bytes.
    const double rs = sizeof(R), nbeta = std::max(1, b.nbeta);
    const double rot_tab = nbeta * rot_table_size(b.P) * rs, coax_tab = b.ncoax * coax_table_size(b.PT) * 2 * rs;
    const double src_by = (double)b.nsrc * nrv * b.psrc * b.psrc * cs;
    const double fl[4] = {nr * rot_flops(b.psrc), nr * coax_flops(b.psrc, b.ptgt), nr * rot_flops(b.ptgt), nr * P2 * 2};
    const double by[4] = {src_by + rot_tab, coax_tab, rot_tab, 2.0 * b.ntgt * nrv * b.ptgt * b.ptgt * cs};
    for (int stage = 0; stage < 4; ++stage) {
        if (b.lane && b.mfma >= 2 && (stage == 1 || stage == 2)) continue;  // inside the fused kernel
        int e = prof_begin(c);
        const char *name = trans_stage<R>(b, tb, stage, nrv, src, dst, ph, c->delta_p, W1, W2, st, accumulate);
        double f = fl[stage], y = by[stage];
        if (b.lane && b.mfma >= 2 && stage == 0) {  // fused: all three stages, each table once
            f = fl[0] + fl[1] + fl[2];
            y = src_by + rot_tab + coax_tab;
        }
        prof_end(c, e, name, f, y);
    }
}

static TransTables<double> tables64(const TransBatch &b, const double2 *coax) {
    return {coax, b.H, b.HT, b.frH, b.frHT, b.frC};
}
static TransTables<float> tables32(const TransBatch &b, const float2 *coax) {
    return {coax, b.H32, b.HT32, b.frH32, b.frHT32, b.frC32};
}

// every batch of the product with its source/target expansions and coaxial tables
struct BatchRef {
    int level, kind;
    std::string name;
    TransBatch *b;
    const double2 *src, *coax;
    double2 *dst;
};
static std::vector<BatchRef> all_batches(fmmbem_ctx *c) {
    std::vector<BatchRef> v;
    const int L = c->tree.depth;
    for (int l = 2; l <= L; ++l) {
        LevelDev &D = c->lev[l];
        const std::string s = "L" + std::to_string(l) + "_";
        v.push_back({l, 0, s + "m2l", &D.m2l, D.M, D.coax_m2l, D.L});
        if (l < L) {
            LevelDev &C = c->lev[l + 1];
            v.push_back({l, 1, s + "up", &D.up, C.M, D.coax_up, D.M});
            v.push_back({l, 2, s + "down", &D.down, D.L, D.coax_up, C.L});
        }
    }
    return v;
}

static void record_shapes(fmmbem_ctx *c) {
    c->shapes.clear();
    for (auto &r : all_batches(c))
        c->shapes.push_back({r.level, r.kind, r.b->lane, r.b->whole, r.b->JT, r.b->mfma, r.b->nreal, 0.0});
}

// Tile-shape autotuner: for every batch, time its four stages (FP64, one vector) under each
// feasible shape -- one job per lane, whole-vector LDS tiles and per-degree LDS tiles with
// several tile sizes -- on the batch's own expansion arrays, and keep the fastest layout.
static void autotune_batches(fmmbem_ctx *c) {
    hipStream_t st = c->stream;
    const double2 *ph = (double2 *)c->buf.find("phA");
    hipEvent_t e0, e1;
    HIP_OK(hipEventCreate(&e0));
    HIP_OK(hipEventCreate(&e1));
    const size_t cap = c->lds_max - 1024;
    c->shapes.clear();
    for (auto &r : all_batches(c)) {
        TransBatch &b = *r.b;
        if (b.njob == 0) continue;
        const std::vector<JobH> &jobs = c->batch_jobs[r.name];
        struct Shape {
            int lane, whole, jt, mfma;
        };
        std::vector<Shape> cand;
        int64_t pad64 = 0, pad32 = 0;
        for (size_t q = 0; q < jobs.size();) {
            size_t e = q;
            while (e < jobs.size() && jobs[e].tab == jobs[q].tab && jobs[e].rot == jobs[q].rot) ++e;
            pad64 += (int64_t)((e - q + 63) / 64) * 64;
            pad32 += (int64_t)((e - q + 31) / 32) * 32;
            q = e;
        }
        if (pad64 <= 2 * (int64_t)jobs.size()) {
            cand.push_back({1, 0, 64, 0});
            if (c->opt.mfma != 0) cand.push_back({1, 0, 64, 1});
            if (c->opt.fused && fused_ok(b)) cand.push_back({1, 0, 64, 2});
            if (c->opt.fused && rcr_ok(b)) {
                cand.push_back({1, 0, 64, 3});
                cand.push_back({1, 0, 64, 4});
            }
        }
        // matrix-core tiles of 32 jobs where classes are small (less padding, less reuse per tile)
        if (c->opt.mfma != 0 && pad32 < pad64 && pad32 <= 2 * (int64_t)jobs.size()) cand.push_back({1, 0, 32, 1});
        for (int whole = 0; whole < 2; ++whole)
            for (int jt : {4, 8, 12, 16, 24, 32, 48, 64})
                if (trans_lds_bytes(jt, b.P, whole) <= cap && (whole == 0 || jt >= 4)) cand.push_back({0, whole, jt, 0});
        double best = 1e300;
        Shape bs = {b.lane, b.whole, b.JT, b.mfma};
        for (const Shape &sh : cand) {
            b.lane = sh.lane;
            b.whole = sh.whole;
            b.JT = sh.jt;
            b.mfma = sh.mfma;
            layout_batch(c, r.name, jobs, b);
            const TransTables<double> tb = tables64(b, r.coax);
            run_batch<double>(c, 1, b, r.src, r.dst, tb, ph);  // warm-up (allocates the work rows)
            // best of three repetitions: shapes within a few per cent of each other would
            // otherwise trade places from run to run
            float ms = 1e30f;
            for (int rep = 0; rep < 3; ++rep) {
                HIP_OK(hipEventRecord(e0, st));
                run_batch<double>(c, 1, b, r.src, r.dst, tb, ph);
                HIP_OK(hipEventRecord(e1, st));
                HIP_OK(hipEventSynchronize(e1));
                float m1 = 0;
                HIP_OK(hipEventElapsedTime(&m1, e0, e1));
                ms = std::min(ms, m1);
            }
            // a later candidate must be 3 % faster to replace the incumbent: near ties resolve to
            // the same shape from run to run (candidates in a fixed order)
            if (ms < 0.97 * best) {
                best = ms;
                bs = sh;
            }
        }
        b.lane = bs.lane;
        b.whole = bs.whole;
        b.JT = bs.jt;
        b.mfma = bs.mfma;
        layout_batch(c, r.name, jobs, b);
        c->shapes.push_back({r.level, r.kind, b.lane, b.whole, b.JT, b.mfma, b.nreal, best});
    }
    HIP_OK(hipStreamSynchronize(st));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    drop_graphs(c);
}

template <class S, class D>
static void convert(fmmbem_ctx *c, int64_t n, const S *a, D *b);
template <>
void convert<double2, float2>(fmmbem_ctx *c, int64_t n, const double2 *a, float2 *b) {
    if (n <= 0) return;
    k_cvt_d2f<<<ceil_div(n, 256), 256, 0, c->cur>>>(n, a, b);
    LAUNCH_OK();
}
template <>
void convert<float2, double2>(fmmbem_ctx *c, int64_t n, const float2 *a, double2 *b) {
    if (n <= 0) return;
    k_cvt_f2d<<<ceil_div(n, 256), 256, 0, c->cur>>>(n, a, b);
    LAUNCH_OK();
}
template <>
void convert<double, float>(fmmbem_ctx *c, int64_t n, const double *a, float *b) {
    if (n <= 0) return;
    k_cvt_real_d2f<<<ceil_div(n, 256), 256, 0, c->cur>>>(n, a, b);
    LAUNCH_OK();
}

// FP32 copies of every table the mixed-precision product reads (made once per wavenumber)
static void ensure_mixed(fmmbem_ctx *c) {
    if (c->mixed_ready) return;
    TreeHost &T = c->tree;
    const int L = T.depth;
    for (int l = 2; l <= L; ++l) {
        LevelDev &D = c->lev[l];
        const int p = D.p;
        std::string s = "L" + std::to_string(l) + "_";
        const int64_t nm = coax_table_size(p) * std::max(D.ntau, 1);
        D.coax_m2l32 = dget<float2>(c->buf, s + "coax_m2l32", nm + TABLE_PAD);
        convert(c, nm + TABLE_PAD, (const double2 *)D.coax_m2l, D.coax_m2l32);
        if (l < L) {
            const int PT = std::max(p, c->lev[l + 1].p);
            D.coax_up32 = dget<float2>(c->buf, s + "coax_up32", coax_table_size(PT) + TABLE_PAD);
            convert(c, coax_table_size(PT) + TABLE_PAD, (const double2 *)D.coax_up, D.coax_up32);
        }
        TransBatch *bs[3] = {&D.m2l, &D.up, &D.down};
        const char *nm3[3] = {"m2l", "up", "down"};
        for (int q = 0; q < 3; ++q) {
            TransBatch &b = *bs[q];
            if (b.njob == 0) continue;
            const int64_t nh = (int64_t)std::max(1, b.nbeta) * rot_table_size(b.P);
            b.H32 = dget<float>(c->buf, s + nm3[q] + "_H32", nh + TABLE_PAD);
            b.HT32 = dget<float>(c->buf, s + nm3[q] + "_HT32", nh + TABLE_PAD);
            convert(c, nh + TABLE_PAD, (const double *)b.H, b.H32);
            convert(c, nh + TABLE_PAD, (const double *)b.HT, b.HT32);
            if (b.frH) {
                const int64_t nr = (int64_t)std::max(1, b.nbeta) * TF_FR_ROT, nc = (int64_t)b.nfrc * TF_FR_COAX;
                b.frH32 = dget<float>(c->buf, s + nm3[q] + "_frH32", nr);
                b.frHT32 = dget<float>(c->buf, s + nm3[q] + "_frHT32", nr);
                b.frC32 = dget<float>(c->buf, s + nm3[q] + "_frC32", nc);
                convert(c, nr, (const double *)b.frH, b.frH32);
                convert(c, nr, (const double *)b.frHT, b.frHT32);
                convert(c, nc, (const double *)b.frC, b.frC32);
            }
        }
    }
    const int64_t nph = (int64_t)NDIR * (2 * c->delta_p + 1);
    float2 *ph = dget<float2>(c->buf, "phA32", nph);
    convert(c, nph, (const double2 *)c->buf.find("phA"), ph);
    float2 *nL = dget<float2>(c->buf, "near_L32", c->near_nnz), *nM = dget<float2>(c->buf, "near_M32", c->near_nnz);
    convert(c, c->near_nnz, (const double2 *)c->buf.find("near_L"), nL);
    convert(c, c->near_nnz, (const double2 *)c->buf.find("near_M"), nM);
    HIP_OK(hipStreamSynchronize(c->stream));
    c->mixed_ready = true;
}

// Zero a device range with a fill kernel (safe inside captured graphs, unlike memset nodes).
static void zero_dev(fmmbem_ctx *c, void *ptr, size_t bytes) {
    if (bytes == 0) return;
    if (bytes % 8) throw FmmError(FMMBEM_EINVAL, "zero_dev: size not a multiple of 8 bytes");
    const int64_t n8 = (int64_t)(bytes / 8);
    k_zero8<<<ceil_div(n8, 256), 256, 0, c->cur>>>(n8, (uint64_t *)ptr);
    LAUNCH_OK();
}

static void rec(fmmbem_ctx *c, int i) {
    if (!c->capturing) HIP_OK(hipEventRecord(c->ev[i], c->cur));
}

// Expansion arrays hold nr vectors per box (vector-inner); grow them when more are asked for.
static void ensure_nr(fmmbem_ctx *c, int nr, bool mixed) {
    if (nr <= c->nr_cap && (!mixed || nr <= c->nr_cap32)) return;
    if (c->capturing) throw FmmError(FMMBEM_EINVAL, "expansion storage must exist before graph capture");
    drop_graphs(c);
    for (int l = 2; l <= c->tree.depth; ++l) {
        LevelDev &D = c->lev[l];
        std::string s = "L" + std::to_string(l) + "_";
        const size_t cnt = (size_t)D.nbox * nr * D.p * D.p;
        if (nr > c->nr_cap) {
            D.M = dget<double2>(c->buf, s + "M", cnt);
            D.L = dget<double2>(c->buf, s + "L", cnt);
        }
        if (mixed) {
            D.M32 = dget<float2>(c->buf, s + "M32", cnt);
            D.L32 = dget<float2>(c->buf, s + "L32", cnt);
        }
    }
    c->nr_cap = std::max(c->nr_cap, nr);
    if (mixed) c->nr_cap32 = std::max(c->nr_cap32, nr);
}

// y (caller order, nr x N) = half * x + L[sigma] + M[mu] at the centroids; sigma/mu in tree
// order with the nr vectors interleaved.
// Fork/join on the product's two streams: events created on first use and reused.  A wait
// refers to the latest record enqueued on the host before it, so every record below is enqueued
// before its wait.
static hipEvent_t fj_event(fmmbem_ctx *c, int slot) {
    while ((int)c->fj.size() <= slot) {
        hipEvent_t e;
        HIP_OK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        c->fj.push_back(e);
    }
    return c->fj[slot];
}
static void ev_record(fmmbem_ctx *c, int slot, hipStream_t s) { HIP_OK(hipEventRecord(fj_event(c, slot), s)); }
static void ev_wait(fmmbem_ctx *c, int slot, hipStream_t s) { HIP_OK(hipStreamWaitEvent(s, fj_event(c, slot), 0)); }
// completion of a *_dev call on the library's stream, waited for by the caller's stream (never
// recorded inside a captured product)
constexpr int EV_CALLER_IN = 39, EV_CALLER_DONE = 40;

// Far-field translations of one product on two streams.  The main stream A runs, straight after
// P2M, the M2M chain (short: it feeds every level's M2L, so it goes first) and then the M2L of the
// deepest levels (l >= L - 2: by far the most jobs), leaf level first; the side stream B, after the
// near field, runs the M2L of the upper levels and then the L2L chain.
//   M2L(l), l < lsplit (B)  waits for M(l) from the chain (A)
//   L2L into l >= lsplit    waits for A's last M2L (level lsplit): A runs its levels in order, so
//   (B)                     then L(l-1) is complete and no M2L still adds into L(l) (which the
//                           stream running M2L(l) zeroes first); B's own order covers the rest
//   join                    A waits for B's last L2L
// Every level's local expansions receive M2L and then L2L in the same order as on one stream.
template <class R>
static void far_field(fmmbem_ctx *c, int nr, bool mixed, const std::function<void()> &after_m2l = nullptr) {
    using C = typename Cx<R>::T;
    const int L = c->tree.depth;
    hipStream_t A = c->stream, B = c->opt.streams >= 2 ? c->side : c->stream;
    const C *ph = (const C *)c->buf.find(mixed ? "phA32" : "phA");
    auto M = [&](int l) -> C * { return mixed ? (C *)c->lev[l].M32 : (C *)c->lev[l].M; };
    auto Lc = [&](int l) -> C * { return mixed ? (C *)c->lev[l].L32 : (C *)c->lev[l].L; };
    auto tab = [&](const TransBatch &b, const double2 *coax64, const float2 *coax32) -> TransTables<R> {
        if constexpr (sizeof(R) == 8) return tables64(b, coax64);
        else return tables32(b, coax32);
    };
    const int lsplit = std::max(2, L - 2);  // levels >= lsplit: M2L on A
    const int EV_M2L = 2, EV_B = 3, EV_M = 4;  // EV_M + l: M(l) ready
    // A: M2M chain
    c->cur = A;
    for (int l = L - 1; l >= 2; --l) {
        LevelDev &P_ = c->lev[l];
        run_batch<R>(c, nr, P_.up, M(l + 1), M(l), tab(P_.up, P_.coax_up, P_.coax_up32), ph, false);
        if (l < lsplit) ev_record(c, EV_M + l, A);
    }
    rec(c, 4);
    // A: M2L of the deep levels
    for (int l = L; l >= lsplit; --l) {
        LevelDev &D = c->lev[l];
        run_batch<R>(c, nr, D.m2l, M(l), Lc(l), tab(D.m2l, D.coax_m2l, D.coax_m2l32), ph, false);
    }
    ev_record(c, EV_M2L, A);
    // A: whatever the caller runs beside the L2L chain (the near field of a product)
    if (after_m2l) after_m2l();
    // B: M2L of the upper levels, then the L2L chain top-down
    c->cur = B;
    for (int l = lsplit - 1; l >= 2; --l) {
        LevelDev &D = c->lev[l];
        ev_wait(c, EV_M + l, B);
        run_batch<R>(c, nr, D.m2l, M(l), Lc(l), tab(D.m2l, D.coax_m2l, D.coax_m2l32), ph, false);
    }
    bool a_done = false;
    for (int l = 3; l <= L; ++l) {
        LevelDev &P_ = c->lev[l - 1];
        if (l >= lsplit && !a_done) {
            ev_wait(c, EV_M2L, B);
            a_done = true;
        }
        run_batch<R>(c, nr, P_.down, Lc(l - 1), Lc(l), tab(P_.down, P_.coax_up, P_.coax_up32), ph);
    }
    if (!a_done) ev_wait(c, EV_M2L, B);
    ev_record(c, EV_B, B);
    c->cur = A;
    ev_wait(c, EV_B, A);
}

static void fmm_pass(fmmbem_ctx *c, int nr, const double2 *sigma, const double2 *mu, const double2 *x, double half,
                     double2 *y, bool exact_far, bool mixed = false) {
    TreeHost &T = c->tree;
    const int L = T.depth;
    hipStream_t A = c->stream, B = c->opt.streams >= 2 ? c->side : c->stream;
    const int64_t n = c->nt;
    const int nleaf = (int)T.leaf_start.size() - 1;
    auto I32 = [&](const char *s) { return (int32_t *)c->buf.find(s); };
    const double4 *ec = (double4 *)c->buf.find("ec"), *en = (double4 *)c->buf.find("en");
    double2 *ynear = dget<double2>(c->scratch, "ynear", (size_t)n * nr);
    ensure_nr(c, nr, mixed);
    struct CurGuard {
        fmmbem_ctx *c;
        ~CurGuard() { c->cur = c->stream; }
    } guard{c};
    auto near_field = [&]() {
        int pe = prof_begin(c);
        const double pairs = exact_far ? (double)n * n : (double)c->p2p_pairs;
        launch_p2p(nr, mixed, nleaf, I32("leaf_start"), I32("nbr_start"), I32("nbr_list"), exact_far ? 1 : 0, ec, en,
                   sigma, mu, c->k, c->rc * c->rc, I32("near_start"), I32("near_col"),
                   c->buf.find(mixed ? "near_L32" : "near_L"), c->buf.find(mixed ? "near_M32" : "near_M"), ynear,
                   c->cur);
        // one-point pairs: ~40 flops each (sincos counted as 20), kernel shared by the nr vectors;
        // bytes: element data, densities, near table and output, each read once
        const double tb = mixed ? 16.0 : 32.0;
        prof_end(c, pe, mixed ? "k_p2p32" : "k_p2p", (40.0 + 16.0 * (nr - 1)) * pairs + 16.0 * nr * c->near_nnz,
                 80.0 * n + 48.0 * n * nr + (8.0 + tb) * c->near_nnz);
    };
    // The near field of a product runs on the main stream after the M2L of the deep levels, beside
    // the side stream's L2L chain (few workgroups per level), and L2P follows both; P2M and the M2M
    // chain at the start have the device to themselves.
    rec(c, 1);
    if (exact_far) near_field();
    rec(c, 2);
    c->cur = A;
    int pe = 0;
    if (!exact_far) {
        LevelDev &LL = c->lev[L];
        const int p = LL.p;
        check_p2m(nr, p);
        const size_t pp = (size_t)p * p;
        pe = prof_begin(c);
        launch_p2m(nr, nleaf, p, I32("leaf_start"), LL.center, ec, en, sigma, mu, c->k, leg_table(c), LL.M, A);
        prof_end(c, pe, "k_p2m", (double)n * pp * 2 * 8.0 * nr, 112.0 * n + 32.0 * n * nr + 16.0 * nleaf * pp * nr);
        if (mixed) {
            // FP32 translations between an FP64 P2M and an FP64 L2P
            pe = prof_begin(c);
            convert(c, (int64_t)LL.nbox * nr * pp, (const double2 *)LL.M, LL.M32);
            prof_end(c, pe, "k_cvt", 0.0, 24.0 * LL.nbox * pp * nr);
        }
        rec(c, 3);
        if (mixed) far_field<float>(c, nr, true, near_field);
        else far_field<double>(c, nr, false, near_field);
        if (mixed) {
            pe = prof_begin(c);
            convert(c, (int64_t)LL.nbox * nr * pp, (const float2 *)LL.L32, LL.L);
            prof_end(c, pe, "k_cvt", 0.0, 24.0 * LL.nbox * pp * nr);
        }
        rec(c, 5);
    } else {
        for (int e = 3; e <= 5; ++e) rec(c, e);
    }
    rec(c, 6);
    LevelDev &LL = c->lev[L];
    pe = prof_begin(c);
    launch_l2p(nr, nleaf, LL.p, I32("leaf_start"), LL.center, ec, LL.L, c->k, leg_table(c), ynear, half,
               I32("perm"), n, x, y, exact_far ? 0 : 1, A);
    prof_end(c, pe, "k_l2p", (double)n * LL.p * LL.p * 8.0 * nr,
             32.0 * n + 16.0 * n * 3 * nr + 16.0 * nleaf * LL.p * LL.p * nr);
    rec(c, 7);
    (void)B;
}

// y = A x for nr vectors (x, y: nr x N device arrays, caller order), nr in {1, 2, 4}
static void matvec_chunk(fmmbem_ctx *c, int nr, const double2 *x, double2 *y, bool exact_far, bool mixed) {
    hipStream_t st = c->stream;
    const int64_t n = c->nt;
    double2 *sigma = dget<double2>(c->scratch, "sigma", (size_t)n * nr);
    double2 *mu = dget<double2>(c->scratch, "mu", (size_t)n * nr);
    rec(c, 0);
    k_densities<<<ceil_div(n * nr, 256), 256, 0, st>>>(n, nr, (int32_t *)c->buf.find("perm"), x,
                                                       (double2 *)c->buf.find("beta"), c->k, sigma, mu);
    LAUNCH_OK();
    if (mixed) ensure_mixed(c);
    fmm_pass(c, nr, sigma, mu, x, 0.5, y, exact_far, mixed);
    rec(c, 8);
}

// ------------------------------------------------------------------ captured products
void drop_graphs(fmmbem_ctx *c) {
    for (auto &g : c->graphs) (void)hipGraphExecDestroy(g.exec);
    c->graphs.clear();
}

// One product of nr vectors by replaying a HIP graph captured on the staging buffers g_x/g_y.
// The graph is (re)captured when none exists for (nr, precision) or when a buffer it refers
// to has been freed since (the buffers' generation counters moved).
static void matvec_graph(fmmbem_ctx *c, int nr, const double2 *x, double2 *y, bool mixed) {
    hipStream_t st = c->stream;
    const int64_t n = c->nt;
    double2 *gx = dget<double2>(c->scratch, "g_x", (size_t)n * 4), *gy = dget<double2>(c->scratch, "g_y", (size_t)n * 4);
    const size_t bytes = sizeof(double2) * n * nr;
    HIP_OK(hipMemcpyAsync(gx, x, bytes, hipMemcpyDeviceToDevice, st));
    fmmbem_ctx::GraphEntry *g = nullptr;
    for (auto &e : c->graphs)
        if (e.nr == nr && e.mixed == mixed) g = &e;
    if (g && (g->gen_buf != c->buf.gen || g->gen_scr != c->scratch.gen)) {
        drop_graphs(c);  // some captured pointer may be stale
        g = nullptr;
    }
    const bool replay = g != nullptr;
    if (replay) {
        rec(c, 0);
        HIP_OK(hipGraphLaunch(g->exec, st));
    } else {
        // eager product first: it allocates everything the product touches, then capture it
        matvec_chunk(c, nr, gx, gy, false, mixed);
        hipGraph_t graph = nullptr;
        HIP_OK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
        c->capturing = true;
        try {
            matvec_chunk(c, nr, gx, gy, false, mixed);
        } catch (...) {
            c->capturing = false;
            (void)hipStreamEndCapture(st, &graph);
            if (graph) (void)hipGraphDestroy(graph);
            throw;
        }
        c->capturing = false;
        HIP_OK(hipStreamEndCapture(st, &graph));
        hipGraphExec_t exec = nullptr;
        hipError_t ie = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        HIP_OK(ie);
        c->graphs.push_back({nr, mixed, exec, c->buf.gen, c->scratch.gen});
    }
    HIP_OK(hipMemcpyAsync(y, gy, bytes, hipMemcpyDeviceToDevice, st));
    // a replay records the phase events only around the whole product, after the copy into y
    if (replay)
        for (int e = 1; e <= 8; ++e) rec(c, e);
}

// any number of vectors, in chunks of 4, 2 and 1 (the kernels' right-hand-side counts)
static void matvec_dev(fmmbem_ctx *c, int nrhs, const double2 *x, double2 *y, bool exact_far, bool mixed = false,
                       bool allow_graph = true) {
    const int64_t n = c->nt;
    const bool graph = allow_graph && c->opt.graphs && !c->prof_on && !exact_far;
    int r = 0;
    while (r < nrhs) {
        const int left = nrhs - r, nr = left >= 4 ? 4 : left >= 2 ? 2 : 1;
        if (graph) matvec_graph(c, nr, x + (int64_t)r * n, y + (int64_t)r * n, mixed);
        else matvec_chunk(c, nr, x + (int64_t)r * n, y + (int64_t)r * n, exact_far, mixed);
        r += nr;
    }
}

static void read_timings(fmmbem_ctx *c) {
    HIP_OK(hipEventSynchronize(c->ev[8]));
    float t;
    auto el = [&](int a, int b) {
        HIP_OK(hipEventElapsedTime(&t, c->ev[a], c->ev[b]));
        return (double)t;
    };
    // the near field (side stream) and P2M (main stream) both start at the fork (event 1)
    c->last.ms[0] = el(0, 1);
    c->last.ms[1] = el(1, 2);
    c->last.ms[2] = el(1, 3);
    c->last.ms[3] = el(3, 4);
    c->last.ms[4] = el(4, 5);  // M2L + L2L
    c->last.ms[5] = 0.0;
    c->last.ms[6] = el(6, 7);
    c->last.ms[7] = el(0, 8);
}

static void rhs_dev(fmmbem_ctx *c, int isrc, double2 *b) {
    hipStream_t st = c->stream;
    const int64_t n = c->nt;
    double2 *sigma = dget<double2>(c->scratch, "sigma", n), *mu = dget<double2>(c->scratch, "mu", n);
    const double *rs = &c->src[3 * isrc];
    k_gamma<<<ceil_div(n, 256), 256, 0, st>>>(n, (double4 *)c->buf.find("ec"), (double4 *)c->buf.find("en"),
                                              (double2 *)c->buf.find("beta"), c->k, rs[0], rs[1], rs[2],
                                              c->src_amp[isrc], sigma, mu);
    LAUNCH_OK();
    HIP_OK(hipEventRecord(c->ev[0], st));
    fmm_pass(c, 1, sigma, mu, nullptr, 0.0, b, false);
    HIP_OK(hipEventRecord(c->ev[8], st));
}

// ------------------------------------------------------------------ indirect formulation (Eq. ibem5)
static bool indirect(const fmmbem_ctx *c) { return c->formulation == FMMBEM_INDIRECT; }

// L' and M' near entries (same CSR as L and M), built once per (mesh, k) when first needed
static void ensure_indirect(fmmbem_ctx *c) {
    if (c->indirect_ready) return;
    hipStream_t st = c->stream;
    double2 *lp = dget<double2>(c->buf, "near_Lp", c->near_nnz), *mp = dget<double2>(c->buf, "near_Mp", c->near_nnz);
    if (c->near_nnz > 0) {
        k_near_quad_n<<<ceil_div(c->near_nnz, 128), 128, 0, st>>>(
            c->near_nnz, (int32_t *)c->buf.find("near_row"), (int32_t *)c->buf.find("near_col"),
            (double4 *)c->buf.find("ec"), (double4 *)c->buf.find("en"), (double *)c->buf.find("ev"), c->k, lp, mp);
        LAUNCH_OK();
    }
    HIP_OK(hipStreamSynchronize(st));
    c->indirect_ready = true;
}

// potential (row 1) and normal derivative (row 2) of the layers (sigma, mu) at the centroids,
// plus the local terms of Eq. ibem5 when x (2N, caller order) is given; y is 2N.  The near field
// runs on the side stream beside P2M and the translations (the same two-stream far field as the
// direct products); with `mixed` the translations run in FP32 between an FP64 P2M and the FP64
// local derivatives and L2P, and the near field stays FP64.
static void fmm_pass_ind(fmmbem_ctx *c, const double2 *sigma, const double2 *mu, const double2 *x, double2 *y,
                         bool exact_far, bool mixed = false) {
    ensure_indirect(c);
    if (mixed) ensure_mixed(c);
    ensure_nr(c, 1, mixed);
    TreeHost &T = c->tree;
    const int L = T.depth;
    hipStream_t A = c->stream, B = c->opt.streams >= 2 ? c->side : c->stream;
    const int64_t n = c->nt;
    const int nleaf = (int)T.leaf_start.size() - 1;
    auto I32 = [&](const char *s) { return (int32_t *)c->buf.find(s); };
    const double4 *ec = (double4 *)c->buf.find("ec"), *en = (double4 *)c->buf.find("en");
    double2 *yv = dget<double2>(c->scratch, "ynear", n), *yn = dget<double2>(c->scratch, "ynearn", n);
    struct CurGuard {
        fmmbem_ctx *c;
        ~CurGuard() { c->cur = c->stream; }
    } guard{c};
    if (!exact_far) {  // fork
        ev_record(c, 0, A);
        ev_wait(c, 0, B);
        c->cur = B;
    }
    int pe = prof_begin(c);
    k_p2p_n<<<nleaf, 64, 0, c->cur>>>(nleaf, I32("leaf_start"), I32("nbr_start"), I32("nbr_list"), exact_far ? 1 : 0,
                                      ec, en, sigma, mu, c->k, c->rc * c->rc, I32("near_start"), I32("near_col"),
                                      (double2 *)c->buf.find("near_L"), (double2 *)c->buf.find("near_M"),
                                      (double2 *)c->buf.find("near_Lp"), (double2 *)c->buf.find("near_Mp"), yv, yn);
    LAUNCH_OK();
    prof_end(c, pe, "k_p2p_n", 100.0 * (exact_far ? (double)n * n : (double)c->p2p_pairs), 0.0);
    c->cur = A;
    LevelDev &LL = c->lev[L];
    const int p = LL.p;
    const size_t q1 = (size_t)(p + 1) * (p + 1), pp = (size_t)p * p;
    double2 *Dz = dget<double2>(c->scratch, "ind_Dz", LL.nbox * q1), *Dp = dget<double2>(c->scratch, "ind_Dp", LL.nbox * q1),
            *Dm = dget<double2>(c->scratch, "ind_Dm", LL.nbox * q1);
    if (!exact_far) {
        pe = prof_begin(c);
        check_p2m(1, p);
        launch_p2m(1, nleaf, p, I32("leaf_start"), LL.center, ec, en, sigma, mu, c->k, leg_table(c), LL.M, A);
        prof_end(c, pe, "k_p2m", (double)n * pp * 2 * 8.0, 112.0 * n + 32.0 * n + 16.0 * nleaf * pp);
        if (mixed) {
            pe = prof_begin(c);
            convert(c, (int64_t)LL.nbox * pp, (const double2 *)LL.M, LL.M32);
            prof_end(c, pe, "k_cvt", 0.0, 24.0 * LL.nbox * pp);
            far_field<float>(c, 1, true);
            pe = prof_begin(c);
            convert(c, (int64_t)LL.nbox * pp, (const float2 *)LL.L32, LL.L);
            prof_end(c, pe, "k_cvt", 0.0, 24.0 * LL.nbox * pp);
        } else {
            far_field<double>(c, 1, false);
        }
        // the far field's join made the main stream wait for the side stream (near field included)
        k_local_derivs<<<nleaf, 256, 0, A>>>(nleaf, p, LL.L, c->k, Dz, Dp, Dm);
        LAUNCH_OK();
    }
    pe = prof_begin(c);
    k_l2p_n<<<nleaf, 64, ((size_t)64 * (p + 3) + (size_t)3 * (p + 1) * (p + 2) / 2) * sizeof(double), A>>>(
        nleaf, p, I32("leaf_start"), LL.center, ec, en, LL.L, Dz, Dp, Dm, c->k, leg_table(c), yv, yn, I32("perm"), n, x,
        (double2 *)c->buf.find("beta"), (double2 *)c->buf.find("betap"), y, exact_far ? 0 : 1);
    LAUNCH_OK();
    prof_end(c, pe, "k_l2p_n", (double)n * q1 * 8.0 * 4, 0.0);
}

static void matvec_ind(fmmbem_ctx *c, const double2 *x, double2 *y, bool exact_far, bool mixed = false) {
    const int64_t n = c->nt;
    double2 *sigma = dget<double2>(c->scratch, "sigma", n), *mu = dget<double2>(c->scratch, "mu", n);
    rec(c, 0);
    k_densities_ind<<<ceil_div(n, 256), 256, 0, c->stream>>>(n, (int32_t *)c->buf.find("perm"), x,
                                                             (double2 *)c->buf.find("beta"),
                                                             (double2 *)c->buf.find("betap"), c->k, sigma, mu);
    LAUNCH_OK();
    fmm_pass_ind(c, sigma, mu, x, y, exact_far, mixed);
    rec(c, 8);
}

static void rhs_ind(fmmbem_ctx *c, int isrc, double2 *b) {
    hipStream_t st = c->stream;
    const int64_t n = c->nt;
    double2 *gm = dget<double2>(c->scratch, "ind_gm", n), *gp = dget<double2>(c->scratch, "ind_gp", n);
    double2 *sigma = dget<double2>(c->scratch, "sigma", n), *mu = dget<double2>(c->scratch, "mu", n);
    const double *rs = &c->src[3 * isrc];
    k_gamma_pm<<<ceil_div(n, 256), 256, 0, st>>>(n, (double4 *)c->buf.find("ec"), (double4 *)c->buf.find("en"),
                                                 (double2 *)c->buf.find("beta"), (double2 *)c->buf.find("betap"), c->k,
                                                 rs[0], rs[1], rs[2], c->src_amp[isrc], gm, gp);
    LAUNCH_OK();
    // sigma = g- + g+, mu = 0; row 2 also gets (g+ - g-)/2
    vec_add(n, gm, gp, sigma, st);
    zero_dev(c, mu, sizeof(double2) * n);
    fmm_pass_ind(c, sigma, mu, nullptr, b, false);
    k_rhs_ind_local<<<ceil_div(n, 256), 256, 0, st>>>(n, (int32_t *)c->buf.find("perm"), gm, gp, b);
    LAUNCH_OK();
}

// ------------------------------------------------------------------ combined (Burton-Miller) direct form
// Eq. (dbem3) plus alpha = i/k times its normal derivative; the same unknown (psi_sc per element)
// and field (Eq. dbem1) as Eq. (dbem4).  Both halves come from one pass of the indirect
// machinery (potential and normal derivative of the layers sigma = -i k beta x, mu = x).
static bool burton_miller(const fmmbem_ctx *c) { return c->formulation == FMMBEM_DIRECT_BM; }
static double2 bm_alpha(const fmmbem_ctx *c) { return cmk(0.0, 1.0 / c->k); }

static void matvec_bm(fmmbem_ctx *c, const double2 *x, double2 *y, bool exact_far, bool mixed = false) {
    const int64_t n = c->nt;
    hipStream_t st = c->stream;
    double2 *sigma = dget<double2>(c->scratch, "sigma", n), *mu = dget<double2>(c->scratch, "mu", n);
    double2 *pq = dget<double2>(c->scratch, "bm_pq", 2 * n);
    rec(c, 0);
    k_densities<<<ceil_div(n, 256), 256, 0, st>>>(n, 1, (int32_t *)c->buf.find("perm"), x,
                                                  (double2 *)c->buf.find("beta"), c->k, sigma, mu);
    LAUNCH_OK();
    fmm_pass_ind(c, sigma, mu, nullptr, pq, exact_far, mixed);
    k_bm_combine<<<ceil_div(n, 256), 256, 0, st>>>(n, (int32_t *)c->buf.find("perm"), x,
                                                   (double2 *)c->buf.find("beta"), c->k, bm_alpha(c), pq, y);
    LAUNCH_OK();
    rec(c, 8);
}

static void rhs_bm(fmmbem_ctx *c, int isrc, double2 *b) {
    hipStream_t st = c->stream;
    const int64_t n = c->nt;
    double2 *sigma = dget<double2>(c->scratch, "sigma", n), *mu = dget<double2>(c->scratch, "mu", n);
    double2 *pq = dget<double2>(c->scratch, "bm_pq", 2 * n);
    const double *rs = &c->src[3 * isrc];
    // sigma = gamma (tree order), mu = 0
    k_gamma<<<ceil_div(n, 256), 256, 0, st>>>(n, (double4 *)c->buf.find("ec"), (double4 *)c->buf.find("en"),
                                              (double2 *)c->buf.find("beta"), c->k, rs[0], rs[1], rs[2],
                                              c->src_amp[isrc], sigma, mu);
    LAUNCH_OK();
    fmm_pass_ind(c, sigma, mu, nullptr, pq, false);
    k_bm_rhs<<<ceil_div(n, 256), 256, 0, st>>>(n, (int32_t *)c->buf.find("perm"), sigma, bm_alpha(c), pq, b);
    LAUNCH_OK();
}

// ------------------------------------------------------------------ normal-derivative form (Eq. dbem5)
// Unknown v = dpsi_sc/dn; A v = v/2 + beta (L[-i k v] + M[zeta v]) through the direct FMM pass;
// b = gamma/2 + beta M[zeta gamma].  zeta = 1/beta: every element needs beta != 0.
static bool dpsi(const fmmbem_ctx *c) { return c->formulation == FMMBEM_DIRECT_DPSI; }
static void check_dpsi_beta(const fmmbem_ctx *c) {
    for (const double2 &b : c->beta)
        if (b.x == 0.0 && b.y == 0.0)
            throw FmmError(FMMBEM_EINVAL, "Eq. dbem5 needs beta != 0 on every element (zeta = 1/beta)");
}

static void matvec_dpsi(fmmbem_ctx *c, const double2 *v, double2 *y, bool exact_far, bool mixed = false) {
    const int64_t n = c->nt;
    hipStream_t st = c->stream;
    if (mixed) ensure_mixed(c);
    double2 *sigma = dget<double2>(c->scratch, "sigma", n), *mu = dget<double2>(c->scratch, "mu", n);
    double2 *P = dget<double2>(c->scratch, "d5_p", n);
    const int32_t *perm = (int32_t *)c->buf.find("perm");
    const double2 *beta = (double2 *)c->buf.find("beta");
    rec(c, 0);
    k_densities_dpsi<<<ceil_div(n, 256), 256, 0, st>>>(n, perm, v, beta, c->k, sigma, mu);
    LAUNCH_OK();
    fmm_pass(c, 1, sigma, mu, nullptr, 0.0, P, exact_far, mixed);
    k_dpsi_combine<<<ceil_div(n, 256), 256, 0, st>>>(n, perm, v, beta, P, y);
    LAUNCH_OK();
    rec(c, 8);
}

static void rhs_dpsi(fmmbem_ctx *c, int isrc, double2 *b) {
    hipStream_t st = c->stream;
    const int64_t n = c->nt;
    double2 *sigma = dget<double2>(c->scratch, "sigma", n), *mu = dget<double2>(c->scratch, "mu", n);
    double2 *P = dget<double2>(c->scratch, "d5_p", n), *gam = dget<double2>(c->scratch, "d5_gam", n);
    const int32_t *perm = (int32_t *)c->buf.find("perm");
    const double2 *beta = (double2 *)c->buf.find("beta");
    const double *rs = &c->src[3 * isrc];
    k_gamma<<<ceil_div(n, 256), 256, 0, st>>>(n, (double4 *)c->buf.find("ec"), (double4 *)c->buf.find("en"), beta,
                                              c->k, rs[0], rs[1], rs[2], c->src_amp[isrc], sigma, mu);
    LAUNCH_OK();
    k_rhs_dpsi_dens<<<ceil_div(n, 256), 256, 0, st>>>(n, perm, beta, sigma, mu, gam);
    LAUNCH_OK();
    HIP_OK(hipEventRecord(c->ev[0], st));
    fmm_pass(c, 1, sigma, mu, nullptr, 0.0, P, false);
    HIP_OK(hipEventRecord(c->ev[8], st));
    k_dpsi_combine<<<ceil_div(n, 256), 256, 0, st>>>(n, perm, gam, beta, P, b);
    LAUNCH_OK();
}

// ------------------------------------------------------------------ operator dispatch, coarser inner FMM
// y = A x (device vectors, caller order) for the context's formulation
static void apply_operator(fmmbem_ctx *c, const double2 *x, double2 *y, bool mixed) {
    if (indirect(c)) matvec_ind(c, x, y, false, mixed);
    else if (burton_miller(c)) matvec_bm(c, x, y, false, mixed);
    else if (dpsi(c)) matvec_dpsi(c, x, y, false, mixed);
    else matvec_dev(c, 1, x, y, false, mixed);
}

}  // namespace fmm

using namespace fmm;

// ------------------------------------------------------------------ fixed field workspace
// Device workspace of fmmbem_eval_field_noalloc: the receiver formula's two density arrays
// (sigma, mu) for at most NOALLOC_MAX_N elements, 32 MiB.  Every device the library runs on holds
// its own copy until the process ends.  Host code never uses the array's name as an address: the
// address on each device comes from hipGetSymbolAddress, taken once per device at context creation
// with that device current.
static constexpr int64_t NOALLOC_MAX_N = (int64_t)1 << 20;
static __device__ __align__(256) double2 scratch[2 * NOALLOC_MAX_N];
static std::mutex g_noalloc_mu;
static std::map<int, double2 *> g_noalloc_ptr;  // device -> address of `scratch` there

// with `device` current
static void noalloc_init(int device) {
    std::lock_guard<std::mutex> lk(g_noalloc_mu);
    if (g_noalloc_ptr.count(device)) return;
    double2 *ptr = nullptr;
    HIP_OK(hipGetSymbolAddress((void **)&ptr, HIP_SYMBOL(scratch)));
    g_noalloc_ptr[device] = ptr;
}

static double2 *noalloc_scratch(int device) {
    std::lock_guard<std::mutex> lk(g_noalloc_mu);
    auto it = g_noalloc_ptr.find(device);
    return it == g_noalloc_ptr.end() ? nullptr : it->second;
}

// The coarser FMM of the inner GMRES (Section 4.3): a context of its own with the truncation rule's
// p_min and excess replaced, on the same inputs; rebuilt when those change.
static fmmbem_ctx *ensure_inner(fmmbem_ctx *c, int p_min, double p_excess) {
    const bool inputs = c->inner_gen != c->input_gen;
    if (c->inner && !inputs && c->inner_pmin == p_min && c->inner_pexc == p_excess) return c->inner;
    fmmbem_options o = c->opt;
    o.p_min = p_min;
    o.p_excess = p_excess;
    if (!c->inner) {
        if (int rc = fmmbem_create(&c->inner, c->device, &o)) throw FmmError(rc, "inner context");
    } else {
        c->inner->opt = o;
        c->inner->k_dirty = true;  // new truncation: tables and batches again
    }
    fmmbem_ctx *in = c->inner;
    auto chk = [&](int rc) {
        if (rc < 0) throw FmmError(rc, "inner context: " + in->err);
    };
    if (inputs) {
        chk(fmmbem_set_mesh(in, c->nv, c->xyz.data(), c->nt, c->tri.data()));
        chk(fmmbem_set_wavenumber(in, c->k));
        std::vector<fmmbem_c64> b(c->nt), bp;
        for (int64_t i = 0; i < c->nt; ++i) b[i] = {c->beta[i].x, c->beta[i].y};
        if (!c->beta_plus.empty()) {
            bp.resize(c->nt);
            for (int64_t i = 0; i < c->nt; ++i) bp[i] = {c->beta_plus[i].x, c->beta_plus[i].y};
        }
        chk(fmmbem_set_admittance(in, b.data(), bp.empty() ? nullptr : bp.data()));
        chk(fmmbem_set_formulation(in, c->formulation));
    }
    ensure_setup(in);
    HIP_OK(hipSetDevice(c->device));
    c->inner_gen = c->input_gen;
    c->inner_pmin = p_min;
    c->inner_pexc = p_excess;
    for (auto &e : c->xev)
        if (!e) HIP_OK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    return in;
}

// ------------------------------------------------------------------ ABI
#define GUARD_BEGIN try {
#define GUARD_END                               \
    }                                           \
    catch (const FmmError &e) {                 \
        if (ctx) ctx->err = e.what();           \
        return e.code;                          \
    }                                           \
    catch (const std::exception &e) {           \
        if (ctx) ctx->err = e.what();           \
        return FMMBEM_EDEVICE;                  \
    }

static int fail(fmmbem_ctx *ctx, int code, const std::string &m) {
    if (ctx) ctx->err = m;
    return code;
}

extern "C" {

void fmmbem_default_options(fmmbem_options *o) {
    o->rc_factor = 1.8;
    o->rc = 0.0;
    o->leaf_max = 64;
    o->p_min = 16;
    o->p_excess = 4.2;
    o->ktau_switch = 1.0;
    o->max_depth = 12;
    o->lds_budget = 0;
    o->graphs = 1;
    o->autotune = 0;
    o->lane_tiles = 1;
    o->streams = 2;
    o->mfma = 1;
    o->fused = 1;
    o->kd_leaf_min = 0.75;
}

void fmmbem_default_solve_opts(fmmbem_solve_opts *o) {
    o->tol = 1e-6;
    o->restart = 30;
    o->maxit = 500;
    o->precond = FMMBEM_PC_NEARBLOCK;
    o->precision = FMMBEM_FP64;
    o->diag_shift = 0.0;
    o->use_x0 = 0;
    o->inner_iters = 0;
    o->basis_fp32 = -1;
    o->inner_tol = 1e-2;
    o->inner_precision = FMMBEM_MIXED;
    o->inner_p_min = 0;
    o->inner_p_excess = 1.0;
    o->reorth = 1;
}

int fmmbem_release_workspace(fmmbem_ctx *ctx) {
    if (!ctx) return FMMBEM_EINVAL;
    GUARD_BEGIN
    HIP_OK(hipSetDevice(ctx->device));
    HIP_OK(hipStreamSynchronize(ctx->stream));
    drop_graphs(ctx);
    ctx->scratch.release_all();
    if (ctx->inner) {
        if (int rc = fmmbem_release_workspace(ctx->inner)) return fail(ctx, rc, "inner context: " + ctx->inner->err);
        HIP_OK(hipSetDevice(ctx->device));
    }
    return FMMBEM_OK;
    GUARD_END
}

int fmmbem_solve_history(fmmbem_ctx *ctx, int32_t max, double *est, int32_t *count) {
    if (!ctx || !count || (max > 0 && !est)) return FMMBEM_EINVAL;
    *count = (int32_t)ctx->history.size();
    for (int i = 0; i < max && i < *count; ++i) est[i] = ctx->history[i];
    return FMMBEM_OK;
}

int fmmbem_create(fmmbem_ctx **out, int hip_device, const fmmbem_options *opt) {
    fmmbem_ctx *ctx = nullptr;
    if (!out) return FMMBEM_EINVAL;
    *out = nullptr;
    try {
        int ndev = 0;
        if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) return FMMBEM_EDEVICE;
        if (hip_device < 0 || hip_device >= ndev) return FMMBEM_EINVAL;
        ctx = new fmmbem_ctx();
        ctx->device = hip_device;
        if (opt) ctx->opt = *opt;
        else fmmbem_default_options(&ctx->opt);
        HIP_OK(hipSetDevice(hip_device));
        HIP_OK(hipStreamCreateWithFlags(&ctx->stream, hipStreamNonBlocking));
        HIP_OK(hipStreamCreateWithFlags(&ctx->side, hipStreamNonBlocking));  // default priority, as the main one
        ctx->cur = ctx->stream;
        {
            hipDeviceProp_t prop;
            HIP_OK(hipGetDeviceProperties(&prop, hip_device));
            size_t lds = prop.sharedMemPerBlockOptin > 0 ? prop.sharedMemPerBlockOptin : prop.sharedMemPerBlock;
            ctx->lds_max = std::max<size_t>(lds, 65536);
            if (ctx->lds_max > 65536) {
                try {
                    trans_configure_lds(ctx->lds_max);
                } catch (const FmmError &) {
                    ctx->lds_max = 65536;
                    (void)hipGetLastError();  // clear the failed attribute request
                }
            }
        }
        for (auto &e : ctx->ev) HIP_OK(hipEventCreate(&e));
        (void)fj_event(ctx, EV_CALLER_DONE);  // every fork/join and caller event exists from here on
        noalloc_init(hip_device);
        *out = ctx;
        return FMMBEM_OK;
    } catch (const FmmError &e) {
        delete ctx;
        return e.code;
    }
}

int fmmbem_destroy(fmmbem_ctx *ctx) {
    if (!ctx) return FMMBEM_OK;
    (void)hipSetDevice(ctx->device);
    if (ctx->inner) (void)fmmbem_destroy(ctx->inner);
    for (auto &e : ctx->xev)
        if (e) (void)hipEventDestroy(e);
    if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
    if (ctx->side) (void)hipStreamSynchronize(ctx->side);
    drop_graphs(ctx);
    ctx->buf.release_all();
    ctx->scratch.release_all();
    for (auto &e : ctx->ev)
        if (e) (void)hipEventDestroy(e);
    for (auto &e : ctx->prof_ev) (void)hipEventDestroy(e);
    if (ctx->stream) (void)hipStreamDestroy(ctx->stream);
    if (ctx->side) (void)hipStreamDestroy(ctx->side);
    for (auto e : ctx->fj) (void)hipEventDestroy(e);
    delete ctx;
    return FMMBEM_OK;
}

const char *fmmbem_last_error(const fmmbem_ctx *ctx) { return ctx ? ctx->err.c_str() : "null context"; }

int fmmbem_set_mesh(fmmbem_ctx *ctx, int64_t nv, const double *xyz, int64_t nt, const int64_t *tri) {
    if (!ctx) return FMMBEM_EINVAL;
    if (nv < 3 || nt < 1 || !xyz || !tri) return fail(ctx, FMMBEM_EINVAL, "empty mesh");
    if (nt > (int64_t)1 << 30) return fail(ctx, FMMBEM_EINVAL, "too many triangles");
    double vol = 0.0;
    for (int64_t j = 0; j < nt; ++j) {
        for (int q = 0; q < 3; ++q)
            if (tri[3 * j + q] < 0 || tri[3 * j + q] >= nv)
                return fail(ctx, FMMBEM_EINVAL, "triangle " + std::to_string(j) + ": vertex index out of range");
        const double *a = xyz + 3 * tri[3 * j], *b = xyz + 3 * tri[3 * j + 1], *e = xyz + 3 * tri[3 * j + 2];
        double u[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]}, v[3] = {e[0] - a[0], e[1] - a[1], e[2] - a[2]};
        double w[3] = {u[1] * v[2] - u[2] * v[1], u[2] * v[0] - u[0] * v[2], u[0] * v[1] - u[1] * v[0]};
        double l = std::sqrt(w[0] * w[0] + w[1] * w[1] + w[2] * w[2]);
        double ext = std::max({std::fabs(u[0]), std::fabs(u[1]), std::fabs(u[2]), std::fabs(v[0]), std::fabs(v[1]), std::fabs(v[2])});
        if (!(l > 1e-14 * ext * ext) || !std::isfinite(l))
            return fail(ctx, FMMBEM_EINVAL, "triangle " + std::to_string(j) + " is degenerate");
        vol += ((a[0] + b[0] + e[0]) * w[0] + (a[1] + b[1] + e[1]) * w[1] + (a[2] + b[2] + e[2]) * w[2]) / 18.0;
    }
    if (!(vol > 0.0))
        return fail(ctx, FMMBEM_EINVAL, "enclosed volume is not positive: normals must point out of the fluid");
    ctx->xyz.assign(xyz, xyz + 3 * nv);
    ctx->tri.assign(tri, tri + 3 * nt);
    ctx->nv = nv;
    ctx->nt = nt;
    ctx->have_mesh = true;
    ctx->mesh_dirty = true;
    ++ctx->input_gen;
    if (ctx->have_beta && (int64_t)ctx->beta.size() != nt) ctx->have_beta = false;
    return FMMBEM_OK;
}

int fmmbem_set_wavenumber(fmmbem_ctx *ctx, double k) {
    if (!ctx) return FMMBEM_EINVAL;
    if (!std::isfinite(k) || !(k > 0.0)) return fail(ctx, FMMBEM_EINVAL, "wavenumber must be finite and > 0");
    if (k != ctx->k || !ctx->have_k) {
        ctx->k_dirty = true;
        ++ctx->input_gen;
    }
    ctx->k = k;
    ctx->have_k = true;
    return FMMBEM_OK;
}

static int check_admittance(fmmbem_ctx *ctx, const fmmbem_c64 *beta, const char *name) {
    for (int64_t i = 0; i < ctx->nt; ++i)
        if (!(beta[i].re >= 0.0) || !std::isfinite(beta[i].re) || !std::isfinite(beta[i].im))
            return fail(ctx, FMMBEM_EINVAL,
                        std::string(name) + "[" + std::to_string(i) + "]: Re(beta) must be finite and >= 0 (passive wall)");
    return FMMBEM_OK;
}

int fmmbem_set_admittance(fmmbem_ctx *ctx, const fmmbem_c64 *beta_minus, const fmmbem_c64 *beta_plus) {
    if (!ctx) return FMMBEM_EINVAL;
    if (!ctx->have_mesh) return fail(ctx, FMMBEM_ENOTREADY, "set the mesh before the admittance");
    if (!beta_minus) return fail(ctx, FMMBEM_EINVAL, "beta_minus is NULL");
    if (int e = check_admittance(ctx, beta_minus, "beta_minus")) return e;
    if (beta_plus)
        if (int e = check_admittance(ctx, beta_plus, "beta_plus")) return e;
    ctx->beta.resize(ctx->nt);
    for (int64_t i = 0; i < ctx->nt; ++i) ctx->beta[i] = cmk(beta_minus[i].re, beta_minus[i].im);
    ctx->beta_plus.clear();
    if (beta_plus) {
        ctx->beta_plus.resize(ctx->nt);
        for (int64_t i = 0; i < ctx->nt; ++i) ctx->beta_plus[i] = cmk(beta_plus[i].re, beta_plus[i].im);
    }
    ctx->have_beta = true;
    ctx->beta_dirty = true;
    ++ctx->input_gen;
    return FMMBEM_OK;
}

int fmmbem_set_sources(fmmbem_ctx *ctx, int32_t ns, const double *rs, const fmmbem_c64 *amp) {
    if (!ctx) return FMMBEM_EINVAL;
    if (ns < 1 || !rs) return fail(ctx, FMMBEM_EINVAL, "need at least one source");
    for (int i = 0; i < 3 * ns; ++i)
        if (!std::isfinite(rs[i])) return fail(ctx, FMMBEM_EINVAL, "source position not finite");
    ctx->src.assign(rs, rs + 3 * ns);
    ctx->src_amp.assign(ns, cmk(1, 0));
    if (amp)
        for (int i = 0; i < ns; ++i) ctx->src_amp[i] = cmk(amp[i].re, amp[i].im);
    return FMMBEM_OK;
}

int fmmbem_set_formulation(fmmbem_ctx *ctx, int f) {
    if (!ctx) return FMMBEM_EINVAL;
    if (f != FMMBEM_DIRECT && f != FMMBEM_DIRECT_DPSI && f != FMMBEM_DIRECT_BM && f != FMMBEM_INDIRECT)
        return fail(ctx, FMMBEM_EINVAL,
                    "formulation must be FMMBEM_DIRECT (Eq. dbem4), FMMBEM_DIRECT_DPSI (Eq. dbem5), "
                    "FMMBEM_DIRECT_BM or FMMBEM_INDIRECT (Eq. ibem5)");
    if (f != ctx->formulation) {
        drop_graphs(ctx);
        ++ctx->input_gen;
        // the leaf blocks and diagonals are the operator's: another formulation rebuilds them
        ctx->precond_ready_nb = ctx->precond_ready_diag = false;
    }
    ctx->formulation = f;
    return FMMBEM_OK;
}

int fmmbem_setup(fmmbem_ctx *ctx) {
    if (!ctx) return FMMBEM_EINVAL;
    GUARD_BEGIN
    HIP_OK(hipSetDevice(ctx->device));
    ensure_setup(ctx);
    return FMMBEM_OK;
    GUARD_END
}

int64_t fmmbem_num_unknowns(const fmmbem_ctx *ctx) {
    if (!ctx || !ctx->have_mesh) return -1;
    return ctx->formulation == FMMBEM_INDIRECT ? 2 * ctx->nt : ctx->nt;
}

// right-hand side of source s into the device vector b (num_unknowns values) on the library stream
static void rhs_one(fmmbem_ctx *ctx, int s, double2 *b) {
    if (indirect(ctx)) rhs_ind(ctx, s, b);
    else if (burton_miller(ctx)) rhs_bm(ctx, s, b);
    else if (dpsi(ctx)) {
        check_dpsi_beta(ctx);
        rhs_dpsi(ctx, s, b);
    } else rhs_dev(ctx, s, b);
}

int fmmbem_rhs(fmmbem_ctx *ctx, fmmbem_c64 *b) {
    if (!ctx) return FMMBEM_EINVAL;
    if (!b) return fail(ctx, FMMBEM_EINVAL, "b is NULL");
    GUARD_BEGIN
    HIP_OK(hipSetDevice(ctx->device));
    if (ctx->src.empty()) return fail(ctx, FMMBEM_ENOTREADY, "sources not set");
    ensure_setup(ctx);
    const int64_t n = fmmbem_num_unknowns(ctx);
    double2 *db = dget<double2>(ctx->scratch, "rhs_out", n);
    for (size_t s = 0; s < ctx->src.size() / 3; ++s) {
        rhs_one(ctx, (int)s, db);
        HIP_OK(hipMemcpyAsync(b + s * n, db, sizeof(double2) * n, hipMemcpyDeviceToHost, ctx->stream));
        HIP_OK(hipStreamSynchronize(ctx->stream));
    }
    return FMMBEM_OK;
    GUARD_END
}

int fmmbem_rhs_dev(fmmbem_ctx *ctx, void *b_dev, void *stream) {
    if (!ctx) return FMMBEM_EINVAL;
    if (!b_dev) return fail(ctx, FMMBEM_EINVAL, "b is NULL");
    GUARD_BEGIN
    HIP_OK(hipSetDevice(ctx->device));
    if (ctx->src.empty()) return fail(ctx, FMMBEM_ENOTREADY, "sources not set");
    ensure_setup(ctx);
    const int64_t n = fmmbem_num_unknowns(ctx);
    hipStream_t caller = (hipStream_t)stream;
    ev_record(ctx, EV_CALLER_IN, caller);
    ev_wait(ctx, EV_CALLER_IN, ctx->stream);
    for (size_t s = 0; s < ctx->src.size() / 3; ++s) rhs_one(ctx, (int)s, (double2 *)b_dev + s * n);
    ev_record(ctx, EV_CALLER_DONE, ctx->stream);
    ev_wait(ctx, EV_CALLER_DONE, caller);
    return FMMBEM_OK;
    GUARD_END
}

int fmmbem_matvec(fmmbem_ctx *ctx, int32_t nrhs, const fmmbem_c64 *x, fmmbem_c64 *y, int precision, int exact_far) {
    if (!ctx) return FMMBEM_EINVAL;
    if (!x || !y || nrhs < 1) return fail(ctx, FMMBEM_EINVAL, "bad vectors");
    if (precision != FMMBEM_FP64 && precision != FMMBEM_MIXED) return fail(ctx, FMMBEM_EINVAL, "unknown precision");
    if (precision == FMMBEM_MIXED && exact_far) return fail(ctx, FMMBEM_EINVAL, "exact_far is an FP64 product");
    GUARD_BEGIN
    HIP_OK(hipSetDevice(ctx->device));
    ensure_setup(ctx);
    if (indirect(ctx)) {
        const int64_t n2 = 2 * ctx->nt;
        double2 *dx = dget<double2>(ctx->scratch, "mv_x", n2), *dy = dget<double2>(ctx->scratch, "mv_y", n2);
        for (int r = 0; r < nrhs; ++r) {
            HIP_OK(hipMemcpyAsync(dx, x + (int64_t)r * n2, sizeof(double2) * n2, hipMemcpyHostToDevice, ctx->stream));
            matvec_ind(ctx, dx, dy, exact_far != 0, precision == FMMBEM_MIXED);
            HIP_OK(hipMemcpyAsync(y + (int64_t)r * n2, dy, sizeof(double2) * n2, hipMemcpyDeviceToHost, ctx->stream));
            HIP_OK(hipStreamSynchronize(ctx->stream));
        }
        return FMMBEM_OK;
    }
    if (burton_miller(ctx) || dpsi(ctx)) {
        const int64_t n = ctx->nt;
        if (dpsi(ctx)) check_dpsi_beta(ctx);
        double2 *dx = dget<double2>(ctx->scratch, "mv_x", n), *dy = dget<double2>(ctx->scratch, "mv_y", n);
        for (int r = 0; r < nrhs; ++r) {
            HIP_OK(hipMemcpyAsync(dx, x + (int64_t)r * n, sizeof(double2) * n, hipMemcpyHostToDevice, ctx->stream));
            if (dpsi(ctx)) matvec_dpsi(ctx, dx, dy, exact_far != 0, precision == FMMBEM_MIXED);
            else matvec_bm(ctx, dx, dy, exact_far != 0, precision == FMMBEM_MIXED);
            HIP_OK(hipMemcpyAsync(y + (int64_t)r * n, dy, sizeof(double2) * n, hipMemcpyDeviceToHost, ctx->stream));
            HIP_OK(hipStreamSynchronize(ctx->stream));
        }
        return FMMBEM_OK;
    }
    const int64_t n = ctx->nt;
    double2 *dx = dget<double2>(ctx->scratch, "mv_x", (size_t)n * std::min(nrhs, 4));
    double2 *dy = dget<double2>(ctx->scratch, "mv_y", (size_t)n * std::min(nrhs, 4));
    int r = 0;
    while (r < nrhs) {
        const int left = nrhs - r, nr = left >= 4 ? 4 : left >= 2 ? 2 : 1;
        HIP_OK(hipMemcpyAsync(dx, x + (int64_t)r * n, sizeof(double2) * n * nr, hipMemcpyHostToDevice, ctx->stream));
        matvec_dev(ctx, nr, dx, dy, exact_far != 0, precision == FMMBEM_MIXED, false);
        HIP_OK(hipMemcpyAsync(y + (int64_t)r * n, dy, sizeof(double2) * n * nr, hipMemcpyDeviceToHost, ctx->stream));
        HIP_OK(hipStreamSynchronize(ctx->stream));
        read_timings(ctx);
        r += nr;
    }
    return FMMBEM_OK;
    GUARD_END
}

int fmmbem_matvec_dev(fmmbem_ctx *ctx, int32_t nrhs, const void *x, void *y, int precision, void *stream) {
    if (!ctx) return FMMBEM_EINVAL;
    if (!x || !y || nrhs < 1) return fail(ctx, FMMBEM_EINVAL, "bad vectors");
    if (precision != FMMBEM_FP64 && precision != FMMBEM_MIXED) return fail(ctx, FMMBEM_EINVAL, "unknown precision");
    GUARD_BEGIN
    HIP_OK(hipSetDevice(ctx->device));
    ensure_setup(ctx);
    const int64_t n = ctx->nt;
    hipStream_t caller = (hipStream_t)stream;
    // order after the caller's stream, run on ours, then make the caller's stream wait
    ev_record(ctx, EV_CALLER_IN, caller);
    ev_wait(ctx, EV_CALLER_IN, ctx->stream);
    if (indirect(ctx)) {
        for (int r = 0; r < nrhs; ++r)
            matvec_ind(ctx, (const double2 *)x + (int64_t)r * 2 * n, (double2 *)y + (int64_t)r * 2 * n, false,
                       precision == FMMBEM_MIXED);
    } else if (burton_miller(ctx)) {
        for (int r = 0; r < nrhs; ++r)
            matvec_bm(ctx, (const double2 *)x + (int64_t)r * n, (double2 *)y + (int64_t)r * n, false,
                      precision == FMMBEM_MIXED);
    } else if (dpsi(ctx)) {
        check_dpsi_beta(ctx);
        for (int r = 0; r < nrhs; ++r)
            matvec_dpsi(ctx, (const double2 *)x + (int64_t)r * n, (double2 *)y + (int64_t)r * n, false,
                        precision == FMMBEM_MIXED);
    } else {
        matvec_dev(ctx, nrhs, (const double2 *)x, (double2 *)y, false, precision == FMMBEM_MIXED);
    }
    // the caller's stream waits for everything enqueued on ours, the copies into y included
    ev_record(ctx, EV_CALLER_DONE, ctx->stream);
    ev_wait(ctx, EV_CALLER_DONE, caller);
    return FMMBEM_OK;
    GUARD_END
}

int fmmbem_profile(fmmbem_ctx *ctx, int enable) {
    if (!ctx) return FMMBEM_EINVAL;
    GUARD_BEGIN
    HIP_OK(hipSetDevice(ctx->device));
    prof_flush(ctx);
    ctx->prof_stats.clear();
    ctx->prof_on = enable != 0;
    return FMMBEM_OK;
    GUARD_END
}

int fmmbem_kernel_stats(fmmbem_ctx *ctx, int max, fmmbem_kstat *out, int *count) {
    if (!ctx || !count) return FMMBEM_EINVAL;
    GUARD_BEGIN
    HIP_OK(hipSetDevice(ctx->device));
    prof_flush(ctx);
    *count = (int)ctx->prof_stats.size();
    for (int i = 0; i < max && i < *count; ++i) out[i] = ctx->prof_stats[i];
    return FMMBEM_OK;
    GUARD_END
}

int fmmbem_last_timings(fmmbem_ctx *ctx, double *ms8) {
    if (!ctx || !ms8) return FMMBEM_EINVAL;
    GUARD_BEGIN
    read_timings(ctx);
    for (int i = 0; i < 8; ++i) ms8[i] = ctx->last.ms[i];
    return FMMBEM_OK;
    GUARD_END
}

// Preconditioner of the solve options (data built on first use): z = P v on device vectors.
// Chunks of at most 64 consecutive unknowns per leaf (the learned preconditioner's samples).
static void ensure_chunks(fmmbem_ctx *c) {
    if (c->chunks_ready) return;
    const TreeHost &T = c->tree;
    const int nleaf = (int)T.leaf_start.size() - 1;
    std::vector<int32_t> cs, cn, cl;
    for (int b = 0; b < nleaf; ++b)
        for (int s = T.leaf_start[b]; s < T.leaf_start[b + 1]; s += 64) {
            cs.push_back(s);
            cn.push_back(std::min(64, T.leaf_start[b + 1] - s));
            cl.push_back(b);
        }
    c->nchunk = (int64_t)cs.size();
    upload(c->buf, "ch_s", cs, c->stream);
    upload(c->buf, "ch_n", cn, c->stream);
    upload(c->buf, "ch_l", cl, c->stream);
    std::vector<double> ka(nleaf, c->k * c->lev[T.depth].side);
    upload(c->buf, "leaf_ka", ka, c->stream);
    HIP_OK(hipStreamSynchronize(c->stream));
    c->chunks_ready = true;
}

// features of v on every chunk -> network output, chunk norms (scratch arrays)
static void mlp_run(fmmbem_ctx *c, const double2 *v, float **out, float **scale) {
    hipStream_t st = c->stream;
    const int64_t M = c->nchunk;
    float *X = dget<float>(c->scratch, "mlp_X", (size_t)M * MLP_IN);
    float *sc = dget<float>(c->scratch, "mlp_scale", M);
    float *A[4];
    for (int l = 0; l < 4; ++l) A[l] = dget<float>(c->scratch, "mlp_A" + std::to_string(l), (size_t)M * MLP_H);
    mlp_features(M, (int32_t *)c->buf.find("ch_s"), (int32_t *)c->buf.find("ch_n"), (int32_t *)c->buf.find("ch_l"),
                 (int32_t *)c->buf.find("perm"), v, (double4 *)c->buf.find("en"), (double2 *)c->buf.find("beta"),
                 (double *)c->buf.find("leaf_ka"), X, sc, st);
    c->mlp.forward(M, X, A, st);
    *out = A[3];
    *scale = sc;
}

// Leaf blocks of m n_b unknowns each (m = 1: one unknown per element; 2: the indirect pair): `fill`
// writes the operator's blocks at the offsets, then every block is inverted in place and the
// preconditioner applies blockdiag(A_BB^{-1}).
static std::function<void(const double2 *, double2 *)> leaf_block_pc(
    fmmbem_ctx *ctx, int m, const std::function<void(const int64_t *, double2 *)> &fill) {
    hipStream_t st = ctx->stream;
    const int64_t n = ctx->nt;
    const int nleaf = (int)ctx->tree.leaf_start.size() - 1;
    if (!ctx->precond_ready_nb) {
        std::vector<int64_t> off(nleaf + 1, 0);
        for (int b = 0; b < nleaf; ++b) {
            const int64_t nb = (int64_t)m * (ctx->tree.leaf_start[b + 1] - ctx->tree.leaf_start[b]);
            if (nb > 1024) throw FmmError(FMMBEM_EINVAL, "leaf too full for the block preconditioner");
            off[b + 1] = off[b] + nb * nb;
        }
        int64_t *doff = upload(ctx->buf, "pc_off", off, st);
        double2 *A = dget<double2>(ctx->buf, "pc_blocks", off[nleaf]);
        int32_t *piv = dget<int32_t>(ctx->scratch, "pc_piv", (size_t)m * n);
        int *status = dget<int>(ctx->scratch, "pc_status", 1);
        HIP_OK(hipMemsetAsync(status, 0, sizeof(int), st));
        fill(doff, A);
        k_leaf_invert<<<nleaf, 256, 0, st>>>(nleaf, (int32_t *)ctx->buf.find("leaf_start"), doff, A, piv, status, m);
        LAUNCH_OK();
        int hs = 0;
        HIP_OK(hipMemcpyAsync(&hs, status, sizeof(int), hipMemcpyDeviceToHost, st));
        HIP_OK(hipStreamSynchronize(st));
        if (hs) throw FmmError(FMMBEM_EBREAKDOWN, "singular leaf block in the near-field preconditioner");
        ctx->precond_ready_nb = true;
    }
    const int32_t *ls = (int32_t *)ctx->buf.find("leaf_start"), *pm = (int32_t *)ctx->buf.find("perm");
    const int64_t *doff = (int64_t *)ctx->buf.find("pc_off");
    const double2 *A = (double2 *)ctx->buf.find("pc_blocks");
    return [=](const double2 *v, double2 *z) {
        k_leaf_apply<<<nleaf, 128, 0, st>>>(nleaf, ls, doff, A, pm, v, z, m, n);
        LAUNCH_OK();
    };
}

static std::function<void(const double2 *, double2 *)> make_precond(fmmbem_ctx *ctx, const fmmbem_solve_opts &o) {
    hipStream_t st = ctx->stream;
    const int64_t n = ctx->nt;
    const int nleaf = (int)ctx->tree.leaf_start.size() - 1;
    if (ctx->formulation == FMMBEM_INDIRECT) {
        // the paper's choice for the indirect BEM: a diagonal preconditioner (here the 2x2 blocks
        // of each element's (psi-, psi+) pair, with the constant diag_shift added)
        if (o.precond == FMMBEM_PC_NONE)
            return [=](const double2 *v, double2 *z) {
                HIP_OK(hipMemcpyAsync(z, v, sizeof(double2) * 2 * n, hipMemcpyDeviceToDevice, st));
            };
        if (o.precond == FMMBEM_PC_NEARBLOCK) {
            // near-field leaf blocks of the two-sided operator (2 n_b unknowns per leaf)
            ensure_indirect(ctx);
            return leaf_block_pc(ctx, 2, [&](const int64_t *doff, double2 *A) {
                k_leaf_blocks_ind<<<nleaf, 256, 0, st>>>(
                    nleaf, (int32_t *)ctx->buf.find("leaf_start"), doff, (double4 *)ctx->buf.find("ec"),
                    (double4 *)ctx->buf.find("en"), (double2 *)ctx->buf.find("beta"), (double2 *)ctx->buf.find("betap"),
                    ctx->k, ctx->rc * ctx->rc, (int32_t *)ctx->buf.find("near_start"), (int32_t *)ctx->buf.find("near_col"),
                    (double2 *)ctx->buf.find("near_L"), (double2 *)ctx->buf.find("near_M"),
                    (double2 *)ctx->buf.find("near_Lp"), (double2 *)ctx->buf.find("near_Mp"), A);
                LAUNCH_OK();
            });
        }
        if (o.precond != FMMBEM_PC_DIAG)
            throw FmmError(FMMBEM_EINVAL, "the indirect formulation takes FMMBEM_PC_NONE, FMMBEM_PC_DIAG or "
                                          "FMMBEM_PC_NEARBLOCK");
        ensure_indirect(ctx);
        double2 *inv = dget<double2>(ctx->buf, "pc_dinv2", 4 * n);
        k_diag2_inv<<<ceil_div(n, 256), 256, 0, st>>>(n, (int32_t *)ctx->buf.find("near_start"),
                                                      (int32_t *)ctx->buf.find("near_col"), (double2 *)ctx->buf.find("near_L"),
                                                      (double2 *)ctx->buf.find("near_Mp"), (double2 *)ctx->buf.find("beta"),
                                                      (double2 *)ctx->buf.find("betap"), ctx->k, o.diag_shift, inv);
        LAUNCH_OK();
        const int32_t *pm = (int32_t *)ctx->buf.find("perm");
        return [=](const double2 *v, double2 *z) {
            k_mul_diag2<<<ceil_div(n, 256), 256, 0, st>>>(n, pm, inv, v, z);
            LAUNCH_OK();
        };
    }
    if (ctx->formulation == FMMBEM_DIRECT_BM) {
        if (o.precond == FMMBEM_PC_NONE)
            return [=](const double2 *v, double2 *z) {
                HIP_OK(hipMemcpyAsync(z, v, sizeof(double2) * n, hipMemcpyDeviceToDevice, st));
            };
        if (o.precond == FMMBEM_PC_NEARBLOCK) {
            ensure_indirect(ctx);
            return leaf_block_pc(ctx, 1, [&](const int64_t *doff, double2 *A) {
                k_leaf_blocks_bm<<<nleaf, 256, 0, st>>>(
                    nleaf, (int32_t *)ctx->buf.find("leaf_start"), doff, (double4 *)ctx->buf.find("ec"),
                    (double4 *)ctx->buf.find("en"), (double2 *)ctx->buf.find("beta"), ctx->k, bm_alpha(ctx),
                    ctx->rc * ctx->rc, (int32_t *)ctx->buf.find("near_start"), (int32_t *)ctx->buf.find("near_col"),
                    (double2 *)ctx->buf.find("near_L"), (double2 *)ctx->buf.find("near_M"),
                    (double2 *)ctx->buf.find("near_Lp"), (double2 *)ctx->buf.find("near_Mp"), A);
                LAUNCH_OK();
            });
        }
        if (o.precond != FMMBEM_PC_DIAG)
            throw FmmError(FMMBEM_EINVAL, "the combined direct formulation takes FMMBEM_PC_NONE, FMMBEM_PC_DIAG or "
                                          "FMMBEM_PC_NEARBLOCK");
        ensure_indirect(ctx);
        double2 *dinv = dget<double2>(ctx->buf, "pc_dinv_bm", n);
        k_diag_bm_inv<<<ceil_div(n, 256), 256, 0, st>>>(
            n, (int32_t *)ctx->buf.find("perm"), (int32_t *)ctx->buf.find("near_start"),
            (int32_t *)ctx->buf.find("near_col"), (double2 *)ctx->buf.find("near_L"), (double2 *)ctx->buf.find("near_M"),
            (double2 *)ctx->buf.find("near_Lp"), (double2 *)ctx->buf.find("near_Mp"), (double2 *)ctx->buf.find("beta"),
            ctx->k, bm_alpha(ctx), o.diag_shift, dinv);
        LAUNCH_OK();
        return [=](const double2 *v, double2 *z) {
            k_mul_diag<<<ceil_div(n, 256), 256, 0, st>>>(n, dinv, v, z);
            LAUNCH_OK();
        };
    }
    if (o.precond == FMMBEM_PC_LEARNED) {
        if (ctx->formulation != FMMBEM_DIRECT)
            throw FmmError(FMMBEM_EINVAL, "the learned preconditioner is for the direct formulation (Eq. dbem4)");
        if (!ctx->mlp.ready) throw FmmError(FMMBEM_ENOTREADY, "learned preconditioner not trained");
        fmmbem_solve_opts nb = o;
        nb.precond = FMMBEM_PC_NEARBLOCK;
        auto base = make_precond(ctx, nb);
        ensure_chunks(ctx);
        const int32_t *cs = (int32_t *)ctx->buf.find("ch_s"), *cn = (int32_t *)ctx->buf.find("ch_n");
        const int32_t *pm = (int32_t *)ctx->buf.find("perm");
        // z = P_near v + learned correction while the guard keeps it (mlp_active)
        return [=](const double2 *v, double2 *z) {
            base(v, z);
            if (!ctx->mlp_active) return;
            float *Y, *sc;
            mlp_run(ctx, v, &Y, &sc);
            mlp_apply(ctx->nchunk, cs, cn, pm, Y, sc, z, st);
        };
    }
    // preconditioner data
    if (o.precond == FMMBEM_PC_DIAG) {
        double2 *dinv = dget<double2>(ctx->buf, "pc_dinv", n);
        k_diag_inv<<<ceil_div(n, 256), 256, 0, st>>>(n, (int32_t *)ctx->buf.find("perm"), (int32_t *)ctx->buf.find("near_start"),
                                                     (int32_t *)ctx->buf.find("near_col"), (double2 *)ctx->buf.find("near_L"),
                                                     (double2 *)ctx->buf.find("near_M"), (double2 *)ctx->buf.find("beta"),
                                                     ctx->k, o.diag_shift, dinv);
        LAUNCH_OK();
    } else if (o.precond == FMMBEM_PC_NEARBLOCK && !ctx->precond_ready_nb) {
        std::vector<int64_t> off(nleaf + 1, 0);
        for (int b = 0; b < nleaf; ++b) {
            int64_t nb = ctx->tree.leaf_start[b + 1] - ctx->tree.leaf_start[b];
            if (nb > 1024) throw FmmError(FMMBEM_EINVAL, "leaf too full for the block preconditioner");
            off[b + 1] = off[b] + nb * nb;
        }
        int64_t *doff = upload(ctx->buf, "pc_off", off, st);
        double2 *A = dget<double2>(ctx->buf, "pc_blocks", off[nleaf]);
        int32_t *piv = dget<int32_t>(ctx->scratch, "pc_piv", n);
        int *status = dget<int>(ctx->scratch, "pc_status", 1);
        HIP_OK(hipMemsetAsync(status, 0, sizeof(int), st));
        k_leaf_blocks<<<nleaf, 256, 0, st>>>(nleaf, (int32_t *)ctx->buf.find("leaf_start"), doff, (double4 *)ctx->buf.find("ec"),
                                             (double4 *)ctx->buf.find("en"), (double2 *)ctx->buf.find("beta"), ctx->k,
                                             ctx->rc * ctx->rc, (int32_t *)ctx->buf.find("near_start"),
                                             (int32_t *)ctx->buf.find("near_col"), (double2 *)ctx->buf.find("near_L"),
                                             (double2 *)ctx->buf.find("near_M"), A);
        LAUNCH_OK();
        k_leaf_invert<<<nleaf, 256, 0, st>>>(nleaf, (int32_t *)ctx->buf.find("leaf_start"), doff, A, piv, status, 1);
        LAUNCH_OK();
        int hs = 0;
        HIP_OK(hipMemcpyAsync(&hs, status, sizeof(int), hipMemcpyDeviceToHost, st));
        HIP_OK(hipStreamSynchronize(st));
        if (hs) throw FmmError(FMMBEM_EBREAKDOWN, "singular leaf block in the near-field preconditioner");
        ctx->precond_ready_nb = true;
    }
    std::function<void(const double2 *, double2 *)> pc;
    if (o.precond == FMMBEM_PC_DIAG) {
        double2 *dinv = (double2 *)ctx->buf.find("pc_dinv");
        pc = [=](const double2 *v, double2 *z) {
            k_mul_diag<<<ceil_div(n, 256), 256, 0, st>>>(n, dinv, v, z);
            LAUNCH_OK();
        };
    } else if (o.precond == FMMBEM_PC_NEARBLOCK) {
        const int32_t *ls = (int32_t *)ctx->buf.find("leaf_start"), *pm = (int32_t *)ctx->buf.find("perm");
        const int64_t *doff = (int64_t *)ctx->buf.find("pc_off");
        const double2 *A = (double2 *)ctx->buf.find("pc_blocks");
        pc = [=](const double2 *v, double2 *z) {
            k_leaf_apply<<<nleaf, 128, 0, st>>>(nleaf, ls, doff, A, pm, v, z, 1, n);
            LAUNCH_OK();
        };
    } else {
        pc = [=](const double2 *v, double2 *z) {
            HIP_OK(hipMemcpyAsync(z, v, sizeof(double2) * n, hipMemcpyDeviceToDevice, st));
        };
    }
    return pc;
}

static int check_solve_opts(fmmbem_ctx *ctx, const fmmbem_solve_opts &o) {
    if (o.restart < 1 || o.maxit < 0 || !(o.tol > 0)) return fail(ctx, FMMBEM_EINVAL, "bad solve options");
    if (o.precision != FMMBEM_FP64 && o.precision != FMMBEM_MIXED) return fail(ctx, FMMBEM_EINVAL, "unknown precision");
    if (o.inner_iters < 0 || (o.inner_iters > 0 && !(o.inner_tol > 0)) ||
        (o.inner_precision != FMMBEM_FP64 && o.inner_precision != FMMBEM_MIXED))
        return fail(ctx, FMMBEM_EINVAL, "bad inner solve options");
    if (o.basis_fp32 < -1 || o.basis_fp32 > 1) return fail(ctx, FMMBEM_EINVAL, "basis_fp32 must be -1, 0 or 1");
    if (o.inner_p_min < 0 || (o.inner_p_min > 0 && !(o.inner_p_excess >= 0)))
        return fail(ctx, FMMBEM_EINVAL, "inner_p_min must be >= 0 and inner_p_excess >= 0");
    if (o.reorth < 0 || o.reorth > 2) return fail(ctx, FMMBEM_EINVAL, "reorth must be 0, 1 or 2");
    if (o.precond < FMMBEM_PC_NONE || o.precond > FMMBEM_PC_LEARNED) return fail(ctx, FMMBEM_EINVAL, "unknown preconditioner");
    return FMMBEM_OK;
}

// x: host array (caller == nullptr) or device array ordered after / before the caller's stream
static int solve_impl(fmmbem_ctx *ctx, int32_t isrc, const fmmbem_solve_opts *opts, void *x, bool dev,
                      hipStream_t caller, fmmbem_solve_report *rep) {
    if (!ctx) return FMMBEM_EINVAL;
    if (!x) return fail(ctx, FMMBEM_EINVAL, "x is NULL");
    fmmbem_solve_opts o;
    fmmbem_default_solve_opts(&o);
    if (opts) o = *opts;
    if (int e = check_solve_opts(ctx, o)) return e;
    GUARD_BEGIN
    HIP_OK(hipSetDevice(ctx->device));
    if (ctx->src.empty()) return fail(ctx, FMMBEM_ENOTREADY, "sources not set");
    if (isrc < 0 || isrc >= (int)(ctx->src.size() / 3)) return fail(ctx, FMMBEM_EINVAL, "bad source index");
    double t_before = 0;
    bool dirty = ctx->mesh_dirty || ctx->k_dirty || ctx->beta_dirty;
    ensure_setup(ctx);
    if (dirty) t_before = ctx->t_setup_last;
    fmmbem_ctx *coarse = nullptr;
    if (o.inner_iters > 0 && o.inner_p_min > 0) {
        auto ti = std::chrono::steady_clock::now();
        coarse = ensure_inner(ctx, o.inner_p_min, o.inner_p_excess);
        t_before += std::chrono::duration<double>(std::chrono::steady_clock::now() - ti).count();
    }
    auto t0 = std::chrono::steady_clock::now();
    hipStream_t st = ctx->stream;
    const bool ind = indirect(ctx), bm = burton_miller(ctx), dp = dpsi(ctx);
    const int64_t n = fmmbem_num_unknowns(ctx);
    auto pc = make_precond(ctx, o);
    if (dp && o.precond == FMMBEM_PC_NEARBLOCK) {
        // Eq. (dbem5)'s operator is Eq. (dbem4)'s similarity transform by diag(beta): its leaf-block
        // inverse is beta P4 zeta (the diagonal preconditioner is the same for both)
        auto p4 = pc;
        double2 *tmp = dget<double2>(ctx->scratch, "d5_pc", n);
        const int32_t *pm = (int32_t *)ctx->buf.find("perm");
        const double2 *be = (double2 *)ctx->buf.find("beta");
        pc = [=](const double2 *v, double2 *z) {
            k_scale_beta<<<ceil_div(n, 256), 256, 0, st>>>(n, pm, be, 1, v, tmp);
            LAUNCH_OK();
            p4(tmp, z);
            k_scale_beta<<<ceil_div(n, 256), 256, 0, st>>>(n, pm, be, 0, z, z);
            LAUNCH_OK();
        };
    }
    double2 *b = dget<double2>(ctx->scratch, "sv_b", n);
    double2 *dx = dget<double2>(ctx->scratch, "sv_x", n);
    if (dp) check_dpsi_beta(ctx);
    if (ind) rhs_ind(ctx, isrc, b);
    else if (bm) rhs_bm(ctx, isrc, b);
    else if (dp) rhs_dpsi(ctx, isrc, b);
    else rhs_dev(ctx, isrc, b);
    if (dev) {
        ev_record(ctx, EV_CALLER_IN, caller);
        ev_wait(ctx, EV_CALLER_IN, st);
    }
    if (o.use_x0) HIP_OK(hipMemcpyAsync(dx, x, sizeof(double2) * n, dev ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, st));
    // the Krylov products run in the requested arithmetic; restart residuals always in FP64
    int64_t n64 = 0, nmx = 0;
    auto product = [&](const double2 *a, double2 *y, bool mixed) {
        apply_operator(ctx, a, y, mixed);
        ++(mixed ? nmx : n64);
    };
    const bool mixed = o.precision == FMMBEM_MIXED;
    auto mv = [&](const double2 *a, double2 *y) { product(a, y, mixed); };
    auto mv64 = [&](const double2 *a, double2 *y) { product(a, y, false); };
    // Inner-outer scheme (Section 4.3): the outer flexible GMRES is preconditioned by a short,
    // low-accuracy GMRES on the same operator (inner_precision), itself preconditioned by `pc`; with
    // inner_p_min > 0 that operator is a second FMM with a smaller truncation number.
    std::function<void(const double2 *, double2 *)> outer_pc = pc;
    int64_t inner_its = 0, ncoarse = 0;
    if (o.inner_iters > 0) {
        const bool imixed = o.inner_precision == FMMBEM_MIXED;
        outer_pc = [&, imixed](const double2 *v, double2 *z) {
            auto imv = [&](const double2 *a, double2 *y) {
                if (!coarse) {
                    product(a, y, imixed);
                    return;
                }
                // the coarser operator runs on its own context's streams: order it after this
                // solve's stream and this stream after it
                HIP_OK(hipEventRecord(ctx->xev[0], st));
                HIP_OK(hipStreamWaitEvent(coarse->stream, ctx->xev[0], 0));
                apply_operator(coarse, a, y, imixed);
                HIP_OK(hipEventRecord(ctx->xev[1], coarse->stream));
                HIP_OK(hipStreamWaitEvent(st, ctx->xev[1], 0));
                ++ncoarse;
            };
            int it = 0, rs = 0;
            double rr = 1.0;
            const bool ib32 = o.basis_fp32 < 0 ? imixed : o.basis_fp32 != 0;
            int s = fgmres(n, st, ctx->scratch, "in_", imv, imv, pc, v, z, o.inner_tol, o.inner_iters, o.inner_iters,
                           false, false, nullptr, it, rs, rr, nullptr, ib32);
            if (s < 0) throw FmmError(s, "inner GMRES failed");
            inner_its += it;
        };
    }
    int iters = 0, restarts = 0;
    double rel = 1.0;
    ctx->history.clear();
    // Guard of the learned correction: it stays only while the residual keeps pace with the
    // plain solver's (3x margin on the training run's estimates, iteration by iteration) and
    // every restart's true FP64 residual improves on the previous one.
    int fallback_at = -1;
    double last_true = 2.0;  // lives as long as the hooks that refer to it
    FgmresHooks hk;
    if (o.precond == FMMBEM_PC_LEARNED) {
        ctx->mlp_active = true;
        hk.on_iter = [&](int it, double est) {
            const auto &ref = ctx->mlp_ref_hist;
            if (ctx->mlp_active && it >= 1 && it <= (int)ref.size() && est > 3.0 * ref[it - 1]) {
                ctx->mlp_active = false;
                fallback_at = it;
            }
        };
        hk.on_restart = [&](const double2 *, const double2 *, double r) {
            if (ctx->mlp_active && r > last_true) {
                ctx->mlp_active = false;
                fallback_at = iters;
            }
            last_true = r;
        };
    }
    const bool b32 = o.basis_fp32 < 0 ? mixed : o.basis_fp32 != 0;
    int status = fgmres(n, st, ctx->scratch, "", mv, mv64, outer_pc, b, dx, o.tol, o.restart, o.maxit, o.use_x0 != 0,
                        true, &ctx->history, iters, restarts, rel, &hk, b32, o.reorth);
    ctx->mlp_active = false;
    HIP_OK(hipMemcpyAsync(x, dx, sizeof(double2) * n, dev ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, st));
    if (dev) {
        ev_record(ctx, EV_CALLER_DONE, st);
        ev_wait(ctx, EV_CALLER_DONE, caller);
    }
    HIP_OK(hipStreamSynchronize(st));
    if (rep) {
        rep->iters = iters;
        rep->restarts = restarts;
        rep->rel_res = rel;
        rep->t_setup_s = t_before;
        rep->t_solve_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        rep->status = status;
        rep->matvecs_fp64 = n64;
        rep->matvecs_mixed = nmx;
        rep->matvecs_coarse = ncoarse;
        rep->inner_iters = inner_its;
        rep->pc_fallback_at = fallback_at;
    }
    if (status < 0) ctx->err = "solver failed";
    return status;
    GUARD_END
}

int fmmbem_solve(fmmbem_ctx *ctx, int32_t isrc, const fmmbem_solve_opts *opts, fmmbem_c64 *x, fmmbem_solve_report *rep) {
    return solve_impl(ctx, isrc, opts, x, false, nullptr, rep);
}

int fmmbem_solve_dev(fmmbem_ctx *ctx, int32_t isrc, const fmmbem_solve_opts *opts, void *x_dev,
                     fmmbem_solve_report *rep, void *stream) {
    return solve_impl(ctx, isrc, opts, x_dev, true, (hipStream_t)stream, rep);
}

int fmmbem_solve_batch(fmmbem_ctx *ctx, int32_t ns, const int32_t *isrc, const fmmbem_solve_opts *opts,
                       fmmbem_c64 *x, fmmbem_solve_report *rep) {
    if (!ctx) return FMMBEM_EINVAL;
    if (!x || !isrc || ns < 1) return fail(ctx, FMMBEM_EINVAL, "bad arguments");
    fmmbem_solve_opts o;
    fmmbem_default_solve_opts(&o);
    if (opts) o = *opts;
    if (int e = check_solve_opts(ctx, o)) return e;
    if (o.inner_iters > 0) return fail(ctx, FMMBEM_EINVAL, "the batched solve has no inner-outer scheme");
    if (o.precond == FMMBEM_PC_LEARNED) return fail(ctx, FMMBEM_EINVAL, "the batched solve has no learned guard");
    if (indirect(ctx) || burton_miller(ctx) || dpsi(ctx))
        return fail(ctx, FMMBEM_EINVAL, "the batched solve is for the direct formulation (Eq. dbem4)");
    GUARD_BEGIN
    HIP_OK(hipSetDevice(ctx->device));
    if (ctx->src.empty()) return fail(ctx, FMMBEM_ENOTREADY, "sources not set");
    for (int s = 0; s < ns; ++s)
        if (isrc[s] < 0 || isrc[s] >= (int)(ctx->src.size() / 3)) return fail(ctx, FMMBEM_EINVAL, "bad source index");
    double t_before = 0;
    bool dirty = ctx->mesh_dirty || ctx->k_dirty || ctx->beta_dirty;
    ensure_setup(ctx);
    if (dirty) t_before = ctx->t_setup_last;
    auto t0 = std::chrono::steady_clock::now();
    hipStream_t st = ctx->stream;
    const int64_t n = ctx->nt;
    auto pc = make_precond(ctx, o);
    double2 *B = dget<double2>(ctx->scratch, "sb_b", (size_t)ns * n);
    double2 *X = dget<double2>(ctx->scratch, "sb_x", (size_t)ns * n);
    for (int s = 0; s < ns; ++s) rhs_dev(ctx, isrc[s], B + (int64_t)s * n);
    if (o.use_x0) HIP_OK(hipMemcpyAsync(X, x, sizeof(double2) * n * ns, hipMemcpyHostToDevice, st));
    const bool mixed = o.precision == FMMBEM_MIXED;
    int64_t n64 = 0, nmx = 0;
    auto mv = [&](int nr, const double2 *a, double2 *y) {
        matvec_dev(ctx, nr, a, y, false, mixed);
        (mixed ? nmx : n64) += nr;
    };
    auto mv64 = [&](int nr, const double2 *a, double2 *y) {
        matvec_dev(ctx, nr, a, y, false, false);
        n64 += nr;
    };
    std::vector<int> iters, restarts, status;
    std::vector<double> rel;
    const bool b32 = o.basis_fp32 < 0 ? mixed : o.basis_fp32 != 0;
    int rc = fgmres_batch(n, st, ctx->scratch, ns, mv, mv64, pc, B, X, o.tol, o.restart, o.maxit, o.use_x0 != 0,
                          iters, restarts, rel, status, b32, o.reorth);
    HIP_OK(hipMemcpyAsync(x, X, sizeof(double2) * n * ns, hipMemcpyDeviceToHost, st));
    HIP_OK(hipStreamSynchronize(st));
    const double ts = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    int worst = FMMBEM_OK;
    for (int s = 0; s < ns; ++s) {
        if (rep) {
            rep[s].iters = iters[s];
            rep[s].restarts = restarts[s];
            rep[s].rel_res = rel[s];
            rep[s].t_setup_s = t_before;
            rep[s].t_solve_s = ts;  // wall time of the whole batch
            rep[s].status = status[s];
            rep[s].matvecs_fp64 = n64;  // products of the whole batch
            rep[s].matvecs_mixed = nmx;
            rep[s].inner_iters = 0;
            rep[s].pc_fallback_at = -1;
        }
        if (status[s] < 0) worst = status[s];
        else if (status[s] != FMMBEM_OK && worst == FMMBEM_OK) worst = status[s];
    }
    if (rc < 0) return fail(ctx, rc, "batched solver failed");
    if (worst < 0) ctx->err = "solver failed";
    return worst;
    GUARD_END
}

// ------------------------------------------------------------------ learned preconditioner
void fmmbem_default_train_opts(fmmbem_train_opts *o) {
    o->restart = 8;
    o->max_pairs = 12;
    o->tol = 1e-7;
    o->maxit = 400;
    o->epochs = 60;
    o->batch = 2048;
    o->lr = 1e-3;
    o->seed = 1;
}

int64_t fmmbem_mlp_param_count(void) { return mlp_param_count(); }

int fmmbem_mlp_init(fmmbem_ctx *ctx, uint64_t seed) {
    if (!ctx) return FMMBEM_EINVAL;
    GUARD_BEGIN
    HIP_OK(hipSetDevice(ctx->device));
    ctx->mlp.init(ctx->buf, seed, ctx->stream);
    HIP_OK(hipStreamSynchronize(ctx->stream));
    return FMMBEM_OK;
    GUARD_END
}

int fmmbem_mlp_get_weights(fmmbem_ctx *ctx, float *w) {
    if (!ctx || !w) return FMMBEM_EINVAL;
    if (!ctx->mlp.ready) return fail(ctx, FMMBEM_ENOTREADY, "network not initialised");
    GUARD_BEGIN
    HIP_OK(hipSetDevice(ctx->device));
    HIP_OK(hipMemcpyAsync(w, ctx->mlp.w32, sizeof(float) * mlp_param_count(), hipMemcpyDeviceToHost, ctx->stream));
    HIP_OK(hipStreamSynchronize(ctx->stream));
    return FMMBEM_OK;
    GUARD_END
}

int fmmbem_mlp_set_weights(fmmbem_ctx *ctx, const float *w) {
    if (!ctx || !w) return FMMBEM_EINVAL;
    GUARD_BEGIN
    HIP_OK(hipSetDevice(ctx->device));
    if (!ctx->mlp.ready) ctx->mlp.init(ctx->buf, 1, ctx->stream);
    HIP_OK(hipMemcpyAsync(ctx->mlp.w32, w, sizeof(float) * mlp_param_count(), hipMemcpyHostToDevice, ctx->stream));
    ctx->mlp.sync_half(ctx->stream);
    HIP_OK(hipStreamSynchronize(ctx->stream));
    return FMMBEM_OK;
    GUARD_END
}

static void mlp_upload_batch(fmmbem_ctx *ctx, int64_t m, const float *X, const float *T, float **Xd, float **Td,
                             float *A[4]) {
    hipStream_t st = ctx->stream;
    *Xd = dget<float>(ctx->scratch, "mlpt_X", (size_t)m * MLP_IN);
    HIP_OK(hipMemcpyAsync(*Xd, X, sizeof(float) * m * MLP_IN, hipMemcpyHostToDevice, st));
    if (T) {
        *Td = dget<float>(ctx->scratch, "mlpt_T", (size_t)m * MLP_OUT);
        HIP_OK(hipMemcpyAsync(*Td, T, sizeof(float) * m * MLP_OUT, hipMemcpyHostToDevice, st));
    }
    for (int l = 0; l < 4; ++l) A[l] = dget<float>(ctx->scratch, "mlpt_A" + std::to_string(l), (size_t)m * MLP_H);
}

int fmmbem_mlp_forward(fmmbem_ctx *ctx, int64_t m, const float *X, float *Y) {
    if (!ctx || !X || !Y || m < 1) return FMMBEM_EINVAL;
    if (!ctx->mlp.ready) return fail(ctx, FMMBEM_ENOTREADY, "network not initialised");
    GUARD_BEGIN
    HIP_OK(hipSetDevice(ctx->device));
    float *Xd, *A[4];
    mlp_upload_batch(ctx, m, X, nullptr, &Xd, nullptr, A);
    ctx->mlp.forward(m, Xd, A, ctx->stream);
    HIP_OK(hipMemcpyAsync(Y, A[3], sizeof(float) * m * MLP_OUT, hipMemcpyDeviceToHost, ctx->stream));
    HIP_OK(hipStreamSynchronize(ctx->stream));
    return FMMBEM_OK;
    GUARD_END
}

int fmmbem_mlp_loss_grad(fmmbem_ctx *ctx, int64_t m, const float *X, const float *T, float *loss, float *grad) {
    if (!ctx || !X || !T || !loss || !grad || m < 1) return FMMBEM_EINVAL;
    if (!ctx->mlp.ready) return fail(ctx, FMMBEM_ENOTREADY, "network not initialised");
    GUARD_BEGIN
    HIP_OK(hipSetDevice(ctx->device));
    hipStream_t st = ctx->stream;
    float *Xd, *Td, *A[4];
    mlp_upload_batch(ctx, m, X, T, &Xd, &Td, A);
    float *g = dget<float>(ctx->scratch, "mlpt_g", mlp_param_count());
    float *ld = dget<float>(ctx->scratch, "mlpt_loss", 1);
    ctx->mlp.forward(m, Xd, A, st);
    ctx->mlp.backward(m, Xd, A, Td, g, ld, ctx->scratch, st);
    HIP_OK(hipMemcpyAsync(grad, g, sizeof(float) * mlp_param_count(), hipMemcpyDeviceToHost, st));
    HIP_OK(hipMemcpyAsync(loss, ld, sizeof(float), hipMemcpyDeviceToHost, st));
    HIP_OK(hipStreamSynchronize(st));
    return FMMBEM_OK;
    GUARD_END
}

int fmmbem_learned_train(fmmbem_ctx *ctx, int32_t isrc, const fmmbem_train_opts *opts, fmmbem_train_report *rep) {
    if (!ctx) return FMMBEM_EINVAL;
    fmmbem_train_opts o;
    fmmbem_default_train_opts(&o);
    if (opts) o = *opts;
    if (o.restart < 1 || o.max_pairs < 1 || o.maxit < 1 || !(o.tol > 0) || o.epochs < 0 || o.batch < 1 || !(o.lr > 0))
        return fail(ctx, FMMBEM_EINVAL, "bad training options");
    GUARD_BEGIN
    HIP_OK(hipSetDevice(ctx->device));
    if (ctx->src.empty()) return fail(ctx, FMMBEM_ENOTREADY, "sources not set");
    if (isrc < 0 || isrc >= (int)(ctx->src.size() / 3)) return fail(ctx, FMMBEM_EINVAL, "bad source index");
    if (indirect(ctx) || burton_miller(ctx) || dpsi(ctx))
        return fail(ctx, FMMBEM_EINVAL, "the learned preconditioner is for the direct formulation (Eq. dbem4)");
    ensure_setup(ctx);
    ensure_chunks(ctx);
    hipStream_t st = ctx->stream;
    const int64_t n = ctx->nt, nch = ctx->nchunk;
    auto t0 = std::chrono::steady_clock::now();
    // 1. the plain solver's restart iterates and residuals
    fmmbem_solve_opts so;
    fmmbem_default_solve_opts(&so);
    so.precond = FMMBEM_PC_NEARBLOCK;
    auto pc = make_precond(ctx, so);
    double2 *b = dget<double2>(ctx->scratch, "tr_b", n), *x = dget<double2>(ctx->scratch, "tr_x", n);
    double2 *XS = dget<double2>(ctx->scratch, "tr_xs", (size_t)o.max_pairs * n);
    double2 *RS = dget<double2>(ctx->scratch, "tr_rs", (size_t)o.max_pairs * n);
    rhs_dev(ctx, isrc, b);
    std::vector<double> prel;
    FgmresHooks hk;
    hk.on_restart = [&](const double2 *xk, const double2 *rk, double rel) {
        if ((int)prel.size() >= o.max_pairs) return;
        const size_t q = prel.size();
        HIP_OK(hipMemcpyAsync(XS + q * n, xk, sizeof(double2) * n, hipMemcpyDeviceToDevice, st));
        HIP_OK(hipMemcpyAsync(RS + q * n, rk, sizeof(double2) * n, hipMemcpyDeviceToDevice, st));
        prel.push_back(rel);
    };
    std::vector<double> hist;
    auto mv = [&](const double2 *a, double2 *y) { matvec_dev(ctx, 1, a, y, false, false); };
    int iters = 0, restarts = 0;
    double rel = 1.0;
    // short cycles give the pairs; the reference solution x* continues from the last of them
    // without restarts, to the requested accuracy
    const int pair_its = o.max_pairs * o.restart;
    fgmres(n, st, ctx->scratch, "tr_", mv, mv, pc, b, x, o.tol, o.restart, pair_its, false, true, &hist, iters,
           restarts, rel, &hk);
    ctx->mlp_ref_hist = hist;
    int iters2 = 0;
    if (rel >= o.tol) {
        std::vector<double> hist2;
        fgmres(n, st, ctx->scratch, "tr_", mv, mv, pc, b, x, o.tol, o.maxit, o.maxit, true, true, &hist2, iters2,
               restarts, rel, nullptr);
    }
    iters += iters2;
    ctx->scratch.release("tr_fg_V");  // the long solve's basis is not needed any more
    ctx->scratch.release("tr_fg_Z");
    // 2. samples: features of r_k, targets (x* - x_k - P_near r_k) / |r_k| per chunk; pairs whose
    // error is not resolved by x* (residual within 10x of x*'s) are left out
    std::vector<int> keep;
    for (size_t q = 0; q < prel.size(); ++q)
        if (prel[q] > 10.0 * rel) keep.push_back((int)q);
    if (keep.empty()) throw FmmError(FMMBEM_EINVAL, "no usable residual/error pairs (solve converged too early)");
    const int64_t M = (int64_t)keep.size() * nch;
    float *Xall = dget<float>(ctx->scratch, "tr_X", (size_t)M * MLP_IN);
    float *Tall = dget<float>(ctx->scratch, "tr_T", (size_t)M * MLP_OUT);
    double2 *e = dget<double2>(ctx->scratch, "tr_e", n), *z0 = dget<double2>(ctx->scratch, "tr_z0", n);
    float *sc = dget<float>(ctx->scratch, "tr_sc", nch);
    const int32_t *cs = (int32_t *)ctx->buf.find("ch_s"), *cn = (int32_t *)ctx->buf.find("ch_n");
    const int32_t *cl = (int32_t *)ctx->buf.find("ch_l"), *pm = (int32_t *)ctx->buf.find("perm");
    for (size_t q = 0; q < keep.size(); ++q) {
        const double2 *rk = RS + (size_t)keep[q] * n;
        vec_sub(n, x, XS + (size_t)keep[q] * n, e, st);
        pc(rk, z0);
        mlp_features(nch, cs, cn, cl, pm, rk, (double4 *)ctx->buf.find("en"), (double2 *)ctx->buf.find("beta"),
                     (double *)ctx->buf.find("leaf_ka"), Xall + q * nch * MLP_IN, sc, st);
        mlp_target(nch, cs, cn, pm, e, z0, sc, Tall + q * nch * MLP_OUT, st);
    }
    HIP_OK(hipStreamSynchronize(st));
    auto t1 = std::chrono::steady_clock::now();
    // mean squared target = loss of a zero correction
    double lz = 0.0;
    {
        std::vector<float> th((size_t)M * MLP_OUT);
        HIP_OK(hipMemcpy(th.data(), Tall, sizeof(float) * th.size(), hipMemcpyDeviceToHost));
        for (float v : th) lz += (double)v * v;
        lz /= (double)M;
    }
    // 3. Adam over shuffled mini-batches
    ctx->mlp.init(ctx->buf, o.seed, st);
    const int64_t B = std::min<int64_t>(o.batch, M);
    float *Xb = dget<float>(ctx->scratch, "tr_Xb", (size_t)B * MLP_IN), *Tb = dget<float>(ctx->scratch, "tr_Tb", (size_t)B * MLP_OUT);
    float *A[4];
    for (int l = 0; l < 4; ++l) A[l] = dget<float>(ctx->scratch, "tr_A" + std::to_string(l), (size_t)B * MLP_H);
    float *g = dget<float>(ctx->scratch, "tr_g", mlp_param_count()), *ld = dget<float>(ctx->scratch, "tr_loss", 1);
    int64_t *idx = dget<int64_t>(ctx->scratch, "tr_idx", M);
    std::vector<int64_t> perm_h(M);
    std::iota(perm_h.begin(), perm_h.end(), 0);
    uint64_t state = o.seed * 0x9E3779B97F4A7C15ull + 12345;
    auto next = [&]() {  // SplitMix64
        uint64_t z = (state += 0x9E3779B97F4A7C15ull);
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        return z ^ (z >> 31);
    };
    double lfirst = 0, llast = 0;
    for (int ep = 0; ep < o.epochs; ++ep) {
        for (int64_t i = M - 1; i > 0; --i) std::swap(perm_h[i], perm_h[next() % (uint64_t)(i + 1)]);
        h2d_now(idx, perm_h.data(), sizeof(int64_t) * M, st);  // perm_h is reshuffled next epoch
        double sum = 0;
        int nb = 0;
        for (int64_t s0 = 0; s0 + B <= M; s0 += B) {  // whole batches only
            gather_rows(B, MLP_IN, idx + s0, Xall, Xb, st);
            gather_rows(B, MLP_OUT, idx + s0, Tall, Tb, st);
            ctx->mlp.forward(B, Xb, A, st);
            ctx->mlp.backward(B, Xb, A, Tb, g, ld, ctx->scratch, st);
            ctx->mlp.adam_step(g, (float)o.lr, st);
            float lh = 0;
            HIP_OK(hipMemcpyAsync(&lh, ld, sizeof(float), hipMemcpyDeviceToHost, st));
            HIP_OK(hipStreamSynchronize(st));
            sum += lh;
            ++nb;
        }
        const double mean = nb ? sum / nb : 0.0;
        if (ep == 0) lfirst = mean;
        llast = mean;
    }
    HIP_OK(hipStreamSynchronize(st));
    auto t2 = std::chrono::steady_clock::now();
    if (rep) {
        rep->samples = M;
        rep->pairs = (int32_t)keep.size();
        rep->solve_iters = iters;
        rep->solve_rel_res = rel;
        rep->loss_zero = lz;
        rep->loss_first = lfirst;
        rep->loss_last = llast;
        rep->t_data_s = std::chrono::duration<double>(t1 - t0).count();
        rep->t_train_s = std::chrono::duration<double>(t2 - t1).count();
    }
    return FMMBEM_OK;
    GUARD_END
}

// Field at nr receivers (device points pts, nr x 3) from the surface unknown x (device, caller
// order) into psi (device), on stream st, with the two density arrays sigma, mu (n each) supplied
// by the caller of this helper (the context's workspace or a fixed device array).
static void eval_field_run(fmmbem_ctx *ctx, int isrc, int64_t nr, const double *pts, const double2 *x, double2 *psi,
                           double2 *sigma, double2 *mu, hipStream_t st) {
    const int64_t n = ctx->nt;
    const double *rs = &ctx->src[3 * isrc];
    const int form = indirect(ctx) ? 3 : dpsi(ctx) ? 1 : 0;
    const double2 *bm = (const double2 *)ctx->buf.find("beta");
    const double2 *bp = indirect(ctx) ? (const double2 *)ctx->buf.find("betap") : bm;
    k_field_dens<<<ceil_div(n, 256), 256, 0, st>>>(n, form, (int32_t *)ctx->buf.find("perm"), x,
                                                   (double4 *)ctx->buf.find("ec"), (double4 *)ctx->buf.find("en"), bm,
                                                   bp, ctx->k, rs[0], rs[1], rs[2], ctx->src_amp[isrc], sigma, mu);
    LAUNCH_OK();
    const double4 *ec = (double4 *)ctx->buf.find("ec"), *en = (double4 *)ctx->buf.find("en");
    const double *ev = (double *)ctx->buf.find("ev");
    // many points: FIELD_FQ per workgroup sharing element tiles in LDS, once there are about three
    // such workgroups per CU; fewer points: one workgroup per point
    if (nr >= (int64_t)FIELD_FQ * 768)
        k_field_tile<<<(unsigned)ceil_div(nr, FIELD_FQ), 256, 0, st>>>(n, nr, pts, ec, en, ev, sigma, mu, ctx->k,
                                                                      ctx->rc * ctx->rc, rs[0], rs[1], rs[2],
                                                                      ctx->src_amp[isrc], psi);
    else
        k_field<<<(unsigned)nr, 256, 0, st>>>(n, pts, ec, en, ev, sigma, mu, ctx->k, ctx->rc * ctx->rc, rs[0], rs[1],
                                              rs[2], ctx->src_amp[isrc], psi);
    LAUNCH_OK();
}

// checks shared by the host and device variants; 0 or an error status
static int eval_field_prepare(fmmbem_ctx *ctx, int32_t isrc, int64_t nr) {
    if (ctx->src.empty()) return fail(ctx, FMMBEM_ENOTREADY, "sources not set");
    if (isrc < 0 || isrc >= (int)(ctx->src.size() / 3)) return fail(ctx, FMMBEM_EINVAL, "bad source index");
    if (nr > 0x7fffffff) return fail(ctx, FMMBEM_EINVAL, "at most 2^31 - 1 receivers per call");
    ensure_setup(ctx);
    if (dpsi(ctx)) check_dpsi_beta(ctx);
    return FMMBEM_OK;
}

int fmmbem_eval_field(fmmbem_ctx *ctx, int32_t isrc, int64_t nr, const double *r, const fmmbem_c64 *x, fmmbem_c64 *psi) {
    if (!ctx) return FMMBEM_EINVAL;
    if (!r || !x || !psi || nr < 0) return fail(ctx, FMMBEM_EINVAL, "bad arguments");
    GUARD_BEGIN
    HIP_OK(hipSetDevice(ctx->device));
    if (int e = eval_field_prepare(ctx, isrc, nr)) return e;
    if (nr == 0) return FMMBEM_OK;
    hipStream_t st = ctx->stream;
    const int64_t n = ctx->nt, nu = fmmbem_num_unknowns(ctx);
    double2 *dx = dget<double2>(ctx->scratch, "fe_x", nu);
    double *dp = dget<double>(ctx->scratch, "fe_pts", 3 * nr);
    double2 *dout = dget<double2>(ctx->scratch, "fe_out", nr);
    double2 *dsg = dget<double2>(ctx->scratch, "fe_sg", n), *dmu = dget<double2>(ctx->scratch, "fe_mu", n);
    h2d_now(dx, x, sizeof(double2) * nu, st);
    h2d_now(dp, r, sizeof(double) * 3 * nr, st);
    eval_field_run(ctx, isrc, nr, dp, dx, dout, dsg, dmu, st);
    HIP_OK(hipMemcpyAsync(psi, dout, sizeof(double2) * nr, hipMemcpyDeviceToHost, st));
    HIP_OK(hipStreamSynchronize(st));
    return FMMBEM_OK;
    GUARD_END
}

int fmmbem_eval_field_noalloc(fmmbem_ctx *ctx, int32_t isrc, int64_t nr, const void *r_dev, const void *x_dev,
                              void *psi_dev, void *stream) {
    if (!ctx) return FMMBEM_EINVAL;
    if (!r_dev || !x_dev || !psi_dev || nr < 0) return fail(ctx, FMMBEM_EINVAL, "bad arguments");
    if (nr > 0x7fffffff) return fail(ctx, FMMBEM_EINVAL, "at most 2^31 - 1 receivers per call");
    if (!ctx->have_mesh) return fail(ctx, FMMBEM_ENOTREADY, "mesh not set");
    if (ctx->nt > NOALLOC_MAX_N)
        return fail(ctx, FMMBEM_EINVAL, "fmmbem_eval_field_noalloc takes at most 1048576 elements (" +
                                            std::to_string(ctx->nt) + " given)");
    if (ctx->mesh_dirty || ctx->k_dirty || ctx->beta_dirty || !ctx->have_k)
        return fail(ctx, FMMBEM_ENOTREADY, "set up first (fmmbem_setup): this call builds nothing");
    if (ctx->src.empty()) return fail(ctx, FMMBEM_ENOTREADY, "sources not set");
    if (isrc < 0 || isrc >= (int)(ctx->src.size() / 3)) return fail(ctx, FMMBEM_EINVAL, "bad source index");
    GUARD_BEGIN
    if (dpsi(ctx)) check_dpsi_beta(ctx);
    if (nr == 0) return FMMBEM_OK;
    HIP_OK(hipSetDevice(ctx->device));
    double2 *ws = noalloc_scratch(ctx->device);
    if (!ws) return fail(ctx, FMMBEM_EDEVICE, "no fixed workspace on this device");
    hipStream_t caller = (hipStream_t)stream;
    ev_record(ctx, EV_CALLER_IN, caller);
    ev_wait(ctx, EV_CALLER_IN, ctx->stream);
    eval_field_run(ctx, isrc, nr, (const double *)r_dev, (const double2 *)x_dev, (double2 *)psi_dev, ws,
                   ws + NOALLOC_MAX_N, ctx->stream);
    ev_record(ctx, EV_CALLER_DONE, ctx->stream);
    ev_wait(ctx, EV_CALLER_DONE, caller);
    return FMMBEM_OK;
    GUARD_END
}

int fmmbem_eval_field_dev(fmmbem_ctx *ctx, int32_t isrc, int64_t nr, const void *r_dev, const void *x_dev,
                          void *psi_dev, void *stream) {
    if (!ctx) return FMMBEM_EINVAL;
    if (!r_dev || !x_dev || !psi_dev || nr < 0) return fail(ctx, FMMBEM_EINVAL, "bad arguments");
    GUARD_BEGIN
    HIP_OK(hipSetDevice(ctx->device));
    if (int e = eval_field_prepare(ctx, isrc, nr)) return e;
    if (nr == 0) return FMMBEM_OK;
    const int64_t n = ctx->nt;
    double2 *dsg = dget<double2>(ctx->scratch, "fe_sg", n), *dmu = dget<double2>(ctx->scratch, "fe_mu", n);
    hipStream_t caller = (hipStream_t)stream;
    ev_record(ctx, EV_CALLER_IN, caller);
    ev_wait(ctx, EV_CALLER_IN, ctx->stream);
    eval_field_run(ctx, isrc, nr, (const double *)r_dev, (const double2 *)x_dev, (double2 *)psi_dev, dsg, dmu,
                   ctx->stream);
    ev_record(ctx, EV_CALLER_DONE, ctx->stream);
    ev_wait(ctx, EV_CALLER_DONE, caller);
    return FMMBEM_OK;
    GUARD_END
}

int fmmbem_get_info(fmmbem_ctx *ctx, fmmbem_info *info) {
    if (!ctx || !info) return FMMBEM_EINVAL;
    GUARD_BEGIN
    HIP_OK(hipSetDevice(ctx->device));
    ensure_setup(ctx);
    std::memset(info, 0, sizeof(*info));
    const TreeHost &T = ctx->tree;
    info->n = ctx->nt;
    info->rc = ctx->rc;
    info->root_side = T.side;
    for (int d = 0; d < 3; ++d) info->root_lo[d] = T.lo[d];
    info->depth = T.depth;
    info->nleaf = (int64_t)T.leaf_start.size() - 1;
    info->leaf_max_occ = T.max_occ;
    info->near_nnz = ctx->near_nnz;
    info->p2p_pairs = ctx->p2p_pairs;
    auto rot = [](int p) {  // real flops of one rotation (per degree a real (2n+1)^2 matrix on a complex vector)
        double s = 0;
        for (int n = 0; n < p; ++n) s += 4.0 * (2.0 * n + 1) * (2.0 * n + 1);
        return s;
    };
    auto coax = [](int ps, int pt) {
        double s = 0;
        int pm = std::min(ps, pt);
        for (int m = -(pm - 1); m <= pm - 1; ++m) s += 8.0 * (pt - std::abs(m)) * (ps - std::abs(m));
        return s;
    };
    for (int l = 0; l <= T.depth && l < 24; ++l) {
        info->p[l] = l >= 2 ? ctx->lev[l].p : 0;
        info->nbox[l] = ctx->lev[l].nbox;
        info->m2l_pairs[l] = l >= 2 ? ctx->lev[l].njob_m2l : 0;
        if (l >= 2) {
            int p = ctx->lev[l].p;
            info->flops_m2l += (double)ctx->lev[l].njob_m2l * (2 * rot(p) + coax(p, p));
            if (l < T.depth) {
                int pc = ctx->lev[l + 1].p;
                info->flops_m2m_l2l += (double)ctx->lev[l + 1].nbox * 2 * (rot(pc) + rot(p) + coax(pc, p));
            }
        }
    }
    int pl = ctx->lev[T.depth].p;
    info->flops_p2m_l2p = (double)ctx->nt * (double)pl * pl * 2 * 8.0;
    info->bytes_p2p = (double)ctx->nt * (2 * 32 + 16 + 16 + 16) + (double)ctx->near_nnz * (4 + 32);
    info->lds_max = (int64_t)ctx->lds_max;
    return FMMBEM_OK;
    GUARD_END
}

int fmmbem_batch_shapes(fmmbem_ctx *ctx, int32_t max, fmmbem_batch_shape *out, int32_t *count) {
    if (!ctx || !count || (max > 0 && !out)) return FMMBEM_EINVAL;
    GUARD_BEGIN
    HIP_OK(hipSetDevice(ctx->device));
    ensure_setup(ctx);
    *count = (int32_t)ctx->shapes.size();
    for (int i = 0; i < max && i < *count; ++i) out[i] = ctx->shapes[i];
    return FMMBEM_OK;
    GUARD_END
}

int fmmbem_solve_many(int32_t count, fmmbem_ctx *const *ctxs, const int32_t *isrc, const fmmbem_solve_opts *opts,
                      fmmbem_c64 *const *x, fmmbem_solve_report *rep, int32_t *status, int32_t threads) {
    if (count < 0 || (count > 0 && (!ctxs || !isrc || !x || !rep || !status))) return FMMBEM_EINVAL;
    if (threads > 1) return FMMBEM_EINVAL;  // one host thread keeps every system in flight
    for (int32_t i = 0; i < count; ++i) {
        if (!ctxs[i] || !x[i]) return FMMBEM_EINVAL;
        status[i] = FMMBEM_OK;
    }
    if (count == 0) return FMMBEM_OK;
    // systems grouped by context, in order of first appearance; a group shares one set of options
    std::vector<fmmbem_ctx *> order;
    std::map<fmmbem_ctx *, std::vector<int>> members;
    for (int32_t i = 0; i < count; ++i) {
        if (!members.count(ctxs[i])) order.push_back(ctxs[i]);
        members[ctxs[i]].push_back(i);
    }
    std::vector<fmmbem_solve_opts> gopt(order.size());
    for (size_t q = 0; q < order.size(); ++q) {
        fmmbem_ctx *ctx = order[q];
        fmmbem_default_solve_opts(&gopt[q]);
        const std::vector<int> &mem = members[ctx];
        if (opts) gopt[q] = opts[mem[0]];
        for (int i : mem)
            if (opts && std::memcmp(&opts[i], &gopt[q], sizeof(fmmbem_solve_opts)) != 0) {
                status[i] = fail(ctx, FMMBEM_EINVAL, "systems of one context need the same solve options");
                return FMMBEM_EINVAL;
            }
        const fmmbem_solve_opts &o = gopt[q];
        if (int e = check_solve_opts(ctx, o)) {
            status[mem[0]] = e;
            return e;
        }
        if (o.inner_iters > 0 || o.precond == FMMBEM_PC_LEARNED) {
            status[mem[0]] = fail(ctx, FMMBEM_EINVAL, "fmmbem_solve_many has no inner-outer scheme and no learned guard");
            return FMMBEM_EINVAL;
        }
        if (ctx->src.empty()) {
            status[mem[0]] = fail(ctx, FMMBEM_ENOTREADY, "sources not set");
            return FMMBEM_ENOTREADY;
        }
        for (int i : mem)
            if (isrc[i] < 0 || isrc[i] >= (int)(ctx->src.size() / 3)) {
                status[i] = fail(ctx, FMMBEM_EINVAL, "bad source index");
                return FMMBEM_EINVAL;
            }
    }
    fmmbem_ctx *ctx = nullptr;  // the context a failure is reported on
    GUARD_BEGIN
    std::vector<double> t_setup(order.size(), 0.0);
    std::vector<FgmresGroup> groups(order.size());
    std::vector<int64_t> n64(order.size(), 0), nmx(order.size(), 0);
    std::vector<std::function<void(const double2 *, double2 *)>> pcs(order.size());
    for (size_t q = 0; q < order.size(); ++q) {
        ctx = order[q];
        HIP_OK(hipSetDevice(ctx->device));
        const bool dirty = ctx->mesh_dirty || ctx->k_dirty || ctx->beta_dirty;
        ensure_setup(ctx);
        if (dirty) t_setup[q] = ctx->t_setup_last;
    }
    const auto t0 = std::chrono::steady_clock::now();
    for (size_t q = 0; q < order.size(); ++q) {
        ctx = order[q];
        fmmbem_ctx *c = ctx;
        const fmmbem_solve_opts &o = gopt[q];
        const std::vector<int> &mem = members[ctx];
        const int nv = (int)mem.size();
        const int64_t n = fmmbem_num_unknowns(ctx);
        hipStream_t st = ctx->stream;
        FgmresGroup &G = groups[q];
        G.n = n;
        G.st = st;
        G.scr = &ctx->scratch;
        G.tag = "many_";
        G.nv = nv;
        double2 *B = dget<double2>(ctx->scratch, "mb_b", (size_t)nv * n);
        double2 *X = dget<double2>(ctx->scratch, "mb_x", (size_t)nv * n);
        if (dpsi(ctx)) check_dpsi_beta(ctx);
        for (int s = 0; s < nv; ++s) {
            rhs_one(ctx, isrc[mem[s]], B + (int64_t)s * n);
            if (o.use_x0) h2d_now(X + (int64_t)s * n, x[mem[s]], sizeof(double2) * n, st);
        }
        const bool mixed = o.precision == FMMBEM_MIXED;
        const bool direct = !indirect(ctx) && !burton_miller(ctx) && !dpsi(ctx);
        int64_t *c64 = &n64[q], *cmx = &nmx[q];
        auto product = [c, direct, n](int nr, const double2 *a, double2 *y, bool mx) {
            if (direct) matvec_dev(c, nr, a, y, false, mx);
            else
                for (int r = 0; r < nr; ++r) apply_operator(c, a + (int64_t)r * n, y + (int64_t)r * n, mx);
        };
        G.matvec = [product, mixed, c64, cmx](int nr, const double2 *a, double2 *y) {
            product(nr, a, y, mixed);
            (mixed ? *cmx : *c64) += nr;
        };
        G.matvec_check = [product, c64](int nr, const double2 *a, double2 *y) {
            product(nr, a, y, false);
            *c64 += nr;
        };
        pcs[q] = make_precond(ctx, o);
        if (dpsi(ctx) && o.precond == FMMBEM_PC_NEARBLOCK) {
            // Eq. (dbem5): leaf blocks of Eq. (dbem4) under the similarity diag(beta), as in fmmbem_solve
            auto p4 = pcs[q];
            double2 *tmp = dget<double2>(ctx->scratch, "d5_pc", n);
            const int32_t *pm = (int32_t *)ctx->buf.find("perm");
            const double2 *be = (double2 *)ctx->buf.find("beta");
            pcs[q] = [=](const double2 *v, double2 *z) {
                k_scale_beta<<<ceil_div(n, 256), 256, 0, st>>>(n, pm, be, 1, v, tmp);
                LAUNCH_OK();
                p4(tmp, z);
                k_scale_beta<<<ceil_div(n, 256), 256, 0, st>>>(n, pm, be, 0, z, z);
                LAUNCH_OK();
            };
        }
        G.precond = pcs[q];
        G.B = B;
        G.X = X;
        G.tol = o.tol;
        G.m = o.restart;
        G.maxit = o.maxit;
        G.reorth = o.reorth;
        G.x0_given = o.use_x0 != 0;
        G.basis32 = o.basis_fp32 < 0 ? mixed : o.basis_fp32 != 0;
    }
    ctx = order[0];
    fgmres_groups(groups);
    const double ts = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    int worst = FMMBEM_OK;
    for (size_t q = 0; q < order.size(); ++q) {
        ctx = order[q];
        const std::vector<int> &mem = members[ctx];
        const int64_t n = fmmbem_num_unknowns(ctx);
        const double2 *X = groups[q].X;
        for (int s = 0; s < (int)mem.size(); ++s) {
            const int i = mem[s];
            HIP_OK(hipMemcpyAsync(x[i], X + (int64_t)s * n, sizeof(double2) * n, hipMemcpyDeviceToHost, ctx->stream));
            status[i] = groups[q].status[s];
            rep[i].iters = groups[q].iters[s];
            rep[i].restarts = groups[q].restarts[s];
            rep[i].rel_res = groups[q].rel_res[s];
            rep[i].t_setup_s = t_setup[q];
            rep[i].t_solve_s = ts;  // wall time of the whole call
            rep[i].status = status[i];
            rep[i].matvecs_fp64 = n64[q];  // products of the system's context
            rep[i].matvecs_mixed = nmx[q];
            rep[i].inner_iters = 0;
            rep[i].pc_fallback_at = -1;
            rep[i].matvecs_coarse = 0;
            if (status[i] < 0) worst = status[i];
            else if (status[i] == FMMBEM_ENOCONV && worst == FMMBEM_OK) worst = FMMBEM_ENOCONV;
        }
        HIP_OK(hipStreamSynchronize(ctx->stream));
    }
    return worst;
    GUARD_END
}

int fmmbem_set_batch_shapes(fmmbem_ctx *ctx, int32_t count, const fmmbem_batch_shape *shapes) {
    if (!ctx || count < 0 || (count > 0 && !shapes)) return FMMBEM_EINVAL;
    GUARD_BEGIN
    HIP_OK(hipSetDevice(ctx->device));
    ensure_setup(ctx);
    std::vector<BatchRef> refs = all_batches(ctx);
    const size_t cap = ctx->lds_max - 1024;
    std::vector<std::pair<size_t, int32_t>> todo;  // (batch, shape index)
    for (int32_t i = 0; i < count; ++i) {
        const fmmbem_batch_shape &sh = shapes[i];
        size_t q = 0;
        while (q < refs.size() && !(refs[q].level == sh.level && refs[q].kind == sh.kind)) ++q;
        if (q == refs.size())
            return fail(ctx, FMMBEM_EINVAL, "no translation batch at level " + std::to_string(sh.level) + ", kind " +
                                                std::to_string(sh.kind));
        const TransBatch &b = *refs[q].b;
        bool ok;
        if (sh.lane)
            ok = sh.whole == 0 &&
                 ((sh.jt == 64 && (sh.mfma == 0 || sh.mfma == 1 || (sh.mfma == 2 && fused_ok(b)) ||
                                   ((sh.mfma == 3 || sh.mfma == 4) && rcr_ok(b)))) ||
                  (sh.jt == 32 && sh.mfma == 1));
        else
            ok = sh.mfma == 0 && (sh.whole == 0 || sh.whole == 1) && sh.jt >= 4 && sh.jt <= 64 && sh.jt % 4 == 0 &&
                 trans_lds_bytes(sh.jt, b.P, sh.whole) <= cap;
        if (!ok)
            return fail(ctx, FMMBEM_EINVAL, "shape does not fit the batch at level " + std::to_string(sh.level) +
                                                ", kind " + std::to_string(sh.kind));
        todo.push_back({q, i});
    }
    for (auto &t : todo) {
        const BatchRef &r = refs[t.first];
        const fmmbem_batch_shape &sh = shapes[t.second];
        TransBatch &b = *r.b;
        b.lane = sh.lane;
        b.whole = sh.whole;
        b.JT = sh.jt;
        b.mfma = sh.mfma;
        layout_batch(ctx, r.name, ctx->batch_jobs[r.name], b);
        for (auto &cs : ctx->shapes)
            if (cs.level == r.level && cs.kind == r.kind) {
                cs.lane = b.lane;
                cs.whole = b.whole;
                cs.jt = b.JT;
                cs.mfma = b.mfma;
                cs.ms = 0.0;
            }
    }
    drop_graphs(ctx);
    HIP_OK(hipStreamSynchronize(ctx->stream));
    return FMMBEM_OK;
    GUARD_END
}

int fmmbem_near_entries_n(fmmbem_ctx *ctx, int64_t *nnz, fmmbem_c64 *Lp, fmmbem_c64 *Mp) {
    if (!ctx || !nnz) return FMMBEM_EINVAL;
    GUARD_BEGIN
    HIP_OK(hipSetDevice(ctx->device));
    ensure_setup(ctx);
    *nnz = ctx->near_nnz;
    if (!Lp && !Mp) return FMMBEM_OK;
    ensure_indirect(ctx);
    const int64_t z = ctx->near_nnz;
    std::vector<double2> l(z), m(z);
    hipStream_t st = ctx->stream;
    HIP_OK(hipMemcpyAsync(l.data(), ctx->buf.find("near_Lp"), 16 * z, hipMemcpyDeviceToHost, st));
    HIP_OK(hipMemcpyAsync(m.data(), ctx->buf.find("near_Mp"), 16 * z, hipMemcpyDeviceToHost, st));
    HIP_OK(hipStreamSynchronize(st));
    for (int64_t e = 0; e < z; ++e) {
        if (Lp) Lp[e] = {l[e].x, l[e].y};
        if (Mp) Mp[e] = {m[e].x, m[e].y};
    }
    return FMMBEM_OK;
    GUARD_END
}

int fmmbem_near_entries(fmmbem_ctx *ctx, int64_t *nnz, int64_t *rows, int64_t *cols, fmmbem_c64 *L, fmmbem_c64 *M) {
    if (!ctx || !nnz) return FMMBEM_EINVAL;
    GUARD_BEGIN
    HIP_OK(hipSetDevice(ctx->device));
    ensure_setup(ctx);
    *nnz = ctx->near_nnz;
    if (!rows) return FMMBEM_OK;
    const int64_t z = ctx->near_nnz;
    std::vector<int32_t> r(z), c(z);
    std::vector<double2> l(z), m(z);
    hipStream_t st = ctx->stream;
    HIP_OK(hipMemcpyAsync(r.data(), ctx->buf.find("near_row"), 4 * z, hipMemcpyDeviceToHost, st));
    HIP_OK(hipMemcpyAsync(c.data(), ctx->buf.find("near_col"), 4 * z, hipMemcpyDeviceToHost, st));
    HIP_OK(hipMemcpyAsync(l.data(), ctx->buf.find("near_L"), 16 * z, hipMemcpyDeviceToHost, st));
    HIP_OK(hipMemcpyAsync(m.data(), ctx->buf.find("near_M"), 16 * z, hipMemcpyDeviceToHost, st));
    HIP_OK(hipStreamSynchronize(st));
    for (int64_t e = 0; e < z; ++e) {
        rows[e] = ctx->tree.perm[r[e]];
        cols[e] = ctx->tree.perm[c[e]];
        if (L) L[e] = {l[e].x, l[e].y};
        if (M) M[e] = {m[e].x, m[e].y};
    }
    return FMMBEM_OK;
    GUARD_END
}

int fmmbem_coaxial_table(int hip_device, int kind, double ktau, int p, int method, fmmbem_c64 *out) {
    if (!out || p < 1 || p > 1000 || !(ktau > 0) || (kind != 0 && kind != 1)) return FMMBEM_EINVAL;
    fmmbem_ctx *ctx = nullptr;
    try {
        HIP_OK(hipSetDevice(hip_device));
        DeviceBuffers scratch;
        double2 *d = dget<double2>(scratch, "out", coax_table_size(p));
        int meth = method < 0 ? (ktau < 1.0 ? 0 : 1) : method;
        std::vector<CoaxJob> jobs{{kind, meth, p, ktau, d}};
        build_coax_tables(jobs, scratch, nullptr);
        HIP_OK(hipMemcpy(out, d, sizeof(double2) * coax_table_size(p), hipMemcpyDeviceToHost));
        scratch.release_all();
        return FMMBEM_OK;
    } catch (const FmmError &e) {
        return e.code;
    }
    (void)ctx;
}

int fmmbem_rotation_table(int hip_device, int p, double *out) {
    if (!out || p < 1 || p > 2000) return FMMBEM_EINVAL;
    try {
        HIP_OK(hipSetDevice(hip_device));
        DeviceBuffers scratch;
        double *D = dget<double>(scratch, "D", rot_table_size(p)), *DT = dget<double>(scratch, "DT", rot_table_size(p));
        build_delta_table(p, D, DT, nullptr);
        HIP_OK(hipMemcpy(out, D, sizeof(double) * rot_table_size(p), hipMemcpyDeviceToHost));
        scratch.release_all();
        return FMMBEM_OK;
    } catch (const FmmError &e) {
        return e.code;
    }
}

}  // extern "C"
