/*
 * fmmbem -- fast-multipole boundary-element Helmholtz solver for room acoustics on one MI355X.
 *
 * C ABI.  The calls follow the statement of the problem in Section 2 of Gumerov & Duraiswami,
 * "Fast multipole accelerated boundary element methods for room acoustics":
 *   - a room surface S of flat triangles whose normals point out of the fluid (Section 2),
 *   - a wavenumber k = omega / c (Eq. sp2),
 *   - a locally reacting wall with specific impedance zeta (Eq. sp3), passed as the
 *     admittance beta = 1/zeta so that a rigid wall is beta = 0 (Eq. sp5),
 *   - unit monopole sources psi_in = G_k(r, r_s) (Eq. sp6),
 * and the direct boundary integral equation for the scattered field (Eq. dbem4),
 *   (A x)_i = 1/2 x_i + sum_j M_ij x_j - i k sum_j L_ij beta_j x_j ,   b = L gamma ,
 *   gamma = -(dpsi_in/dn) + i k beta psi_in                         (Eq. sp7, k/(i zeta) = -i k beta),
 * discretised with constant elements collocated at triangle centroids.  L and M are the single-
 * and double-layer operators of Eq. (dbem2).  Entries of element pairs closer than the cutoff
 * r_c are integrated accurately, the others by the one-point rule, and the far part of the
 * product is evaluated by the fast multipole method of Section 3.3 (octree, multipole and local
 * spherical expansions of Eq. shft0, rotation-coaxial-rotation translations with the stabilised
 * coaxial recursion of Section 3.3.1), as the matrix-vector product inside flexible GMRES.
 *
 * Conventions
 *   - Every call returns an int status (FMMBEM_OK = 0, negative = error) and, on error, sets a
 *     per-context message readable with fmmbem_last_error().  Nothing aborts or throws across
 *     the ABI.
 *   - Host-array inputs are copied at the call; the caller keeps ownership.  Outputs go into
 *     caller-allocated buffers of the documented size.  The context owns all device memory.
 *   - Complex numbers are fmmbem_c64 {re, im} (same layout as C99 double _Complex).
 *   - Vectors of unknowns are in the caller's triangle order.
 *   - *_dev calls take device pointers (e.g. from torch tensors) and a hipStream_t passed as
 *     void*; they enqueue on that stream and return when the work is enqueued or finished as
 *     documented per call.
 *   - One context per host thread; calls on one context are not thread-safe.
 *   - Units are SI (m, 1/m).
 */
#ifndef FMMBEM_H
#define FMMBEM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fmmbem_ctx fmmbem_ctx;
typedef struct {
    double re, im;
} fmmbem_c64;

enum {
    FMMBEM_OK = 0,
    FMMBEM_ENOCONV = 1,     /* solve hit maxit: x is valid but not converged */
    FMMBEM_EINVAL = -1,     /* bad argument (message says which) */
    FMMBEM_ENOMEM = -2,     /* device allocation failed */
    FMMBEM_EDEVICE = -3,    /* HIP runtime error */
    FMMBEM_ENOTREADY = -4,  /* required input not set yet */
    FMMBEM_EBREAKDOWN = -5, /* Krylov breakdown that is not a solution */
    FMMBEM_ENAN = -6        /* non-finite value met in the solver */
};

/* formulations (Section 3.1 / 3.2) */
enum {
    FMMBEM_DIRECT = 0,  /* Eq. dbem4: unknown psi_sc at each element (N unknowns) */
    FMMBEM_DIRECT_DPSI = 1, /* Eq. dbem5: unknown dpsi_sc/dn at each element (N unknowns); needs
                               beta != 0 everywhere (zeta = 1/beta); fmmbem_eval_field takes this
                               unknown; preconditioners none, diagonal, leaf blocks; one vector per
                               pass.  Its operator is Eq. dbem4's similarity transform by
                               diag(beta), with slower FGMRES convergence for large zeta (Sec. 3.1) */
    FMMBEM_DIRECT_BM = 2, /* combined (Burton-Miller) direct equation: Eq. dbem3 plus alpha = i/k
                             times its normal derivative (Section 3.2 jump relations), the same
                             unknown and field as Eq. dbem4; adds the near entries of L' and M';
                             preconditioners FMMBEM_PC_NONE, FMMBEM_PC_DIAG or FMMBEM_PC_NEARBLOCK;
                             one vector per pass */
    FMMBEM_INDIRECT = 3 /* Eq. ibem5: every element two-sided, unknowns (psi-, psi+) = the field on
                           the side the normal leaves (the room) and on the side it points to
                           (2N unknowns, psi- block first); FP64 and MIXED products (MIXED: FP32
                           translations, FP64 near field) */
};

/* arithmetic of the matrix-vector product */
enum {
    FMMBEM_FP64 = 0,  /* every step in FP64 */
    FMMBEM_MIXED = 1  /* near field and translations in FP32 with FP32 accumulation; tables,
                         recursions and the Krylov algebra stay FP64 */
};

/* preconditioner slot of flexible GMRES (Section 4.3 names an inner FMM-GMRES and a diagonal one) */
enum {
    FMMBEM_PC_NONE = 0,
    FMMBEM_PC_DIAG = 1,       /* z_i = v_i / (A_ii + diag_shift) */
    FMMBEM_PC_NEARBLOCK = 2,  /* exact inverse of the operator restricted to each octree leaf */
    FMMBEM_PC_LEARNED = 3     /* NEARBLOCK plus a trained per-leaf MLP correction (fmmbem_learned_train),
                                 dropped for the rest of the solve when the residual falls behind the
                                 plain solver's (guard) */
};

/* construction options; pass NULL for defaults */
typedef struct {
    double rc_factor;    /* near cutoff r_c = rc_factor * sqrt(2 * mean triangle area); default 1.8 */
    double rc;           /* if > 0, absolute r_c in m (overrides rc_factor) */
    int leaf_max;        /* octree depth: smallest uniform depth whose non-empty leaves hold at most
                            leaf_max elements on average (subject to leaf side > r_c); default 64 */
    int p_min;           /* minimum truncation number p (expansion degrees n < p); default 16 */
    double p_excess;     /* truncation rule p_l = max(p_min, ceil(kd + p_excess kd^(1/3))), kd = k d_l with
                            d_l the box side at level l; default 4.2.  Larger p than the one-box-separated
                            translation supports (n + n' well above k|t|) amplifies round-off through the
                            growth of h_{n+n'}(k|t|), so p is not raised beyond what the accuracy needs. */
    double ktau_switch;  /* coaxial coefficients: original recursion if k*tau < ktau_switch,
                            stabilised recursion otherwise (Section 3.3.1); default 1.0 */
    int max_depth;       /* cap on the octree depth; default 12 */
    int lds_budget;      /* LDS bytes per workgroup for translation tiles (0 = 64 KiB); larger tiles
                            share tables more but leave fewer workgroups per compute unit */
    int graphs;          /* nonzero: products on device vectors (solves, fmmbem_matvec_dev) replay a
                            captured HIP graph per (vector count, precision) through staging
                            buffers; per-phase timings then report only the total.  default 1 */
    int autotune;        /* nonzero: at setup, time each translation batch under the candidate tile
                            shapes and keep the fastest (adds setup time); default 0 */
    int lane_tiles;      /* 1: translation batches whose table classes hold many jobs (padding to
                            64-job tiles wastes at most a fifth, or, for batches on matrix-core
                            tiles, padding to 32 at most doubles the jobs) run job tiles, tables
                            read as wave-uniform values; 2: every batch does; 0: LDS tile kernels
                            everywhere; default 1 */
    int streams;         /* 2: the upper levels' M2L and the L2L chain of a product run on a
                            second stream beside the M2M chain, the deep levels' M2L and the near
                            field; 1: one stream; default 2 */
    int mfma;            /* matrix-core tiles for the stages of job-tile batches (each
                            degree/order of a 64- or 32-job tile as a real GEMM on
                            v_mfma_f64_16x16x4f64, FP32: v_mfma_f32_16x16x4f32): 1 for batches with
                            p >= 24 under the fixed rule (32-job tiles where the classes are
                            small), and the autotuner measures them for every job-tile batch; 2
                            for every job-tile batch; 0 never; default 1 */
    int fused;           /* lane batches with p_src = p_tgt = p <= 16 may run all three stages in
                            one kernel on matrix cores: with the jobs' vectors resident in LDS
                            (any such p; at p = 16, 8 jobs' vectors of one right-hand side shared
                            by the wavefronts of a workgroup, fixed rule at p = 16), or,
                            for FP64 products of one vector at p = 16, resident in the registers
                            of the wavefront that transforms them.  1: under the fixed rule and
                            as autotuner candidates (timed in FP64), and in mixed-precision
                            products for every such lane batch (an LDS-resident kernel, faster
                            in FP32 wherever measured); 0 never; default 1 */
    double kd_leaf_min;  /* lower bound on k times the leaf side: the octree stops refining before
                            its leaves get smaller than kd_leaf_min / k, because at small k tau the
                            singular coaxial tables lose their small entries to round-off (the
                            product's error rises to 3e-4 at k d = 0.37 and to O(1) at 0.18 with
                            p = 16); low frequencies then take larger leaves and more near-field
                            pairs.  The depth follows k: a change of wavenumber that moves the bound
                            rebuilds the octree.  0 disables; default 0.75 */
} fmmbem_options;

void fmmbem_default_options(fmmbem_options *opt);

/* Create a context on HIP device `hip_device`.  *out receives the handle. */
int fmmbem_create(fmmbem_ctx **out, int hip_device, const fmmbem_options *opt);
int fmmbem_destroy(fmmbem_ctx *ctx);
const char *fmmbem_last_error(const fmmbem_ctx *ctx);

/* Surface mesh.  xyz: nv*3 vertex coordinates (m).  tri: nt*3 vertex indices, each triangle
 * ordered so that (v1-v0)x(v2-v0) points out of the fluid.  EINVAL on an index out of range, a
 * degenerate (zero-area) triangle, or a closed mesh whose enclosed volume sum_j A_j (c_j.n_j)/3
 * is not positive (inward normals).  There is no per-element two-sided mask: in the indirect
 * formulation (Eq. ibem5) every element carries both unknowns (psi-, psi+), a closed wall's outer
 * face taking the admittance beta_plus (by default the wall's own), a thin baffle being a
 * zero-thickness plate and an open doorway a hole (its elements left out of the mesh). */
int fmmbem_set_mesh(fmmbem_ctx *ctx, int64_t nv, const double *xyz, int64_t nt, const int64_t *tri);

/* Wavenumber k = 2 pi f / c > 0 (Eq. sp2).  EINVAL if not finite and positive. */
int fmmbem_set_wavenumber(fmmbem_ctx *ctx, double k);

/* Admittance beta = 1/zeta per triangle (Eq. sp3/sp4), nt values each; Re(beta) >= 0 and finite
 * (passive wall), else EINVAL naming the element.  beta = 0 is a rigid wall (Eq. sp5), beta = 1
 * absorbs normal incidence fully.  beta_minus is the admittance of the face the normal leaves (the
 * room side; the only one the direct formulations use); beta_plus that of the face it points to
 * (indirect formulation, Eq. ibem4-ibem5), NULL for the same material on both faces.  Both arrays
 * are copied; a later call replaces both. */
int fmmbem_set_admittance(fmmbem_ctx *ctx, const fmmbem_c64 *beta_minus, const fmmbem_c64 *beta_plus);

/* Unit monopole sources (Eq. sp6): ns positions rs (ns*3), optional complex amplitudes (NULL = 1). */
int fmmbem_set_sources(fmmbem_ctx *ctx, int32_t ns, const double *rs, const fmmbem_c64 *amp);

/* FMMBEM_DIRECT, FMMBEM_DIRECT_DPSI, FMMBEM_DIRECT_BM or FMMBEM_INDIRECT.  The indirect formulation adds the near entries of L'
 * and the hypersingular M' (Eq. ibem3; built on first use) and evaluates the normal derivative
 * of the far field at every element; preconditioners: FMMBEM_PC_NONE, FMMBEM_PC_DIAG (2x2
 * element blocks) or FMMBEM_PC_NEARBLOCK (the operator on each leaf's 2 n_b unknowns, inverted). */
int fmmbem_set_formulation(fmmbem_ctx *ctx, int formulation);

/* Build what is out of date: octree and interaction lists (mesh), translation and rotation
 * tables and near-field entries (k), preconditioner data.  Idempotent; matvec/solve call it. */
int fmmbem_setup(fmmbem_ctx *ctx);

/* Number of unknowns: N for the direct formulation, 2N for the indirect one; -1 if no mesh.
 * Every vector argument below (x, y, b) has this length per right-hand side. */
int64_t fmmbem_num_unknowns(const fmmbem_ctx *ctx);

/* Right-hand side, one vector per source (b is ns x num_unknowns): b = L gamma (Eq. dbem4), or
 * for Eq. ibem5 (L[g- + g+], (g+ - g-)/2 + L'[g- + g+]) with g-+ = -+ dpsi_in/dn + i k beta-+ psi_in. */
int fmmbem_rhs(fmmbem_ctx *ctx, fmmbem_c64 *b);

/* Same into device memory: b_dev holds ns x num_unknowns fmmbem_c64 values (the caller's
 * allocation, e.g. a torch tensor).  The work runs on the library's stream after the work already
 * enqueued on `stream` (hipStream_t, NULL = the null stream), and `stream` is made to wait for
 * it; the call returns once everything is enqueued. */
int fmmbem_rhs_dev(fmmbem_ctx *ctx, void *b_dev, void *stream);

/* y = A x for nrhs vectors (x, y: nrhs*N, host memory).  precision: FMMBEM_FP64 / FMMBEM_MIXED
 * (direct: FP32 near-field kernel and translations; indirect: FP32 translations, FP64 near field;
 * both keep densities, P2M, L2P and the output FP64).
 * With `exact_far` != 0 the far field is summed pair by pair instead of by the FMM (all-pairs
 * O(N^2) product, for validation; FP64 only). */
int fmmbem_matvec(fmmbem_ctx *ctx, int32_t nrhs, const fmmbem_c64 *x, fmmbem_c64 *y, int precision, int exact_far);

/* Same on device pointers (nrhs*N fmmbem_c64 values each, caller-owned): the product runs on the
 * library's streams after the work already enqueued on `stream` (hipStream_t, NULL = the null
 * stream), and `stream` is made to wait for all of it, the copies into y_dev included, so work
 * enqueued on `stream` afterwards sees the finished y.  Returns after enqueueing; exact_far is not
 * offered here. */
int fmmbem_matvec_dev(fmmbem_ctx *ctx, int32_t nrhs, const void *x_dev, void *y_dev, int precision, void *stream);

typedef struct {
    double tol;        /* relative residual target ||b - A x|| / ||b||; default 1e-6 */
    int restart;       /* Krylov dimension m of FGMRES(m); default 30 */
    int maxit;         /* total iteration cap; default 500 */
    int precond;       /* FMMBEM_PC_*; default FMMBEM_PC_NEARBLOCK */
    int precision;     /* arithmetic of the inner products A z: FMMBEM_FP64 or FMMBEM_MIXED */
    double diag_shift; /* constant added to the diagonal in FMMBEM_PC_DIAG; default 0 */
    int use_x0;        /* nonzero: x holds the initial guess on entry */
    /* Inner-outer scheme (Section 4.3: flexible GMRES preconditioned by a low-accuracy FMM
     * GMRES).  inner_iters > 0: every outer preconditioner application runs up to inner_iters
     * GMRES steps (no restart) on A z = v with products in inner_precision, preconditioned by
     * `precond`, stopping early at relative residual inner_tol.  Default 0 (off), 1e-2, MIXED. */
    int inner_iters;
    double inner_tol;
    int inner_precision;
    /* Storage of the Krylov vectors (V and the preconditioned Z): 1 FP32 (half the basis traffic
     * of the Arnoldi steps; inner products, Hessenberg matrix, rotations, iterate and restart
     * residuals stay FP64), 0 FP64, -1 (default) FP32 exactly when the products are MIXED (for
     * the inner solves: when inner_precision is). */
    int basis_fp32;
    /* Coarser inner operator (Section 4.3: the inner GMRES uses a low-accuracy FMM).  inner_p_min
     * > 0 (with inner_iters > 0): the inner GMRES applies an FMM with the truncation rule's p_min
     * and excess replaced by inner_p_min and inner_p_excess, set up once on the same mesh,
     * wavenumber, admittance and formulation (its own tables and near-field entries, kept until
     * one of those changes); 0 (default): the inner GMRES applies the solve's own operator.
     * inner_p_excess defaults to 1.0; a negative inner_p_min, or a negative excess with
     * inner_p_min > 0, is FMMBEM_EINVAL.  The coarser context doubles the FMM's device memory. */
    int inner_p_min;
    double inner_p_excess;
    /* Classical Gram-Schmidt of the outer Arnoldi step (and of the batched solve): 0 one pass;
     * 1 (default) a second pass when the first left less than 1/sqrt(2) of the new vector's norm;
     * 2 always two passes.  Inner solves use 1. */
    int reorth;
} fmmbem_solve_opts;

typedef struct {
    int iters;            /* FGMRES iterations (= matrix-vector products after the first residual) */
    int restarts;
    double rel_res;       /* final relative residual measured with the FP64 FMM operator */
    double t_setup_s;     /* setup seconds spent inside this call (the coarser inner context's included) */
    double t_solve_s;     /* iteration seconds */
    int status;
    int64_t matvecs_fp64;  /* FMM products of the call, by arithmetic (outer, restart and inner) */
    int64_t matvecs_mixed;
    int64_t inner_iters;   /* total inner GMRES steps */
    int32_t pc_fallback_at; /* FMMBEM_PC_LEARNED: iteration at which the guard dropped the learned
                               correction, -1 if it acted throughout */
    int64_t matvecs_coarse; /* products of the coarser inner operator (inner_p_min > 0) */
} fmmbem_solve_report;

void fmmbem_default_solve_opts(fmmbem_solve_opts *o);

/* Solve A x = b for source `isrc` (b from fmmbem_rhs) by flexible GMRES (Section 4.3).
 * x: N values (in: initial guess if use_x0, out: solution).  Returns FMMBEM_OK on
 * convergence, FMMBEM_ENOCONV at maxit (x still the best iterate), or an error. */
int fmmbem_solve(fmmbem_ctx *ctx, int32_t isrc, const fmmbem_solve_opts *opts, fmmbem_c64 *x,
                 fmmbem_solve_report *rep);

/* Same with x in device memory (num_unknowns fmmbem_c64 values, caller-owned): the initial guess
 * (use_x0) is read after the work already enqueued on `stream` (hipStream_t, NULL = the null
 * stream), and `stream` is made to wait for the write of the solution.  The solve itself needs
 * host decisions at every iteration, so the call returns when it has finished. */
int fmmbem_solve_dev(fmmbem_ctx *ctx, int32_t isrc, const fmmbem_solve_opts *opts, void *x_dev,
                     fmmbem_solve_report *rep, void *stream);

/* Solve the systems of ns sources together (batching): isrc[s] names the source of system s;
 * x is ns*N (in: initial guesses if use_x0; out: solutions), rep has ns entries.  The systems
 * run FGMRES in lock step and every step applies one product to all systems still iterating
 * (kernel evaluations, expansions' basis functions and translation tables shared).  Each
 * system converges, restarts and stops on its own; rep[s].t_solve_s and the product counts
 * are those of the whole batch.  Returns FMMBEM_OK when every system converged, else the
 * first failure or FMMBEM_ENOCONV.  inner_iters must be 0. */
int fmmbem_solve_batch(fmmbem_ctx *ctx, int32_t ns, const int32_t *isrc, const fmmbem_solve_opts *opts,
                       fmmbem_c64 *x, fmmbem_solve_report *rep);

/* Solve many systems together from the calling thread (batching over frequencies, sources, rooms,
 * formulations): system i is source isrc[i] of context ctxs[i].  Systems of one context form a
 * group that runs flexible GMRES in lock step with one batched product per step (as
 * fmmbem_solve_batch; other formulations than Eq. dbem4 apply one product per system); the groups
 * -- contexts of other frequencies or rooms, each with its own mesh, N, octree depth and truncation
 * numbers -- advance in turn, each group's next product enqueued on its own streams as soon as its
 * Arnoldi step is done and each Arnoldi step waiting for its own group's stream only, so several
 * contexts' products are in flight on the device at once.  x[i] holds fmmbem_num_unknowns(ctxs[i])
 * values (in: initial guess if use_x0; out: solution); opts is NULL (defaults) or holds count
 * entries, equal for the systems of one context (else FMMBEM_EINVAL); inner_iters must be 0 and
 * precond not FMMBEM_PC_LEARNED.  rep[i] and status[i] receive each system's report and code;
 * rep[i].t_solve_s is the wall time of the whole call and the product counts are those of the
 * system's context.  threads must be 0 or 1 (EINVAL otherwise: one host thread keeps every system
 * in flight).  The result is FMMBEM_OK when all converged, FMMBEM_ENOCONV when some reached
 * maxit, else the first error.  An argument error returns before anything runs.  The contexts
 * must not be used by another host thread meanwhile. */
int fmmbem_solve_many(int32_t count, fmmbem_ctx *const *ctxs, const int32_t *isrc, const fmmbem_solve_opts *opts,
                      fmmbem_c64 *const *x, fmmbem_solve_report *rep, int32_t *status, int32_t threads);

/* ---- learned preconditioner ------------------------------------------------------------
 * A multilayer perceptron applied to every chunk of <= 64 consecutive unknowns of an octree
 * leaf: input 140 = the chunk's residual over its norm (64 complex, zero padded), k times the
 * leaf side, occupancy/64, mean and spread of the normals, mean admittance, a constant 1;
 * three ReLU layers of 128; output 128 = correction d (64 complex) added as |v_chunk| d to the
 * near-field block step.  Weights: FP16 in the forward pass, FP32 master copy, FP32
 * accumulation.  Parameter vector layout: per layer W (in x out, row-major) then b (out). */
typedef struct {
    int restart;      /* cycle length of the data-generating plain solve (max_pairs cycles): its
                         restart iterates x_k and residuals r_k give the pairs (r_k, x* - x_k);
                         default 8 */
    int max_pairs;    /* pairs kept (earliest first); default 12 */
    double tol;       /* accuracy of the reference solution x*, obtained by continuing from the
                         last cycle without restarts; pairs whose residual is not 10x above
                         x*'s are dropped; default 1e-7 */
    int maxit;        /* iteration cap of that continuation; default 400 */
    int epochs;       /* passes over the samples; default 60 */
    int batch;        /* samples per Adam step; default 2048 */
    double lr;        /* Adam step size; default 1e-3 */
    uint64_t seed;    /* weight initialisation and sample order; default 1 */
} fmmbem_train_opts;

typedef struct {
    int64_t samples;      /* chunks x pairs used */
    int32_t pairs;
    int32_t solve_iters;  /* iterations of the data-generating solves (cycles + continuation) */
    double solve_rel_res;
    double loss_zero;     /* mean squared target (loss of a zero correction) */
    double loss_first;    /* mean loss over the first epoch */
    double loss_last;     /* mean loss over the last epoch */
    double t_data_s, t_train_s;
} fmmbem_train_report;

void fmmbem_default_train_opts(fmmbem_train_opts *o);

/* Generate residual/error pairs with the plain near-field-block FGMRES on source isrc, then
 * train the network on them (Adam).  The trained weights stay in the context. */
int fmmbem_learned_train(fmmbem_ctx *ctx, int32_t isrc, const fmmbem_train_opts *opts, fmmbem_train_report *rep);

/* Direct access to the network for checks: parameter count, seeded initialisation, weights
 * (host float arrays of fmmbem_mlp_param_count()), forward pass Y = net(X) (X: m x 140,
 * Y: m x 128, host), and the mean squared error sum_i |net(X_i) - T_i|^2 / m with its
 * gradient (packed like the weights). */
int64_t fmmbem_mlp_param_count(void);
int fmmbem_mlp_init(fmmbem_ctx *ctx, uint64_t seed);
int fmmbem_mlp_get_weights(fmmbem_ctx *ctx, float *w);
int fmmbem_mlp_set_weights(fmmbem_ctx *ctx, const float *w);
int fmmbem_mlp_forward(fmmbem_ctx *ctx, int64_t m, const float *X, float *Y);
int fmmbem_mlp_loss_grad(fmmbem_ctx *ctx, int64_t m, const float *X, const float *T, float *loss, float *grad);

/* Free the per-call work arrays (Krylov bases, translation work rows, staging) now rather
 * than at fmmbem_destroy; they are allocated again when next needed.  Captured product graphs
 * are dropped with them, and so is the workspace of the coarser context that inner solves with
 * inner_p_min > 0 keep (its tables stay). */
int fmmbem_release_workspace(fmmbem_ctx *ctx);

/* Arnoldi estimate of the relative residual after each outer iteration of the last solve:
 * *count receives the number of iterations, est[0..min(max,count)) the values. */
int fmmbem_solve_history(fmmbem_ctx *ctx, int32_t max, double *est, int32_t *count);

/* Total field at nr points inside the room from the solved surface field x of source isrc
 * (Eq. dbem1): psi(r) = G(r, r_s) + L[gamma + i k beta x](r) - M[x](r); indirect (Eq. ibem1,
 * ibem4): psi = G(r, r_s) + L[sigma] + M[mu], sigma = g- + g+ + i k (beta- psi- + beta+ psi+),
 * mu = psi+ - psi-.  psi: nr values. */
int fmmbem_eval_field(fmmbem_ctx *ctx, int32_t isrc, int64_t nr, const double *r, const fmmbem_c64 *x,
                      fmmbem_c64 *psi);

/* Same on device memory: r_dev nr*3 doubles, x_dev num_unknowns and psi_dev nr fmmbem_c64 values
 * (caller-owned).  Runs on the library's stream after the work already enqueued on `stream`
 * (hipStream_t, NULL = the null stream), which is made to wait for it; returns after enqueueing.
 * nr < 2^31. */
int fmmbem_eval_field_dev(fmmbem_ctx *ctx, int32_t isrc, int64_t nr, const void *r_dev, const void *x_dev,
                          void *psi_dev, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): fmmbem_eval_field_dev with its two density arrays in a
 * fixed device array of the library (32 MiB, held by every device the library runs on until the
 * process ends) instead of the context's workspace.  It calls no hipMalloc, hipFree or other
 * allocating routine and builds nothing: the context must be set up already (fmmbem_setup, or any
 * earlier product, solve or field call, after the last setter), else FMMBEM_ENOTREADY.  At most
 * 1,048,576 elements (FMMBEM_EINVAL beyond).  Arguments, stream ordering and results are those of
 * fmmbem_eval_field_dev.  All calls on one device share the array: calls that overlap on one
 * device (two host threads, or streams not ordered with each other) race and give wrong fields. */
int fmmbem_eval_field_noalloc(fmmbem_ctx *ctx, int32_t isrc, int64_t nr, const void *r_dev, const void *x_dev,
                              void *psi_dev, void *stream);

/* ---- inspection (tests, benchmarks) ---------------------------------------------------- */

typedef struct {
    int64_t n;          /* unknowns */
    double rc;          /* near cutoff used (m) */
    double root_side;   /* bounding cube side D (m) */
    double root_lo[3];  /* bounding cube corner */
    int depth;          /* leaf level L (root = level 0) */
    int64_t nleaf;      /* non-empty leaves */
    int leaf_max_occ;   /* fullest leaf */
    int64_t near_nnz;   /* accurate near entries incl. self */
    int64_t p2p_pairs;  /* one-point-rule pairs evaluated per product by the near-field kernel */
    int p[24];          /* truncation number per level (0 where unused) */
    int64_t nbox[24];   /* boxes per level */
    int64_t m2l_pairs[24];
    double flops_m2l;   /* algorithmic flops of one product, per phase (FP64 real flops) */
    double flops_m2m_l2l;
    double flops_p2m_l2p;
    double bytes_p2p;   /* algorithmic HBM bytes of the near-field kernel per product */
    int64_t lds_max;    /* LDS bytes a workgroup may use on this device */
} fmmbem_info;

int fmmbem_get_info(fmmbem_ctx *ctx, fmmbem_info *info);

/* Accurate near entries (sorted by row, caller order): count via *nnz when rows == NULL. */
int fmmbem_near_entries(fmmbem_ctx *ctx, int64_t *nnz, int64_t *rows, int64_t *cols, fmmbem_c64 *L, fmmbem_c64 *M);

/* Tile shape of every translation batch (from the fixed rule, or measured when the options
 * ask for autotuning): level, kind 0 = M2L at that level, 1 = M2M into it, 2 = L2L out of it,
 * one-job-per-lane flag, whole-vector flag, jobs per tile, matrix-core mode of a lane batch (0
 * lane kernels, 1 matrix-core tiles stage by stage, 2 the fused LDS-resident kernel of 16 or 32
 * jobs per workgroup, 3 the fused kernel with each wavefront's 8 jobs' vectors in its registers
 * (FP64 products of one vector), 4 the fused kernel with 8 jobs' vectors in LDS shared by four
 * wavefronts, one right-hand side per workgroup; 3 and 4 apply at p = 16, products of several
 * vectors run mode 2 for mode 3, and FP32 products run mode 4 for mode 3), and the measured
 * FP64 time of the batch's four stages (0 when not measured). */
typedef struct {
    int32_t level, kind, lane, whole, jt, mfma;
    int64_t jobs;
    double ms;
} fmmbem_batch_shape;
int fmmbem_batch_shapes(fmmbem_ctx *ctx, int32_t max, fmmbem_batch_shape *out, int32_t *count);

/* Set the tile shape of translation batches, for instance to replay the shapes that
 * fmmbem_batch_shapes reported for the same mesh, wavenumber and options in an earlier run (the
 * autotuner's choice, so that a second process times or profiles exactly the same launches).
 * Each entry names its batch by (level, kind) and gives lane, whole, jt and mfma; jobs and ms are
 * ignored; batches not listed keep their shape.  Lane shapes need whole = 0 and jt = 64 (mfma 2
 * only where p_src = p_tgt <= 16, mfma 3 and 4 only where p_src = p_tgt = 16), or jt = 32 with
 * mfma = 1; LDS tiles need mfma = 0, jt a multiple of 4 in [4, 64] and
 * tiles that fit the LDS.  Every entry is checked before any is applied: an unknown batch or a
 * shape that does not fit returns FMMBEM_EINVAL and changes nothing.  Shapes hold until the
 * batches are rebuilt: a new mesh, or a wavenumber that changes the truncation number of the
 * batch's level or of the level below (a new wavenumber with the same truncation numbers keeps
 * each level's batches, shapes included). */
int fmmbem_set_batch_shapes(fmmbem_ctx *ctx, int32_t count, const fmmbem_batch_shape *shapes);

/* The L' and M' near entries (Eq. ibem3) in the order of fmmbem_near_entries (count via *nnz
 * when both arrays are NULL). */
int fmmbem_near_entries_n(fmmbem_ctx *ctx, int64_t *nnz, fmmbem_c64 *Lp, fmmbem_c64 *Mp);

/* Coaxial translation coefficients (Eq. shft0.1) computed on device `hip_device`:
 * kind 0 = (S|R), 1 = (R|R); method 0 = original recursion, 1 = stabilised, -1 = by the
 * ktau < 1 switch.  out: blocks m = 0..p-1, each (p-m)x(p-m) row-major (rows n' = m..p-1,
 * cols n = m..p-1), sum_m (p-m)^2 complex values. */
int fmmbem_coaxial_table(int hip_device, int kind, double ktau, int p, int method, fmmbem_c64 *out);

/* Real rotation matrices Delta^n = T^n(R_y(pi/2)) for n < p, where
 * Y_n^m(u) = sum_m' T^n_{mm'}(Q) Y_n^m'(Q u); block n is (2n+1)^2 row-major (rows m, cols m',
 * index + n), sum_n (2n+1)^2 doubles. */
int fmmbem_rotation_table(int hip_device, int p, double *out);

/* Kernel-level profiling.  When enabled, every kernel launch of the matrix-vector product is
 * bracketed by hipEvents on the library's stream and its algorithmic work (flops, HBM bytes,
 * counted from the problem sizes, not from hardware counters) is accumulated per kernel class. */
typedef struct {
    char name[32];
    int64_t launches;
    double ms;     /* summed device time of the launches */
    double flops;  /* summed algorithmic FP64/FP32 flops */
    double bytes;  /* summed algorithmic HBM bytes */
} fmmbem_kstat;

/* enable != 0: reset the statistics and start collecting; 0: stop. */
int fmmbem_profile(fmmbem_ctx *ctx, int enable);
/* Copy up to `max` kernel classes into out; *count receives the number of classes.  Waits for
 * the work enqueued so far. */
int fmmbem_kernel_stats(fmmbem_ctx *ctx, int max, fmmbem_kstat *out, int *count);

/* Per-phase device time of the last matvec in milliseconds (hipEvent based):
 * [0] densities, [1] P2P+near, [2] P2M, [3] M2M, [4] M2L, [5] L2L, [6] L2P+combine, [7] total.
 * The FMM product runs on two streams: the near field and the upper tree levels beside P2M and
 * the leaf-level translations, so the phases overlap: [1] and [2] both count from the fork after
 * [0], [3] is the M2M chain from the end of P2M, [4] the remaining translations up to the join
 * (M2L and L2L together; [5] is 0).  [7] is the wall time of the whole product. */
int fmmbem_last_timings(fmmbem_ctx *ctx, double *ms8);

#ifdef __cplusplus
}
#endif

#endif /* FMMBEM_H */
