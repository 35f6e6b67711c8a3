// Internal declarations of the fmmbem library (not part of the ABI).
#pragma once
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <map>
#include <string>
#include <vector>

#include <hip/hip_fp16.h>

#include <functional>

#include "../../include/fmmbem.h"
#include "common.h"
#include "specfun.h"

namespace fmm {

// ---------------------------------------------------------------- device memory
// Named, growable device allocations owned by a context.
struct DeviceBuffers {
    std::map<std::string, std::pair<void *, size_t>> bufs;
    uint64_t gen = 0;  // bumped whenever a buffer is freed (pointers held elsewhere may be stale)
    void *get(const std::string &name, size_t bytes) {
        if (bytes == 0) bytes = 16;
        auto it = bufs.find(name);
        if (it != bufs.end() && it->second.second >= bytes) return it->second.first;
        if (it != bufs.end()) {
            HIP_OK(hipFree(it->second.first));
            bufs.erase(it);
            ++gen;
        }
        void *p = nullptr;
        HIP_OK(hipMalloc(&p, bytes));
        bufs[name] = {p, bytes};
        return p;
    }
    void *find(const std::string &name) const {
        auto it = bufs.find(name);
        return it == bufs.end() ? nullptr : it->second.first;
    }
    void release(const std::string &name) {
        auto it = bufs.find(name);
        if (it != bufs.end()) {
            (void)hipFree(it->second.first);
            bufs.erase(it);
            ++gen;
        }
    }
    void release_all() {
        for (auto &kv : bufs) (void)hipFree(kv.second.first);
        bufs.clear();
        ++gen;
    }
};

template <class T>
T *dget(DeviceBuffers &b, const std::string &name, size_t count) {
    return (T *)b.get(name, sizeof(T) * count);
}

// Host-to-device copy from memory the host frees or rewrites right after (temporaries, buffers
// reused on the next step): an asynchronous copy from pageable memory may still read its source
// after the call returns, so wait for it.
inline void h2d_now(void *dst, const void *src, size_t bytes, hipStream_t st) {
    if (bytes == 0) return;
    HIP_OK(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, st));
    HIP_OK(hipStreamSynchronize(st));
}

// ---------------------------------------------------------------- tables
struct CoaxJob {
    int kind;    // 0 = (S|R), 1 = (R|R)
    int method;  // 0 = original (propagation in n), 1 = stabilised
    int p;
    double ktau;
    double2 *out;
};
int64_t coax_ws_size(int p);
void build_coax_tables(const std::vector<CoaxJob> &jobs, DeviceBuffers &scratch, hipStream_t st);
void build_delta_table(int p, double *D, double *DT, hipStream_t st);

// ---------------------------------------------------------------- octree (host)
// translation directions: 343 box offsets (dx,dy,dz) in [-3,3]^3, index (dx+3)*49+(dy+3)*7+(dz+3),
// then 8 child->parent unit diagonals (index 343 + octant) used by M2M (t = parent - child)
// and their negatives (index 351 + octant) used by L2L (t = child - parent).
constexpr int NDIR = 343 + 16;
inline int dir_of_offset(int dx, int dy, int dz) { return (dx + 3) * 49 + (dy + 3) * 7 + (dz + 3); }

struct LevelHost {
    int level;
    double side;                    // box side d_l
    int p;                          // truncation number
    std::vector<uint64_t> code;     // sorted Morton codes of the non-empty boxes
    std::vector<int32_t> parent;    // index at level-1 (levels >= 1)
    std::vector<int8_t> octant;     // child octant within the parent
    std::vector<int32_t> child_start, child_list;  // children at level+1 (CSR)
    // M2L interaction list, grouped by target box (CSR)
    std::vector<int32_t> m2l_start, m2l_src;
    std::vector<int16_t> m2l_dir;
    std::vector<int> m2l_tau_of_dir;  // size 343: index into the distinct |t| list, or -1
    std::vector<double> m2l_taus;     // distinct |t| (m)
};

struct TreeHost {
    double lo[3], side;  // bounding cube
    int depth;           // leaf level L
    std::vector<int32_t> perm;        // sorted position -> caller index
    std::vector<int32_t> leaf_start;  // CSR of sorted elements per leaf (level L box)
    std::vector<int32_t> nbr_start, nbr_list;  // P2P source leaves per target leaf
    std::vector<LevelHost> lv;        // index = level (0..L); levels < 2 hold no expansions
    int max_occ = 0;
};

void box_center(const TreeHost &T, int l, uint64_t code, double *c);
void build_tree(const double *centroids, int64_t n, const double *vlo, const double *vhi, double rc,
                int leaf_max, int max_depth, double min_leaf, TreeHost &T);

// ---------------------------------------------------------------- translation batches
// One set of translation jobs (a level's M2L, M2M or L2L), sorted by coaxial table and padded
// so that every tile of JT jobs shares one table (padding jobs have tgt = -1).
struct TransBatch {
    int64_t njob = 0, nreal = 0;
    int JT = 4, psrc = 0, ptgt = 0, P = 0, PT = 0;
    int32_t *src = nullptr, *tgt = nullptr;
    int16_t *dir = nullptr;
    int32_t *tile_coax = nullptr, *tile_rot = nullptr;  // tables per tile
    double *H = nullptr, *HT = nullptr;                 // rotation tables of the batch's polar angles
    int nbeta = 0;
    float *H32 = nullptr, *HT32 = nullptr;              // FP32 copies (mixed precision)
    int whole = 0;                                      // whole-vector tiles (small p) or per-degree slices
    int lane = 0;                                       // one job per lane, 64-job tiles (many jobs per class)
    int mfma = 0;                                       // lane batch on matrix cores: 1 stage by stage, 2 fused in LDS
                                                        // (p <= 16), 3 fused in registers, 4 fused with 8 jobs'
                                                        // vectors in LDS shared by 4 waves (p = 16)
    int64_t ntgt = 0;                                   // target boxes
    int32_t *tgt_start = nullptr, *tgt_jobs = nullptr;  // jobs of each target (CSR, padded job indices)
    // lane batches: consecutive jobs of one class with one target form a run (never crossing a
    // SEG_ALIGN-job boundary); seg[j] = run length at the run's first job, 0 elsewhere.  The back
    // rotation stores each run's sum in the first job's row and the CSR lists first jobs only.
    int8_t *seg = nullptr;
    int64_t nout = 0;  // rows the back rotation stores (runs of lane batches, else jobs)
    int64_t nsrc = 0;  // distinct source expansions the batch reads
    int ncoax = 1;     // coaxial tables the batch's classes use
    // fused tiles: the rotation tables and the batch's coaxial tables in the order in which the
    // lanes hold matrix-core fragments, zero past every block (built when p_src = p_tgt <= 16)
    double *frH = nullptr, *frHT = nullptr, *frC = nullptr;
    float *frH32 = nullptr, *frHT32 = nullptr, *frC32 = nullptr;
    int nfrc = 0;  // coaxial classes in frC
};
// runs of the back-rotation output never cross a multiple of this many (real) jobs, so that a
// run lies in one 32-lane half tile (the fused kernel's block) for 1, 2 or 4 right-hand sides
constexpr int SEG_ALIGN = 8;
// receivers per workgroup of the tiled field kernel (k_field_tile)
constexpr int FIELD_FQ = 8;
// one translation job before tiling
struct JobH {
    int32_t src, tgt;
    int16_t dir;
    int tab;  // coaxial table
    int rot;  // polar-angle class
};

int trans_pick_jt(int P, size_t lds_budget, int whole);
int trans_fused_pmax();
int trans_rcr_p();  // the truncation number of the register-resident fused tiles
// fragment-order tables of the fused tiles, per class: rotation 8 degree pairs x 2 degrees x
// 8 K chunks x 2 row blocks x 64 lanes; coaxial 16 orders x 4 K chunks x (re, im) x 64 lanes
constexpr int TF_FR_STEP = 2 * 8 * 2 * 64, TF_FR_ROT = 8 * TF_FR_STEP;
constexpr int TF_FR_ORDER = 4 * 2 * 64, TF_FR_COAX = 16 * TF_FR_ORDER;
void build_fused_tables(int P, int PT, int nbeta, const double *H, const double *HT, int ncoax, const double2 *coax,
                        double *frH, double *frHT, double *frC, hipStream_t st);
size_t trans_lds_bytes(int JT, int P, int whole);
void trans_configure_lds(size_t lds_max);
template <class R>
const char *trans_stage(const TransBatch &b, const TransTables<R> &tb, int stage, int nr, const typename Cx<R>::T *src,
                        typename Cx<R>::T *dst, const typename Cx<R>::T *ph, int PH, typename Cx<R>::T *W1,
                        typename Cx<R>::T *W2, hipStream_t st, bool accumulate = true);
void build_rot_tables(const std::vector<double> &betas, int P, const double *D, double *H, double *HT,
                      DeviceBuffers &scratch, hipStream_t st);

// ---------------------------------------------------------------- per-level device data
struct LevelDev {
    int p = 0;
    int64_t nbox = 0;
    double side = 0;
    double4 *center = nullptr;   // box centres
    double2 *M = nullptr;        // multipole coefficients nbox * p^2
    double2 *L = nullptr;        // local coefficients nbox * p^2
    // M2L jobs (target-grouped): src box, target box, direction, |t| table
    int64_t njob_m2l = 0;
    int32_t *m2l_tgt = nullptr, *m2l_src = nullptr, *m2l_start = nullptr;
    int16_t *m2l_dir = nullptr;
    int8_t *m2l_tau = nullptr;
    double2 *coax_m2l = nullptr;  // ntau tables of coax_table_size(p)
    int ntau = 0;
    double2 *coax_up = nullptr;   // (R|R) for the link to level+1 (square, size p)
    int32_t *parent = nullptr;    // parent index at level-1
    int8_t *octant = nullptr;
    int32_t *child_start = nullptr;  // children at level+1 (CSR), sorted so that child jobs group
    TransBatch m2l, up, down;        // M2L at this level; M2M from level+1 into this; L2L into level+1
    // FP32 copies for the mixed-precision product
    float2 *M32 = nullptr, *L32 = nullptr, *coax_m2l32 = nullptr, *coax_up32 = nullptr;
};

struct Timings {
    double ms[8] = {0};
};

// ------------------------------------------------------------------ learned preconditioner
constexpr int MLP_IN = 140, MLP_H = 128, MLP_OUT = 128;
struct Mlp {
    float *w32 = nullptr, *m1 = nullptr, *m2 = nullptr;  // master weights and Adam moments (packed)
    __half *w16 = nullptr;                                // FP16 copy (the backward pass)
    __half *w16t = nullptr;  // FP16 copy per layer transposed, out x in padded to 16 (matrix-core forward)
    int64_t step = 0;
    bool ready = false;
    void init(DeviceBuffers &buf, uint64_t seed, hipStream_t st);
    void sync_half(hipStream_t st);
    void forward(int64_t M, const float *X, float *const A[4], hipStream_t st) const;
    void backward(int64_t M, const float *X, float *const A[4], const float *T, float *grad, float *loss_dev,
                  DeviceBuffers &scr, hipStream_t st) const;
    void adam_step(const float *grad, float lr, hipStream_t st);
};
int64_t mlp_param_count();
void mlp_features(int64_t nchunk, const int32_t *cs, const int32_t *cn, const int32_t *cl, const int32_t *perm,
                  const double2 *v, const double4 *en, const double2 *beta, const double *leaf_ka, float *X,
                  float *scale, hipStream_t st);
void mlp_apply(int64_t nchunk, const int32_t *cs, const int32_t *cn, const int32_t *perm, const float *Y,
               const float *scale, double2 *z, hipStream_t st);
void mlp_target(int64_t nchunk, const int32_t *cs, const int32_t *cn, const int32_t *perm, const double2 *e,
                const double2 *z0, const float *scale, float *T, hipStream_t st);

void gather_rows(int64_t B, int width, const int64_t *idx, const float *src, float *dst, hipStream_t st);
void vec_sub(int64_t n, const double2 *a, const double2 *b, double2 *out, hipStream_t st);
void vec_add(int64_t n, const double2 *a, const double2 *b, double2 *out, hipStream_t st);

// one group of systems of the lock-step FGMRES (fgmres_groups): nv systems sharing an operator,
// their right-hand sides B and iterates X (nv x n, device), the products on stream st
struct FgmresGroup {
    int64_t n = 0;
    hipStream_t st = nullptr;
    DeviceBuffers *scr = nullptr;
    std::string tag;  // scratch-name prefix of the group's Krylov bases
    int nv = 0;
    std::function<void(int, const double2 *, double2 *)> matvec, matvec_check;
    std::function<void(const double2 *, double2 *)> precond;
    const double2 *B = nullptr;
    double2 *X = nullptr;
    double tol = 1e-6;
    int m = 30, maxit = 500, reorth = 1;
    bool x0_given = false, basis32 = false;
    std::vector<int> iters, restarts, status;  // per system (outputs)
    std::vector<double> rel_res;
};
void fgmres_groups(std::vector<FgmresGroup> &groups);

// optional observers of a flexible GMRES run
struct FgmresHooks {
    std::function<void(const double2 *x, const double2 *r, double rel)> on_restart;  // true residual
    std::function<void(int it, double est)> on_iter;                                  // Arnoldi estimate
};

}  // namespace fmm

// ---------------------------------------------------------------- the context
struct fmmbem_ctx {
    int device = 0;
    // coarser FMM for inner GMRES solves (same inputs, smaller truncation), owned; rebuilt when the
    // inputs change (input_gen counts the setters' calls)
    fmmbem_ctx *inner = nullptr;
    uint64_t input_gen = 0, inner_gen = ~0ULL;
    int inner_pmin = 0;
    double inner_pexc = 0.0;
    hipEvent_t xev[2] = {};
    double tree_min_leaf = 0.0;  // smallest leaf side the octree was allowed (kd_leaf_min / k at build)
    fmmbem_options opt{};
    std::string err;
    hipStream_t stream = nullptr;
    // second stream of the product (near field and the upper tree levels run beside the leaf
    // level), the stream the helpers currently enqueue on, and the fork/join events
    hipStream_t side = nullptr, cur = nullptr;
    std::vector<hipEvent_t> fj;
    hipEvent_t ev[9] = {};
    fmm::DeviceBuffers buf;      // persistent per-setup arrays
    fmm::DeviceBuffers scratch;  // per-call workspaces

    // inputs (host copies, caller order)
    std::vector<double> xyz;
    std::vector<int64_t> tri;
    int64_t nv = 0, nt = 0;
    double k = 0.0;
    std::vector<double2> beta;
    std::vector<double> src;
    std::vector<double2> src_amp;
    int formulation = FMMBEM_DIRECT;

    // dirty flags
    bool mesh_dirty = true, k_dirty = true, beta_dirty = true;
    bool have_mesh = false, have_k = false, have_beta = false;

    // derived
    double rc = 0.0;
    fmm::TreeHost tree;
    std::vector<fmm::LevelDev> lev;
    // learned preconditioner: chunks of <= 64 unknowns per leaf, the network, its reference rate
    fmm::Mlp mlp;
    int64_t nchunk = 0;
    bool chunks_ready = false;
    std::vector<double> mlp_ref_hist;  // plain solver's residual estimates in the training run
    bool mlp_active = false;           // the guard still lets the learned correction act
    std::vector<std::vector<int32_t>> iota_h;  // per level: 0..nbox (one job per child)
    int pmax = 0, delta_p = 0;
    size_t lds_max = 65536;
    int64_t near_nnz = 0;
    int64_t p2p_pairs = 0;
    bool precond_ready_nb = false, precond_ready_diag = false;
    std::vector<double> history;  // Arnoldi residual estimate per outer iteration of the last solve
    bool mixed_ready = false;
    std::map<std::string, std::vector<fmm::JobH>> batch_jobs;  // sorted jobs per batch (re-layout)
    // truncation numbers (p_l, p_{l+1}) each level's batches were built with; cleared with the octree
    std::map<int, std::pair<int, int>> batch_p;
    std::vector<fmmbem_batch_shape> shapes;                      // tile shape chosen per batch
    std::vector<double2> beta_plus;  // admittance of the + faces (indirect formulation); empty: = beta
    bool indirect_ready = false;     // L' and M' near entries exist for the current (mesh, k)
    int nr_cap = 1, nr_cap32 = 0;  // vectors per box the FP64 / FP32 expansion arrays hold
    bool capturing = false;        // a graph capture is in progress: no allocation, no timing events
    struct GraphEntry {
        int nr;
        bool mixed;
        hipGraphExec_t exec;
        uint64_t gen_buf, gen_scr;
    };
    std::vector<GraphEntry> graphs;  // captured products (staging buffers g_x -> g_y)  // FP32 copies of the tables exist for the current wavenumber
    fmm::Timings last;
    double t_setup_last = 0.0;
    // kernel profiling (fmmbem_profile)
    bool prof_on = false;
    std::vector<hipEvent_t> prof_ev;
    int prof_used = 0;
    struct ProfRec {
        int cls, a, b;
        double flops, bytes;
    };
    std::vector<ProfRec> prof_pend;
    std::vector<fmmbem_kstat> prof_stats;
};
