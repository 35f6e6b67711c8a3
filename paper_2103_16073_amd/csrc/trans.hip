// Rotation - coaxial translation - back-rotation (Section 3.3) for tiles of translations.
//
// A translation job moves one expansion (multipole of a source box, or local of a parent) into
// another frame.  With t = |t| (sin b cos a, sin b sin a, cos b):
//   forward rotation   c'_n = H_n(b) (e^{i m a} c_n)          (t now along +z)
//   coaxial step       d'^m_{n'} = sum_n (E|F)^{|m|}_{n'n}(|t|) c'^m_n
//   back rotation      d_n = e^{-i m a} H_n(b)^T d'_n
// where H_n(b) is the real orthogonal rotation matrix of degree n for the polar angle b (tables
// per distinct b, see k_rot_tables in tables.hip).  Jobs are sorted so that every tile of JT jobs
// shares |t| and b: each table value read from memory then feeds the whole tile.
//
// Three launches per batch, each parallel over (tile, degree) or (tile, order):
//   k_tr_rot_fwd  gathers the sources, applies the phase and H      -> W1 (P^2 per job)
//   k_tr_coax     applies the coaxial block of each order m         -> W2
//   k_tr_rot_back applies H^T and the phase, accumulates into targets (FP64 atomics)
// Threads compute 4 jobs x 4 rows each, so one table read feeds 8 (rotation) or 16 (coaxial)
// fused multiply-adds; the tile's slice of the vectors sits in LDS.
#include <utility>

#include "internal.h"

namespace fmm {

// Scalar-generic complex helpers: the same kernels run in FP64 and in FP32 (mixed mode).
template <class C> __device__ inline C mkc(double r, double i) { C v; v.x = r; v.y = i; return v; }
template <class C> __device__ inline C mulc(C a, C b) { C v; v.x = a.x * b.x - a.y * b.y; v.y = a.x * b.y + a.y * b.x; return v; }
template <class C> __device__ inline C mulcc(C a, C b) { C v; v.x = a.x * b.x + a.y * b.y; v.y = a.y * b.x - a.x * b.y; return v; }
template <class C> __device__ inline C addc(C a, C b) { C v; v.x = a.x + b.x; v.y = a.y + b.y; return v; }

template <class R>
struct TransArgsT {
    using C = typename Cx<R>::T;
    int64_t njob;               // virtual jobs: real jobs x nr right-hand sides
    int JT, psrc, ptgt, P, PT, PH;
    int nr;                     // right-hand sides; virtual job J = real job J / nr, vector J % nr
    const C *src;               // source expansions (psrc^2 per box)
    C *dst;                     // target expansions (ptgt^2 per box), accumulated
    const int32_t *jsrc, *jtgt; // per job; jtgt < 0 marks padding
    const int16_t *jdir;
    const int32_t *tile_coax;   // coaxial table per tile
    const int32_t *tile_rot;    // rotation table per tile
    const C *coax;              // coaxial tables, coax_table_size(PT) each
    const R *H, *HT;            // rotation tables (rot_table_size(P) each) and their transposes
    const C *ph;                // e^{i m a} per direction, 2*PH+1 per direction
    C *W1, *W2;                 // work rows, P^2 per job
    const int8_t *jseg;         // lane batches: run length at the first job of a run, else 0
    const R *frH, *frHT, *frC;  // fused tiles: fragment-order tables (TF_FR_ROT, TF_FR_COAX per class)
};

constexpr int RJ = 4, RR = 4;

// source expansion row of virtual job J (sources hold nr vectors per box, vector-inner)
template <class R>
__device__ inline int64_t src_row(const TransArgsT<R> &a, int64_t J) {
    return (int64_t)a.jsrc[J / a.nr] * a.nr + J % a.nr;
}

// ------------------------------------------------------------------ forward rotation
template <class R>
__global__ void __launch_bounds__(256) k_tr_rot_fwd(TransArgsT<R> a) {
    using C = typename Cx<R>::T;
    extern __shared__ double2 lds_raw[];
    C *lds = (C *)lds_raw;
    const int n = blockIdx.y;
    if (n >= a.psrc) return;
    const int w = 2 * n + 1, JT = a.JT;
    C *xs = lds;  // JT x w
    const int64_t t0 = (int64_t)blockIdx.x * JT;
    const int nj = (int)min((int64_t)JT, a.njob - t0);
    const int ps2 = a.psrc * a.psrc, P2 = a.P * a.P, phs = 2 * a.PH + 1;
    for (int e = threadIdx.x; e < nj * w; e += blockDim.x) {
        const int j = e / w, q = e - j * w, m = q - n;
        const int64_t job = t0 + j;
        xs[j * w + q] = mulc(a.ph[(int64_t)a.jdir[job / a.nr] * phs + a.PH + m], a.src[src_row(a, job) * ps2 + n * n + q]);
    }
    __syncthreads();
    const R *HTn = a.HT + (int64_t)a.tile_rot[blockIdx.x / a.nr] * rot_table_size(a.P) + rot_block_off(n);
    const int ng = (nj + RJ - 1) / RJ, nr = (w + RR - 1) / RR;
    for (int e = threadIdx.x; e < ng * nr; e += blockDim.x) {
        const int g = e / nr, r0 = (e - g * nr) * RR;
        R ar[RJ][RR], ai[RJ][RR];
#pragma unroll
        for (int u = 0; u < RJ; ++u)
#pragma unroll
            for (int v = 0; v < RR; ++v) ar[u][v] = ai[u][v] = 0.0;
        const C *x[RJ];
#pragma unroll
        for (int u = 0; u < RJ; ++u) x[u] = xs + min(g * RJ + u, nj - 1) * w;
        for (int m = 0; m < w; ++m) {
            const R *hrow = HTn + m * w;  // HT[m][mp] = H[mp][m]
            R h[RR];
#pragma unroll
            for (int v = 0; v < RR; ++v) h[v] = (r0 + v < w) ? hrow[r0 + v] : 0.0;
#pragma unroll
            for (int u = 0; u < RJ; ++u) {
                const C xv = x[u][m];
#pragma unroll
                for (int v = 0; v < RR; ++v) {
                    ar[u][v] = fma(h[v], xv.x, ar[u][v]);
                    ai[u][v] = fma(h[v], xv.y, ai[u][v]);
                }
            }
        }
#pragma unroll
        for (int u = 0; u < RJ; ++u) {
            const int j = g * RJ + u;
            if (j >= nj) break;
            C *out = a.W1 + (t0 + j) * (int64_t)P2 + n * n;
#pragma unroll
            for (int v = 0; v < RR; ++v)
                if (r0 + v < w) out[r0 + v] = mkc<C>(ar[u][v], ai[u][v]);
        }
    }
}

// ------------------------------------------------------------------ coaxial step
template <class R>
__global__ void __launch_bounds__(256) k_tr_coax(TransArgsT<R> a) {
    using C = typename Cx<R>::T;
    extern __shared__ double2 lds_raw[];
    C *lds = (C *)lds_raw;
    const int m = (int)blockIdx.y - (a.P - 1);
    const int am = m < 0 ? -m : m;
    if (am >= a.ptgt) return;
    const int JT = a.JT, P2 = a.P * a.P;
    const int64_t t0 = (int64_t)blockIdx.x * JT;
    const int nj = (int)min((int64_t)JT, a.njob - t0);
    const int pm = min(a.psrc, a.ptgt);
    const int rows = a.ptgt - am;
    if (am >= pm) {  // no source of this order
        for (int e = threadIdx.x; e < nj * rows; e += blockDim.x) {
            const int j = e / rows, nn = am + (e - j * rows);
            a.W2[(t0 + j) * (int64_t)P2 + nn * nn + nn + m] = mkc<C>(0, 0);
        }
        return;
    }
    const int cin = a.psrc - am;
    C *col = lds;  // JT x cin
    for (int e = threadIdx.x; e < nj * cin; e += blockDim.x) {
        const int j = e / cin, q = e - j * cin, n = am + q;
        col[j * cin + q] = a.W1[(t0 + j) * (int64_t)P2 + n * n + n + m];
    }
    __syncthreads();
    const int B = a.PT - am;
    const C *Tm = a.coax + (int64_t)a.tile_coax[blockIdx.x / a.nr] * coax_table_size(a.PT) + coax_block_off(a.PT, am);
    const int ng = (nj + RJ - 1) / RJ, nr = (rows + RR - 1) / RR;
    for (int e = threadIdx.x; e < ng * nr; e += blockDim.x) {
        const int g = e / nr, r0 = (e - g * nr) * RR;  // output rows nn = am + r0 + v
        R ar[RJ][RR], ai[RJ][RR];
#pragma unroll
        for (int u = 0; u < RJ; ++u)
#pragma unroll
            for (int v = 0; v < RR; ++v) ar[u][v] = ai[u][v] = 0.0;
        const C *x[RJ];
#pragma unroll
        for (int u = 0; u < RJ; ++u) x[u] = col + min(g * RJ + u, nj - 1) * cin;
        for (int q = 0; q < cin; ++q) {
            // (E|F)_{n' n} = (-1)^{n+n'} (E|F)_{n n'}: read row n = am + q of the block
            const C *trow = Tm + (int64_t)q * B;
            C t[RR];
#pragma unroll
            for (int v = 0; v < RR; ++v) {
                const int rr = r0 + v;
                C tv = rr < rows ? trow[rr] : mkc<C>(0, 0);
                if ((q + rr) & 1) tv = mkc<C>(-tv.x, -tv.y);
                t[v] = tv;
            }
#pragma unroll
            for (int u = 0; u < RJ; ++u) {
                const C xv = x[u][q];
#pragma unroll
                for (int v = 0; v < RR; ++v) {
                    ar[u][v] = fma(t[v].x, xv.x, fma(-t[v].y, xv.y, ar[u][v]));
                    ai[u][v] = fma(t[v].x, xv.y, fma(t[v].y, xv.x, ai[u][v]));
                }
            }
        }
#pragma unroll
        for (int u = 0; u < RJ; ++u) {
            const int j = g * RJ + u;
            if (j >= nj) break;
            C *out = a.W2 + (t0 + j) * (int64_t)P2;
#pragma unroll
            for (int v = 0; v < RR; ++v) {
                const int nn = am + r0 + v;
                if (r0 + v < rows) out[nn * nn + nn + m] = mkc<C>(ar[u][v], ai[u][v]);
            }
        }
    }
}

// ------------------------------------------------------------------ back rotation
template <class R>
__global__ void __launch_bounds__(256) k_tr_rot_back(TransArgsT<R> a) {
    using C = typename Cx<R>::T;
    extern __shared__ double2 lds_raw[];
    C *lds = (C *)lds_raw;
    const int n = blockIdx.y;
    if (n >= a.ptgt) return;
    const int w = 2 * n + 1, JT = a.JT;
    C *ys = lds;  // JT x w
    __shared__ int16_t sdir[64];
    const int64_t t0 = (int64_t)blockIdx.x * JT;
    const int nj = (int)min((int64_t)JT, a.njob - t0);
    const int P2 = a.P * a.P, phs = 2 * a.PH + 1;
    for (int j = threadIdx.x; j < nj; j += blockDim.x) sdir[j] = a.jdir[(t0 + j) / a.nr];
    for (int e = threadIdx.x; e < nj * w; e += blockDim.x) {
        const int j = e / w, q = e - j * w;
        ys[j * w + q] = a.W2[(t0 + j) * (int64_t)P2 + n * n + q];
    }
    __syncthreads();
    const R *Hn = a.H + (int64_t)a.tile_rot[blockIdx.x / a.nr] * rot_table_size(a.P) + rot_block_off(n);
    const int ng = (nj + RJ - 1) / RJ, nr = (w + RR - 1) / RR;
    for (int e = threadIdx.x; e < ng * nr; e += blockDim.x) {
        const int g = e / nr, r0 = (e - g * nr) * RR;
        R ar[RJ][RR], ai[RJ][RR];
#pragma unroll
        for (int u = 0; u < RJ; ++u)
#pragma unroll
            for (int v = 0; v < RR; ++v) ar[u][v] = ai[u][v] = 0.0;
        const C *y[RJ];
#pragma unroll
        for (int u = 0; u < RJ; ++u) y[u] = ys + min(g * RJ + u, nj - 1) * w;
        for (int mp = 0; mp < w; ++mp) {
            const R *hrow = Hn + mp * w;  // H[mp][m]: (H^T y)_m = sum_mp H[mp][m] y_mp
            R h[RR];
#pragma unroll
            for (int v = 0; v < RR; ++v) h[v] = (r0 + v < w) ? hrow[r0 + v] : 0.0;
#pragma unroll
            for (int u = 0; u < RJ; ++u) {
                const C yv = y[u][mp];
#pragma unroll
                for (int v = 0; v < RR; ++v) {
                    ar[u][v] = fma(h[v], yv.x, ar[u][v]);
                    ai[u][v] = fma(h[v], yv.y, ai[u][v]);
                }
            }
        }
#pragma unroll
        for (int u = 0; u < RJ; ++u) {
            const int j = g * RJ + u;
            if (j >= nj) break;
            C *out = a.W1 + (t0 + j) * (int64_t)P2 + n * n;
#pragma unroll
            for (int v = 0; v < RR; ++v) {
                const int q = r0 + v;
                if (q >= w) break;
                const C f = a.ph[(int64_t)sdir[j] * phs + a.PH + (q - n)];
                out[q] = mulcc(mkc<C>(ar[u][v], ai[u][v]), f);  // e^{-i m a}
            }
        }
    }
}

// ------------------------------------------------------------------ whole-vector tiles (small p)
// The tile's complete coefficient vectors (JT x P^2) are staged in LDS once; one flat work index
// covers every (degree or order, row group, job group), so a block needs a single barrier.
// Work items per degree n: ceil((2n+1)/RR) row groups; prefix sums are recomputed on the fly.
__device__ inline void deg_of_item(int it, int nmax, int &n, int &rg) {
    // items of degree n: ceil((2n+1)/RR); find n with prefix(n) <= it < prefix(n+1)
    int acc = 0;
    for (n = 0; n < nmax; ++n) {
        const int c = (2 * n + 1 + RR - 1) / RR;
        if (it < acc + c) {
            rg = it - acc;
            return;
        }
        acc += c;
    }
    n = nmax;
    rg = 0;
}
__host__ __device__ inline int items_rot(int p) {
    int s = 0;
    for (int n = 0; n < p; ++n) s += (2 * n + 1 + RR - 1) / RR;
    return s;
}

template <class R, bool FWD>
__global__ void __launch_bounds__(256) k_tw_rot(TransArgsT<R> a) {
    using C = typename Cx<R>::T;
    extern __shared__ double2 lds_raw[];
    C *lds = (C *)lds_raw;
    const int JT = a.JT, P2 = a.P * a.P, phs = 2 * a.PH + 1;
    const int pin = FWD ? a.psrc : a.ptgt;  // degrees handled
    C *X = lds;  // JT x P2 (degrees < pin valid)
    __shared__ int16_t sdir[64];
    const int64_t t0 = (int64_t)blockIdx.x * JT;
    const int nj = (int)min((int64_t)JT, a.njob - t0);
    const int pin2 = pin * pin;
    for (int j = threadIdx.x; j < nj; j += blockDim.x) sdir[j] = a.jdir[(t0 + j) / a.nr];
    __syncthreads();
    for (int e = threadIdx.x; e < nj * pin2; e += blockDim.x) {
        const int j = e / pin2, c = e - j * pin2;
        C v;
        if (FWD) {
            const int n = (int)sqrtf((float)c + 0.5f), m = c - n * n - n;
            v = mulc(a.ph[(int64_t)sdir[j] * phs + a.PH + m], a.src[src_row(a, t0 + j) * (a.psrc * a.psrc) + c]);
        } else {
            v = a.W2[(t0 + j) * (int64_t)P2 + c];
        }
        X[j * P2 + c] = v;
    }
    __syncthreads();
    const R *Hb = (FWD ? a.HT : a.H) + (int64_t)a.tile_rot[blockIdx.x / a.nr] * rot_table_size(a.P);
    const int ng = (nj + RJ - 1) / RJ, nit = items_rot(pin);
    for (int e = threadIdx.x; e < ng * nit; e += blockDim.x) {
        const int g = e / nit;
        int n, rg;
        deg_of_item(e - g * nit, pin, n, rg);
        const int w = 2 * n + 1, r0 = rg * RR;
        const R *Hn = Hb + rot_block_off(n);
        R ar[RJ][RR], ai[RJ][RR];
#pragma unroll
        for (int u = 0; u < RJ; ++u)
#pragma unroll
            for (int v = 0; v < RR; ++v) ar[u][v] = ai[u][v] = 0.0;
        const C *x[RJ];
#pragma unroll
        for (int u = 0; u < RJ; ++u) x[u] = X + min(g * RJ + u, nj - 1) * P2 + n * n;
        for (int k = 0; k < w; ++k) {
            const R *hrow = Hn + k * w;
            R h[RR];
#pragma unroll
            for (int v = 0; v < RR; ++v) h[v] = (r0 + v < w) ? hrow[r0 + v] : 0.0;
#pragma unroll
            for (int u = 0; u < RJ; ++u) {
                const C xv = x[u][k];
#pragma unroll
                for (int v = 0; v < RR; ++v) {
                    ar[u][v] = fma(h[v], xv.x, ar[u][v]);
                    ai[u][v] = fma(h[v], xv.y, ai[u][v]);
                }
            }
        }
#pragma unroll
        for (int u = 0; u < RJ; ++u) {
            const int j = g * RJ + u;
            if (j >= nj) break;
            C *out = a.W1 + (t0 + j) * (int64_t)P2 + n * n;
#pragma unroll
            for (int v = 0; v < RR; ++v) {
                const int q = r0 + v;
                if (q >= w) break;
                C val = mkc<C>(ar[u][v], ai[u][v]);
                if (!FWD) val = mulcc(val, a.ph[(int64_t)sdir[j] * phs + a.PH + (q - n)]);
                out[q] = val;
            }
        }
    }
}

// coaxial step, whole vectors: items over (order m, row group) x job groups
template <class R>
__global__ void __launch_bounds__(256) k_tw_coax(TransArgsT<R> a) {
    using C = typename Cx<R>::T;
    extern __shared__ double2 lds_raw[];
    C *lds = (C *)lds_raw;
    const int JT = a.JT, P2 = a.P * a.P;
    C *X = lds;  // JT x ps2
    const int64_t t0 = (int64_t)blockIdx.x * JT;
    const int nj = (int)min((int64_t)JT, a.njob - t0);
    const int ps2 = a.psrc * a.psrc, pt = a.ptgt;
    for (int e = threadIdx.x; e < nj * ps2; e += blockDim.x) {
        const int j = e / ps2, c = e - j * ps2;
        X[j * ps2 + c] = a.W1[(t0 + j) * (int64_t)P2 + c];
    }
    __syncthreads();
    const C *T = a.coax + (int64_t)a.tile_coax[blockIdx.x / a.nr] * coax_table_size(a.PT);
    const int pm = min(a.psrc, a.ptgt);
    // items: orders m in -(pt-1)..pt-1, row groups ceil((pt-|m|)/RR)
    int nit = 0;
    for (int m = -(pt - 1); m <= pt - 1; ++m) nit += (pt - (m < 0 ? -m : m) + RR - 1) / RR;
    const int ng = (nj + RJ - 1) / RJ;
    for (int e = threadIdx.x; e < ng * nit; e += blockDim.x) {
        const int g = e / nit;
        int it = e - g * nit, m = -(pt - 1);
        for (;; ++m) {
            const int c = (pt - (m < 0 ? -m : m) + RR - 1) / RR;
            if (it < c) break;
            it -= c;
        }
        const int am = m < 0 ? -m : m, r0 = it * RR, rows = pt - am;
        R ar[RJ][RR], ai[RJ][RR];
#pragma unroll
        for (int u = 0; u < RJ; ++u)
#pragma unroll
            for (int v = 0; v < RR; ++v) ar[u][v] = ai[u][v] = 0.0;
        if (am < pm) {
            const int B = a.PT - am;
            const C *Tm = T + coax_block_off(a.PT, am);
            const C *x[RJ];
#pragma unroll
            for (int u = 0; u < RJ; ++u) x[u] = X + min(g * RJ + u, nj - 1) * ps2;
            for (int n = am; n < a.psrc; ++n) {
                const int q = n - am;
                const C *trow = Tm + (int64_t)q * B;
                C tt[RR];
#pragma unroll
                for (int v = 0; v < RR; ++v) {
                    const int rr = r0 + v;
                    C tv = rr < rows ? trow[rr] : mkc<C>(0, 0);
                    if ((q + rr) & 1) tv = mkc<C>(-tv.x, -tv.y);
                    tt[v] = tv;
                }
                const int c = n * n + n + m;
#pragma unroll
                for (int u = 0; u < RJ; ++u) {
                    const C xv = x[u][c];
#pragma unroll
                    for (int v = 0; v < RR; ++v) {
                        ar[u][v] = fma(tt[v].x, xv.x, fma(-tt[v].y, xv.y, ar[u][v]));
                        ai[u][v] = fma(tt[v].x, xv.y, fma(tt[v].y, xv.x, ai[u][v]));
                    }
                }
            }
        }
#pragma unroll
        for (int u = 0; u < RJ; ++u) {
            const int j = g * RJ + u;
            if (j >= nj) break;
            C *out = a.W2 + (t0 + j) * (int64_t)P2;
#pragma unroll
            for (int v = 0; v < RR; ++v) {
                const int nn = am + r0 + v;
                if (r0 + v < rows) out[nn * nn + nn + m] = mkc<C>(ar[u][v], ai[u][v]);
            }
        }
    }
}

// ------------------------------------------------------------------ one job per lane (many jobs per class)
// A wavefront takes 64 consecutive (virtual) jobs of one table class, one job per lane: every
// table value is then the same for all lanes (scalar loads, an SGPR operand of the FMA) and each
// lane keeps its own rows in registers, RC output rows at a time.  Job rows stay in job-major
// layout (P^2 per job), as for the tile kernels.  blockIdx.y picks every nsplit-th degree/order.
constexpr int LANE_JT = 64;

// Wave-uniform, read-only table rows: read through the constant address space so that they
// come in with scalar loads (the kernel only reads the tables).
template <class T> using cst_ptr = const __attribute__((address_space(4))) T *;
template <class T> __device__ inline cst_ptr<T> as_cst(const T *p, int64_t off) {
    return (cst_ptr<T>)(p + __builtin_amdgcn_readfirstlane((int)off));
}
template <class R, int N> __device__ inline void load_row(R (&h)[N], cst_ptr<R> row) {
#pragma unroll
    for (int v = 0; v < N; ++v) h[v] = row[v];
}
// acc_v += h_v x for a table row of RC values, read 16 (or 8) at a time (bounded scalar registers)
template <class R, class C, int RC>
__device__ inline void rot_fma_row(cst_ptr<R> row, C x, R (&ar)[RC], R (&ai)[RC]) {
    constexpr int HS = RC % 16 == 0 ? 16 : 8;
    static_assert(RC % HS == 0, "row chunks are multiples of 8");
#pragma unroll
    for (int h0 = 0; h0 < RC; h0 += HS) {
        R h[HS];
#pragma unroll
        for (int v = 0; v < HS; ++v) h[v] = row[h0 + v];
#pragma unroll
        for (int v = 0; v < HS; ++v) {
            ar[h0 + v] = fma(h[v], x.x, ar[h0 + v]);
            ai[h0 + v] = fma(h[v], x.y, ai[h0 + v]);
        }
    }
}
// acc_v += s_v T_v x with T_v = (t[2v], t[2v+1]) and s_v = (-1)^v, negated when NEG
template <class R, class C, int RC, bool NEG>
__device__ inline void coax_acc(const R (&t)[2 * RC], C x, R (&ar)[RC], R (&ai)[RC]) {
#pragma unroll
    for (int v = 0; v < RC; ++v) {
        const bool neg = ((v & 1) != 0) != NEG;
        const R tx = neg ? -t[2 * v] : t[2 * v], ty = neg ? -t[2 * v + 1] : t[2 * v + 1];
        ar[v] = fma(tx, x.x, fma(-ty, x.y, ar[v]));
        ai[v] = fma(tx, x.y, fma(ty, x.x, ai[v]));
    }
}
static_assert(TABLE_PAD >= 32, "lane kernels read up to 31 entries past a table row");

// XCD-aware block order.  Consecutive workgroups go to the 8 XCDs in turn, and each XCD has its own
// L2; renumbering the (tile, split) grid so that each XCD takes one contiguous range of the
// class-sorted tiles keeps every translation table in the L2 of one XCD (and in the scalar caches
// of the waves that work through that range together).  A bijection of [0, gridDim.x gridDim.y).
constexpr unsigned NXCD = 8;
__device__ inline void xcd_block(int &tile, int &split) {
    const unsigned nx = gridDim.x, ny = gridDim.y, n = nx * ny;
    const unsigned L = blockIdx.x + blockIdx.y * nx;
    const unsigned x = L % NXCD, l = L / NXCD, q = n / NXCD, r = n % NXCD;
    const unsigned p = x * q + min(x, r) + l;
    tile = (int)(p / ny);
    split = (int)(p % ny);
}

// Intermediate rows of lane batches are tile-interleaved: coefficient c of virtual job J at
// ((J / 64) P^2 + c) 64 + J % 64, so that a wavefront's 64 lanes touch 64 consecutive values.
__device__ inline int64_t tl_idx(int64_t J, int c, int P2) { return ((J >> 6) * P2 + c) * LANE_JT + (J & 63); }

// Output rows are produced in chunks of RCK rows per lane (accumulators in registers).  The chunk
// size is picked per degree (per order in the coaxial step) as the smallest of 8, 16, 24, 32 (4, 8,
// 12, 16) rows that covers the rows left, so that few FMAs fall on rows past the degree.
#define TL_ROT_CHUNK(rem, CALL)                                                       \
    if ((rem) <= 8) CALL(8); else if ((rem) <= 16) CALL(16); else if ((rem) <= 24) CALL(24); \
    else CALL(32)
#define TL_COAX_CHUNK(rem, CALL) \
    if ((rem) <= 4) CALL(4); else if ((rem) <= 8) CALL(8); else if ((rem) <= 12) CALL(12); else CALL(16)

// Forward rotation: sources (box-major) -> W1 (interleaved).  The degree-n slices are staged
// through LDS 8 columns at a time: one load instruction reads 8 jobs x 8 consecutive
// coefficients, i.e. whole 128-byte lines (a lane reading its own row alone would fetch each
// line for 16 bytes once the wave's 64 rows no longer fit L1).
constexpr int TL_CW = 8;
template <class R, int RCK, bool PF>
__device__ inline void tl_rot_fwd_chunk(const TransArgsT<R> &a, typename Cx<R>::T (*S)[TL_CW + 1], const int64_t *soff,
                                        const int32_t *sdir, const R *Hn, int n, int w, int r0, int64_t J, bool live,
                                        int P2, int lane) {
    using C = typename Cx<R>::T;
    const int sj = lane >> 3, sq = lane & 7;  // staging: job sj + 8 i, column sq
    R ar[RCK], ai[RCK];
#pragma unroll
    for (int v = 0; v < RCK; ++v) ar[v] = ai[v] = 0;
    for (int c0 = 0; c0 < w; c0 += TL_CW) {
        const int cw = min(TL_CW, w - c0);
        __syncthreads();
        if (sq < cw) {
            const int c = c0 + sq;
#pragma unroll
            for (int i0 = 0; i0 < LANE_JT / 8; i0 += 4) {
                C xs[4], ps[4];  // four jobs' loads in flight before the first use
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int j = sj + 8 * (i0 + i);
                    xs[i] = a.src[soff[j] + n * n + c];
                    ps[i] = a.ph[sdir[j] + c - n];
                }
#pragma unroll
                for (int i = 0; i < 4; ++i) S[sj + 8 * (i0 + i)][sq] = mulc(ps[i], xs[i]);  // e^{i m a} c_n^m
            }
        }
        __syncthreads();
        // rows past w read the next table entries (TABLE_PAD spare); never stored.  With PF the
        // next table row is loaded before the current one is used.
        if (PF) {
            R h[RCK];
            load_row<R, RCK>(h, as_cst(Hn, c0 * w + r0));
            for (int q = 0; q < cw; ++q) {
                const C xv = S[lane][q];
                R hn[RCK];
                load_row<R, RCK>(hn, as_cst(Hn, (c0 + q + 1) * w + r0));  // spare-padded
#pragma unroll
                for (int v = 0; v < RCK; ++v) {
                    ar[v] = fma(h[v], xv.x, ar[v]);
                    ai[v] = fma(h[v], xv.y, ai[v]);
                }
#pragma unroll
                for (int v = 0; v < RCK; ++v) h[v] = hn[v];
            }
        } else {
            for (int q = 0; q < cw; ++q) {
                const C xv = S[lane][q];
                rot_fma_row<R, C, RCK>(as_cst(Hn, (c0 + q) * w + r0), xv, ar, ai);
            }
        }
    }
    if (live) {
#pragma unroll
        for (int v = 0; v < RCK; ++v)
            if (r0 + v < w) a.W1[tl_idx(J, n * n + r0 + v, P2)] = mkc<C>(ar[v], ai[v]);
    }
}

template <class R, bool PF>
__global__ void __launch_bounds__(64) k_tl_rot_fwd(TransArgsT<R> a, int nsplit) {
    using C = typename Cx<R>::T;
    __shared__ C S[LANE_JT][TL_CW + 1];
    __shared__ int64_t soff[LANE_JT];
    __shared__ int32_t sdir[LANE_JT];
    const int lane = threadIdx.x;
    int tile, split;
    xcd_block(tile, split);
    const int64_t J0 = (int64_t)tile * LANE_JT, J = J0 + lane;
    const bool live = J < a.njob;
    const int64_t Jc = live ? J : a.njob - 1;
    const int P2 = a.P * a.P, phs = 2 * a.PH + 1, ps2 = a.psrc * a.psrc;
    soff[lane] = src_row(a, Jc) * ps2;
    sdir[lane] = a.jdir[Jc / a.nr] * phs + a.PH;
    const int tr = __builtin_amdgcn_readfirstlane(a.tile_rot[tile / a.nr]);
    const R *Hb = a.HT + (int64_t)tr * rot_table_size(a.P);
    for (int n = split; n < a.psrc; n += nsplit) {
        const int w = 2 * n + 1;
        const R *Hn = Hb + rot_block_off(n);  // HT: row c holds column c of H
        for (int r0 = 0; r0 < w; r0 += 32) {
#define TL_FWD(K) tl_rot_fwd_chunk<R, K, PF>(a, S, soff, sdir, Hn, n, w, r0, J, live, P2, lane)
            TL_ROT_CHUNK(w - r0, TL_FWD);
#undef TL_FWD
        }
    }
}

// Back rotation: W2 (interleaved) -> W1 (job-major, for the per-target reduction), through an
// LDS transpose 8 rows at a time.  With one block per tile (nsplit == 1) the outputs come in
// increasing coefficient order; in FP64 they pass through a ring of RING coefficients per job and
// leave in whole 128-byte lines (G coefficients), so no line of the job-major rows is written in
// parts (in FP32 the ring measured slower and its LDS would cost occupancy).
template <class R> struct TlRing {
    using C = typename Cx<R>::T;
    static constexpr bool ON = sizeof(R) == 8;
    static constexpr int OT = 8, G = 128 / sizeof(C), RING = 16, OW = ON ? RING : OT;
    static_assert(!ON || G + OT <= RING, "ring too small for a pending line and a transpose group");
};
// sum of column q of lanes j, j + nr, ..., j + (len-1) nr (one run of a target, one vector)
template <class C, int W>
__device__ inline C run_sum(C (*O)[W], int j, int len, int nr, int q) {
    C v = O[j][q];
    for (int k = 1; k < len; ++k) v = addc(v, O[j + k * nr][q]);
    return v;
}
template <class R, int RCK, bool PF>
__device__ inline void tl_rot_back_chunk(const TransArgsT<R> &a, typename Cx<R>::T (*O)[TlRing<R>::OW + 1], const R *Hn,
                                         const typename Cx<R>::T *ph, int n, int w, int r0, int64_t J0, int64_t Jc,
                                         const int *segl, int P2, int lane, bool ordered, int &base, int &cnext) {
    using C = typename Cx<R>::T;
    using RG = TlRing<R>;
    R ar[RCK], ai[RCK];
#pragma unroll
    for (int v = 0; v < RCK; ++v) ar[v] = ai[v] = 0;
    if (PF) {
        C xv = a.W2[tl_idx(Jc, n * n, P2)];
        R h[RCK];
        load_row<R, RCK>(h, as_cst(Hn, r0));
        for (int c = 0; c < w; ++c) {
            // next table row and next input value first (spare-padded table, clamped index)
            R hn[RCK];
            load_row<R, RCK>(hn, as_cst(Hn, (c + 1) * w + r0));
            const C xn = a.W2[tl_idx(Jc, n * n + min(c + 1, w - 1), P2)];
#pragma unroll
            for (int v = 0; v < RCK; ++v) {
                ar[v] = fma(h[v], xv.x, ar[v]);
                ai[v] = fma(h[v], xv.y, ai[v]);
            }
#pragma unroll
            for (int v = 0; v < RCK; ++v) h[v] = hn[v];
            xv = xn;
        }
    } else {
        C xv = a.W2[tl_idx(Jc, n * n, P2)];
        for (int c = 0; c < w; ++c) {
            const C xn = a.W2[tl_idx(Jc, n * n + min(c + 1, w - 1), P2)];
            rot_fma_row<R, C, RCK>(as_cst(Hn, c * w + r0), xv, ar, ai);
            xv = xn;
        }
    }
    // transpose to job-major rows OT rows at a time
#pragma unroll
    for (int h0 = 0; h0 < RCK; h0 += RG::OT) {
        const int rc = min(RG::OT, w - r0 - h0);
        if (rc <= 0) break;
        const int c0 = n * n + r0 + h0;
        __syncthreads();
#pragma unroll
        for (int v = 0; v < RG::OT; ++v)
            if (v < rc) {
                const C val = mulcc(mkc<C>(ar[h0 + v], ai[h0 + v]), ph[r0 + h0 + v - n]);  // e^{-i m a}
                O[lane][ordered ? (c0 + v) % RG::RING : v] = val;
            }
        __syncthreads();
        if (ordered) {
            cnext = c0 + rc;
            while (cnext - base >= RG::G) {  // one store instruction: 64/G jobs x one whole line
                const int q = lane % RG::G;
#pragma unroll
                for (int i = 0; i < RG::G; ++i) {
                    const int j = lane / RG::G + (64 / RG::G) * i;
                    const int len = segl[j];
                    if (len > 0) a.W1[(J0 + j) * (int64_t)P2 + base + q] = run_sum(O, j, len, a.nr, (base + q) % RG::RING);
                }
                base += RG::G;
            }
        } else {
            // one store instruction: 8 jobs x 8 consecutive coefficients
            const int q = lane & 7;
            if (q < rc) {
#pragma unroll
                for (int i = 0; i < LANE_JT / 8; ++i) {
                    const int j = (lane >> 3) + 8 * i;
                    const int len = segl[j];
                    if (len > 0) a.W1[(J0 + j) * (int64_t)P2 + c0 + q] = run_sum(O, j, len, a.nr, q);
                }
            }
        }
    }
}

template <class R, bool PF>
__global__ void __launch_bounds__(64) k_tl_rot_back(TransArgsT<R> a, int nsplit) {
    using C = typename Cx<R>::T;
    using RG = TlRing<R>;
    __shared__ C O[LANE_JT][RG::OW + 1];
    __shared__ int segl[LANE_JT];  // per lane: run length if the lane's job starts a run, else 0
    const bool ordered = RG::ON && nsplit == 1;
    int base = 0, cnext = 0;  // first coefficient not yet stored; next coefficient to be produced
    const int lane = threadIdx.x;
    int tile, split;
    xcd_block(tile, split);
    const int64_t J0 = (int64_t)tile * LANE_JT, J = J0 + lane;
    const int64_t Jc = J < a.njob ? J : a.njob - 1;
    const int P2 = a.P * a.P, phs = 2 * a.PH + 1;
    const int nlive = (int)min((int64_t)LANE_JT, a.njob - J0);
    // a run of real jobs h..h+len-1 holds, for vector r, lanes (h - h0) nr + r + k nr
    segl[lane] = lane < nlive ? a.jseg[J / a.nr] : 0;
    const int tr = __builtin_amdgcn_readfirstlane(a.tile_rot[tile / a.nr]);
    const R *Hb = a.H + (int64_t)tr * rot_table_size(a.P);
    const C *ph = a.ph + (int64_t)a.jdir[Jc / a.nr] * phs + a.PH;
    for (int n = split; n < a.ptgt; n += nsplit) {
        const int w = 2 * n + 1;
        const R *Hn = Hb + rot_block_off(n);  // (H^T y)_r = sum_c H[c][r] y_c: row c of H
        for (int r0 = 0; r0 < w; r0 += 32) {
#define TL_BACK(K) tl_rot_back_chunk<R, K, PF>(a, O, Hn, ph, n, w, r0, J0, Jc, segl, P2, lane, ordered, base, cnext)
            TL_ROT_CHUNK(w - r0, TL_BACK);
#undef TL_BACK
        }
    }
    if (ordered && cnext > base) {  // the last, partial line
        const int cnt = cnext - base;
        for (int e = lane; e < nlive * RG::G; e += LANE_JT) {
            const int j = e / RG::G, q = e % RG::G;
            const int len = segl[j];
            if (q < cnt && len > 0) a.W1[(J0 + j) * (int64_t)P2 + base + q] = run_sum(O, j, len, a.nr, (base + q) % RG::RING);
        }
    }
}

// Coaxial step: W1 (interleaved) -> W2 (interleaved), fully coalesced.
template <class R, int RCK, bool PF>
__device__ inline void tl_coax_chunk(const TransArgsT<R> &a, const typename Cx<R>::T *Tm, int m, int am, int rows,
                                     int cin, int B, int r0, int64_t J, int64_t Jc, bool live, int P2) {
    using C = typename Cx<R>::T;
    R ar[RCK], ai[RCK];
#pragma unroll
    for (int v = 0; v < RCK; ++v) ar[v] = ai[v] = 0;
    // (E|F)_{n' n} = (-1)^{n+n'} (E|F)_{n n'}: row n of the block, entries n'; rows past `rows`
    // read spare table entries (TABLE_PAD) and are never stored.  The sign is fixed per unrolled
    // row for each parity of q + r0, so it folds into the FMAs.
    R t[2 * RCK];
    load_row<R, 2 * RCK>(t, as_cst((const R *)Tm, 2 * (int64_t)r0));
    int n = am;
    C xv = a.W1[tl_idx(Jc, n * n + n + m, P2)];
    for (int q = 0; q < cin; ++q, ++n) {
        R tn[PF ? 2 * RCK : 1];
        if (PF) load_row<R, PF ? 2 * RCK : 1>(tn, as_cst((const R *)Tm, 2 * ((int64_t)(q + 1) * B + r0)));
        const int nn1 = min(n + 1, a.psrc - 1);
        const C xn = a.W1[tl_idx(Jc, nn1 * nn1 + nn1 + m, P2)];
        if (((q + r0) & 1) == 0) coax_acc<R, C, RCK, false>(t, xv, ar, ai);
        else coax_acc<R, C, RCK, true>(t, xv, ar, ai);
        if (PF) {
#pragma unroll
            for (int v = 0; v < 2 * RCK; ++v) t[v] = tn[PF ? v : 0];
        } else if (q + 1 < cin) {
            load_row<R, 2 * RCK>(t, as_cst((const R *)Tm, 2 * ((int64_t)(q + 1) * B + r0)));
        }
        xv = xn;
    }
    if (live) {
#pragma unroll
        for (int v = 0; v < RCK; ++v) {
            const int nn = am + r0 + v;
            if (r0 + v < rows) a.W2[tl_idx(J, nn * nn + nn + m, P2)] = mkc<C>(ar[v], ai[v]);
        }
    }
}

template <class R, bool PF>
__global__ void __launch_bounds__(64) k_tl_coax(TransArgsT<R> a, int nsplit) {
    using C = typename Cx<R>::T;
    int tile, split;
    xcd_block(tile, split);
    const int64_t J = (int64_t)tile * LANE_JT + threadIdx.x;
    const bool live = J < a.njob;
    const int64_t Jc = live ? J : a.njob - 1;
    const int P2 = a.P * a.P, pt = a.ptgt, pm = min(a.psrc, a.ptgt);
    const int tc = __builtin_amdgcn_readfirstlane(a.tile_coax[tile / a.nr]);
    const C *T = a.coax + (int64_t)tc * coax_table_size(a.PT);
    for (int mi = split; mi < 2 * pt - 1; mi += nsplit) {
        const int m = mi - (pt - 1), am = m < 0 ? -m : m;
        const int rows = pt - am;
        if (am >= pm) {  // no source of this order
            if (live)
                for (int q = 0; q < rows; ++q) {
                    const int nn = am + q;
                    a.W2[tl_idx(J, nn * nn + nn + m, P2)] = mkc<C>(0, 0);
                }
            continue;
        }
        const int B = a.PT - am, cin = a.psrc - am;
        const C *Tm = T + coax_block_off(a.PT, am);
        for (int r0 = 0; r0 < rows; r0 += 16) {
#define TL_CX(K) tl_coax_chunk<R, K, PF>(a, Tm, m, am, rows, cin, B, r0, J, Jc, live, P2)
            TL_COAX_CHUNK(rows - r0, TL_CX);
#undef TL_CX
        }
    }
}

// ------------------------------------------------------------------ matrix-core tiles (large p)
// For large p a degree (order) of a 64-job tile is a real GEMM: Y (rows x 128 columns: job j, real
// and imaginary part) = M X with M the tile's (2n+1)^2 rotation block or (p-|m|)^2 coaxial block.
// FP64 matrix cores, v_mfma_f64_16x16x4f64, fragments of lane l: A[l%16][l/16], B[l/16][l%16],
// D[l/16 + 4i][l%16] (i = 0..3).  A workgroup of 4 wavefronts takes one (tile, degree) or (tile,
// order); wavefront w owns columns 32w..32w+31 (jobs 16w..16w+15), all rows, in groups of row
// blocks (16 rows each).  Same tile layout and work rows as the lane kernels.
// FP32 (mixed products): v_mfma_f32_16x16x4f32, same A and B fragments, D[4 (l/16) + i][l%16].
template <class R> struct TmOp;
template <> struct TmOp<double> {
    typedef double v4 __attribute__((ext_vector_type(4)));
    static __device__ inline v4 mma(double a, double b, v4 c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
    static __device__ inline int row(int kq, int i) { return kq + 4 * i; }
};
template <> struct TmOp<float> {
    typedef float v4 __attribute__((ext_vector_type(4)));
    static __device__ inline v4 mma(float a, float b, v4 c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
    static __device__ inline int row(int kq, int i) { return 4 * kq + i; }
};
constexpr int TM_KC = 8;    // K rows per LDS chunk (double-buffered) of the rotations
constexpr int TM_LD = 130;  // LDS row stride (doubles) of the staged A and B chunks

// Rotation of degree n for one tile of TMJ jobs (64 or 32: 2 TMJ columns, the four wavefronts owning
// TMJ / 2 columns each, in NCB = TMJ / 32 blocks of 16), as a GEMM over K chunks staged in LDS
// (double-buffered: the global loads of chunk c+1 are issued before the matrix-core work on chunk
// c).  RBG row blocks of 16 rows per pass; a workgroup takes the passes pass, pass + npass, ... of
// its degree.
//   FWD:  Y = H X, X = e^{i m a} c_n of the sources, A[r][k] = H[r][k] = HT[k][r]; rows -> W1.
//   !FWD: Y = H^T X, X = W2 rows, A[r][k] = H[k][r]; the pass's outputs go through LDS, are
//         phased (e^{-i m a}), summed over the runs of one target and stored job-major in W1.
template <class R, bool FWD, int RBG, int TMJ>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4, 4))) k_tm_rot(TransArgsT<R> a, int npass) {
    using C = typename Cx<R>::T;
    using Op = TmOp<R>;
    using v4 = typename Op::v4;
    constexpr int RG = 16 * RBG;            // rows per pass
    constexpr int NCOL = 2 * TMJ;           // real columns of a tile
    constexpr int NCB = TMJ / 32;           // 16-column blocks per wavefront
    // K chunks of 8 and passes of 64 rows: 33 KB of LDS, four workgroups per CU (measured at levels
    // 2-5 of the 1M L-room against chunks of 16 and passes of 128 / 64 rows: back rotation 1.51 ->
    // 1.15 ms, forward rotation 1.90 -> 1.66 ms per product).  The back rotation's outputs leave
    // through the same LDS block 32 rows at a time (64-row passes instead of 32: FP64 product
    // 10.97 -> 10.88 ms, mixed 9.00 -> 8.86 ms).
    constexpr int KC = TM_KC;
    constexpr int EQ = RBG < 2 ? RBG : 2;  // back: row blocks per epilogue step (32 rows through LDS)
    constexpr int LDSN = FWD ? 4 * KC * TM_LD : (4 * KC > 16 * EQ ? 4 * KC : 16 * EQ) * TM_LD;
    static_assert(RG <= 128 && RBG % EQ == 0, "pass too large for the LDS block");
    static_assert(TMJ == 64 || TMJ == 32, "tiles of 64 or 32 jobs");
    __shared__ R lds[LDSN];
    __shared__ int64_t soff[TMJ];
    __shared__ int32_t sdir[TMJ];
    __shared__ int segl[TMJ];
    auto As = [&](int buf, int k, int r) -> R & { return lds[(buf * KC + k) * TM_LD + r]; };
    auto Bs = [&](int buf, int k, int c) -> R & { return lds[((2 + buf) * KC + k) * TM_LD + c]; };
    int tile, nq;
    xcd_block(tile, nq);
    const int n = nq / npass, pass = nq - n * npass;  // degree, and the pass's share of its row groups
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int64_t J0 = (int64_t)tile * TMJ;
    const int P2 = a.P * a.P, phs = 2 * a.PH + 1, ps2 = a.psrc * a.psrc;
    if (tid < TMJ) {
        const int64_t J = J0 + tid, Jc = J < a.njob ? J : a.njob - 1;
        soff[tid] = FWD ? src_row(a, Jc) * ps2 : 0;
        sdir[tid] = a.jdir[Jc / a.nr] * phs + a.PH;
        segl[tid] = (!FWD && J < a.njob) ? a.jseg[J / a.nr] : 0;
    }
    __syncthreads();
    const int w = 2 * n + 1, RB = (w + 15) / 16;
    const int tr = a.tile_rot[tile / a.nr];
    const R *Mn = (FWD ? a.HT : a.H) + (int64_t)tr * rot_table_size(a.P) + rot_block_off(n);
    const R *Xin = (const R *)a.W2;
    const int colw = (NCOL / 4) * wv + (lane & 15), kq = lane >> 4;
    const int nch = (w + KC - 1) / KC;
    constexpr int NA = KC * RG / 256;   // A values staged per thread
    constexpr int NB = KC * NCOL / 256;  // B values staged per thread
    for (int rb0 = pass * RBG; rb0 < RB; rb0 += npass * RBG) {
        const int r0 = rb0 * 16;
        // the forward rotation keeps the loaded phases and source coefficients until the LDS store,
        // so that the next chunk's loads stay in flight through the matrix-core work (1.66 -> 1.35 ms
        // per product at levels 2-5 of the 1M L-room, against multiplying them as they arrive)
        R ra[NA], rbv[FWD ? 1 : NB];
        C rph[FWD ? NB / 2 : 1], rsr[FWD ? NB / 2 : 1];
        auto gload = [&](int kc) {
#pragma unroll
            for (int i = 0; i < NA; ++i) {
                const int e = tid + 256 * i, kk = e / RG, rr = e % RG, k = kc + kk, r = r0 + rr;
                ra[i] = (k < w && r < w) ? Mn[(int64_t)k * w + r] : R(0);
            }
            if (FWD) {
#pragma unroll
                for (int i = 0; i < NB / 2; ++i) {
                    const int e = tid + 256 * i, kk = e % KC, j = e / KC, k = kc + kk;  // a job's KC rows: one segment
                    rph[i] = k < w ? a.ph[sdir[j] + k - n] : mkc<C>(0, 0);
                    rsr[i] = k < w ? a.src[soff[j] + n * n + k] : mkc<C>(0, 0);
                }
            } else {
#pragma unroll
                for (int i = 0; i < NB; ++i) {
                    const int e = tid + 256 * i, kk = e / NCOL, col = e % NCOL, k = kc + kk;
                    rbv[i] = k < w ? Xin[((int64_t)tile * P2 + n * n + k) * NCOL + col] : R(0);
                }
            }
        };
        auto lstore = [&](int buf) {
#pragma unroll
            for (int i = 0; i < NA; ++i) {
                const int e = tid + 256 * i;
                As(buf, e / RG, e % RG) = ra[i];
            }
            if (FWD) {
#pragma unroll
                for (int i = 0; i < NB / 2; ++i) {
                    const int e = tid + 256 * i, kk = e % KC, j = e / KC;
                    const C x = mulc(rph[i], rsr[i]);  // e^{i m a} c_n^m
                    Bs(buf, kk, 2 * j) = x.x;
                    Bs(buf, kk, 2 * j + 1) = x.y;
                }
            } else {
#pragma unroll
                for (int i = 0; i < NB; ++i) {
                    const int e = tid + 256 * i;
                    Bs(buf, e / NCOL, e % NCOL) = rbv[i];
                }
            }
        };
        v4 acc[RBG][NCB];
#pragma unroll
        for (int q = 0; q < RBG; ++q)
#pragma unroll
            for (int cb = 0; cb < NCB; ++cb) acc[q][cb] = v4{0, 0, 0, 0};
        gload(0);
        __syncthreads();  // the previous pass's readers of the LDS block are done
        lstore(0);
        __syncthreads();
        for (int c = 0; c < nch; ++c) {
            const int buf = c & 1;
            if (c + 1 < nch) gload((c + 1) * KC);
            const int kn = min(KC, w - c * KC);
            for (int ks = 0; ks < kn; ks += 4) {
                R bv[NCB];
#pragma unroll
                for (int cb = 0; cb < NCB; ++cb) bv[cb] = Bs(buf, ks + kq, colw + 16 * cb);
#pragma unroll
                for (int q = 0; q < RBG; ++q) {
                    if (rb0 + q >= RB) break;
                    const R av = As(buf, ks + kq, q * 16 + (lane & 15));
#pragma unroll
                    for (int cb = 0; cb < NCB; ++cb) acc[q][cb] = Op::mma(av, bv[cb], acc[q][cb]);
                }
            }
            if (c + 1 < nch) {
                lstore(buf ^ 1);
                __syncthreads();
            }
        }
        if (FWD) {
            R *Wout = (R *)a.W1;
#pragma unroll
            for (int q = 0; q < RBG; ++q) {
                if (rb0 + q >= RB) break;
#pragma unroll
                for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const int r = (rb0 + q) * 16 + Op::row(kq, i);
                        if (r < w) Wout[((int64_t)tile * P2 + n * n + r) * NCOL + colw + 16 * cb] = acc[q][cb][i];
                    }
            }
        } else {
            // the pass's output rows go through the LDS block EQ row blocks (ER rows x NCOL columns)
            // at a time: phase, run sums and job-major stores (consecutive threads: consecutive rows
            // of one job)
            constexpr int ER = 16 * EQ, NE = ER * TMJ / 256;
#pragma unroll
            for (int q0 = 0; q0 < RBG; q0 += EQ) {
                if (rb0 + q0 >= RB) break;
                __syncthreads();
#pragma unroll
                for (int q = 0; q < EQ; ++q)
#pragma unroll
                    for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
                        for (int i = 0; i < 4; ++i)
                            lds[(q * 16 + Op::row(kq, i)) * TM_LD + colw + 16 * cb] = acc[q0 + q][cb][i];
                __syncthreads();
                const int rs = r0 + 16 * q0, nrow = min(ER, w - rs);
                // phase every (row, job) in place first, four phase loads in flight at a time, so
                // that the run sums below read LDS only
                constexpr int NG = NE < 4 ? NE : 4;
#pragma unroll
                for (int i0 = 0; i0 < NE; i0 += NG) {
                    C phv[NG];
#pragma unroll
                    for (int i = 0; i < NG; ++i) {
                        const int e = tid + 256 * (i0 + i), j = e / ER, rr = e % ER;
                        phv[i] = rr < nrow ? a.ph[sdir[j] + rs + rr - n] : mkc<C>(0, 0);
                    }
#pragma unroll
                    for (int i = 0; i < NG; ++i) {
                        const int e = tid + 256 * (i0 + i), j = e / ER, rr = e % ER;
                        R *x = &lds[rr * TM_LD + 2 * j];
                        const C v = mulcc(mkc<C>(x[0], x[1]), phv[i]);  // e^{-i m a}
                        x[0] = v.x;
                        x[1] = v.y;
                    }
                }
                __syncthreads();
                for (int e = tid; e < ER * TMJ; e += 256) {
                    const int j = e / ER, rr = e % ER, r = rs + rr;
                    const int len = segl[j];
                    if (rr >= nrow || len == 0) continue;
                    C v = mkc<C>(0, 0);
                    for (int t = 0; t < len; ++t) {
                        const int jj = j + t * a.nr;
                        v = addc(v, mkc<C>(lds[rr * TM_LD + 2 * jj], lds[rr * TM_LD + 2 * jj + 1]));
                    }
                    a.W1[(J0 + j) * (int64_t)P2 + n * n + r] = v;
                }
            }
        }
    }
}

// Coaxial step of order m for one tile of TMJ jobs: Y = T X with the complex (p-|m|)^2 block T
// (entries (-1)^{n+n'} (E|F)_{n n'}, as in the lane kernel) applied to the W1 rows of order m, K
// chunks staged in LDS as for the rotations.  With X' the input with each job's real and imaginary
// columns swapped and the new real one negated (read from the partner column of X in LDS),
// Y = Re(T) X + Im(T) X' column by column, so one accumulator set takes both real GEMMs.
// RBG row blocks of 16 rows per pass, K chunks of KC rows.
template <class R, int TMJ, int RBG, int KC>
__global__ void __launch_bounds__(256) k_tm_coax(TransArgsT<R> a, int npass) {
    using C = typename Cx<R>::T;
    using Op = TmOp<R>;
    using v4 = typename Op::v4;
    constexpr int RG = 16 * RBG, LA = RG + 2;
    constexpr int NCOL = 2 * TMJ, NCB = TMJ / 32;
    constexpr int NA = (KC * RG + 255) / 256, NX = (KC * TMJ + 255) / 256;  // staged values per thread
    static_assert(TMJ == 64 || TMJ == 32, "tiles of 64 or 32 jobs");
    static_assert(KC % 4 == 0 && (KC * RG) % 64 == 0 && (KC * TMJ) % 64 == 0, "whole wavefronts per staged chunk");
    // A: real part (chunks 0, 1) and imaginary part (2, 3), RG + 2 columns; B: X (2 chunks)
    __shared__ R ldsA[4 * KC * LA];
    __shared__ R ldsB[2 * KC * TM_LD];
    auto Ar = [&](int buf, int k, int r) -> R & { return ldsA[(buf * KC + k) * LA + r]; };
    auto Ai = [&](int buf, int k, int r) -> R & { return ldsA[((2 + buf) * KC + k) * LA + r]; };
    auto Bs = [&](int buf, int k, int c) -> R & { return ldsB[(buf * KC + k) * TM_LD + c]; };
    int tile, mq;
    xcd_block(tile, mq);
    const int mi = mq / npass, pass = mq - mi * npass;  // order index, and the pass's share of its row groups
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int P2 = a.P * a.P, pt = a.ptgt, pm = min(a.psrc, a.ptgt);
    const int m = mi - (pt - 1), am = m < 0 ? -m : m;
    const int rows = pt - am;
    R *Wout = (R *)a.W2;
    const C *Xin = a.W1;
    if (am >= pm) {  // no source of this order
        if (pass != 0) return;
        for (int e = tid; e < rows * NCOL; e += 256) {
            const int nn = am + e / NCOL;
            Wout[((int64_t)tile * P2 + nn * nn + nn + m) * NCOL + e % NCOL] = R(0);
        }
        return;
    }
    const int B = a.PT - am, cin = a.psrc - am, RB = (rows + 15) / 16;
    const C *Tm = a.coax + (int64_t)a.tile_coax[tile / a.nr] * coax_table_size(a.PT) + coax_block_off(a.PT, am);
    const int colw = (NCOL / 4) * wv + (lane & 15), kq = lane >> 4;
    const R swp = (colw & 1) ? R(1) : R(-1);
    const int nch = (cin + KC - 1) / KC;
    for (int rb0 = pass * RBG; rb0 < RB; rb0 += npass * RBG) {
        const int r0 = rb0 * 16;
        C ta[NA];
        C xb[NX];  // (re, im) of NX (k, job) inputs
        auto gload = [&](int kc) {
#pragma unroll
            for (int i = 0; i < NA; ++i) {
                const int e = tid + 256 * i, kk = e / RG, rr = e % RG, k = kc + kk, r = r0 + rr;
                C t = (e < KC * RG && k < cin && r < rows) ? Tm[(int64_t)k * B + r] : mkc<C>(0, 0);
                if ((k + r) & 1) t = mkc<C>(-t.x, -t.y);
                ta[i] = t;
            }
#pragma unroll
            for (int i = 0; i < NX; ++i) {
                const int e = tid + 256 * i, kk = e / TMJ, j = e % TMJ, k = kc + kk, nb = am + k;
                xb[i] = (e < KC * TMJ && k < cin) ? Xin[((int64_t)tile * P2 + nb * nb + nb + m) * TMJ + j] : mkc<C>(0, 0);
            }
        };
        auto lstore = [&](int buf) {
#pragma unroll
            for (int i = 0; i < NA; ++i) {
                const int e = tid + 256 * i;
                if (e < KC * RG) {
                    Ar(buf, e / RG, e % RG) = ta[i].x;
                    Ai(buf, e / RG, e % RG) = ta[i].y;
                }
            }
#pragma unroll
            for (int i = 0; i < NX; ++i) {
                const int e = tid + 256 * i, kk = e / TMJ, j = e % TMJ;
                if (e < KC * TMJ) {
                    Bs(buf, kk, 2 * j) = xb[i].x;
                    Bs(buf, kk, 2 * j + 1) = xb[i].y;
                }
            }
        };
        v4 acc[RBG][NCB];
#pragma unroll
        for (int q = 0; q < RBG; ++q)
#pragma unroll
            for (int cb = 0; cb < NCB; ++cb) acc[q][cb] = v4{0, 0, 0, 0};
        gload(0);
        __syncthreads();
        lstore(0);
        __syncthreads();
        for (int c = 0; c < nch; ++c) {
            const int buf = c & 1;
            if (c + 1 < nch) gload((c + 1) * KC);
            const int kn = min(KC, cin - c * KC);
            for (int ks = 0; ks < kn; ks += 4) {
                R bv[NCB], wv2[NCB];
#pragma unroll
                for (int cb = 0; cb < NCB; ++cb) {
                    bv[cb] = Bs(buf, ks + kq, colw + 16 * cb);
                    // X': column 2j holds -Im x_j, column 2j+1 holds Re x_j (the partner column)
                    wv2[cb] = swp * Bs(buf, ks + kq, (colw + 16 * cb) ^ 1);
                }
#pragma unroll
                for (int q = 0; q < RBG; ++q) {
                    if (rb0 + q >= RB) break;
                    const R ar = Ar(buf, ks + kq, q * 16 + (lane & 15));
                    const R ai = Ai(buf, ks + kq, q * 16 + (lane & 15));
#pragma unroll
                    for (int cb = 0; cb < NCB; ++cb) {
                        acc[q][cb] = Op::mma(ar, bv[cb], acc[q][cb]);
                        acc[q][cb] = Op::mma(ai, wv2[cb], acc[q][cb]);
                    }
                }
            }
            if (c + 1 < nch) {
                lstore(buf ^ 1);
                __syncthreads();
            }
        }
#pragma unroll
        for (int q = 0; q < RBG; ++q) {
            if (rb0 + q >= RB) break;
#pragma unroll
            for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int r = (rb0 + q) * 16 + Op::row(kq, i), nn = am + r;
                    if (r < rows) Wout[((int64_t)tile * P2 + nn * nn + nn + m) * NCOL + colw + 16 * cb] = acc[q][cb][i];
                }
        }
    }
}

// ------------------------------------------------------------------ fused translation tiles (p <= 16)
// All three stages for 32 (virtual) jobs of a 64-job tile in one workgroup.  The jobs' coefficient
// vectors stay in LDS (row c holds 32 jobs x real/imaginary part); each of the 4 wavefronts owns
// 16 columns (8 jobs) and transforms them in place on matrix cores -- forward rotation degree by
// degree, coaxial step order by order, back rotation degree by degree -- with no workgroup
// barrier between steps: every wavefront reads its own fragments of the step's table block from
// memory (L2-resident, shared by the tile's jobs) into registers, one step ahead.  HBM sees the
// source gather and the back-rotated rows (one per run of one target), not the work rows of the
// three-pass kernels.  psrc = ptgt = P <= TF_PMAX.
constexpr int TF_PMAX = 16, TF_PH = 2 * TF_PMAX - 1;
constexpr int TF_GU = 8;  // source loads in flight per thread

// Steps of the fused kernel: pairs of degrees (2k, 2k + 1) of the forward rotation, then the
// coaxial orders +-|m| (one table block serves both), then pairs of degrees of the back rotation;
// the two halves of a step are independent, so each wavefront keeps two matrix-core chains in
// flight.
//
// A fragments of one step for one lane: TfRot v[d][i][b] = A[16 b + (lane & 15)][4 i + (lane >> 4)]
// of the rotation block of degree 2k + d (b: row block); TfCoax v[i][b] the same entry of the
// coaxial block of |m| times (-1)^{k+r} (b = 0 real part, b = 1 imaginary part).  They come from
// tables stored in exactly this order (k_fr_rot, k_fr_coax: one contiguous value per lane, zero
// past each block), so a step's loads need no index arithmetic and its operands no masks; only
// the slots a step uses are loaded, one step before it.
template <class R> struct TfRot { R v[2][8][2]; };
template <class R> struct TfCoax { R v[4][2]; };

template <class R, int KS, int RB>
__device__ __forceinline__ void tf_load_rot_k(TfRot<R> &f, const R *M) {
#pragma unroll
    for (int d = 0; d < 2; ++d)
#pragma unroll
        for (int i = 0; i < KS; ++i)
#pragma unroll
            for (int b = 0; b < RB; ++b) f.v[d][i][b] = M[((d * 8 + i) * 2 + b) * 64];
}

// M: the class's fragment-order rotation table (of HT for the forward rotation, of H for the
// back rotation) offset by the lane; step k uses K chunks 0..k and row blocks 0..(k >= 4)
template <class R>
__device__ __forceinline__ void tf_load_rot(TfRot<R> &f, const R *M, int k) {
    M += (int64_t)k * TF_FR_STEP;
    switch (k) {
    case 0: tf_load_rot_k<R, 1, 1>(f, M); break;
    case 1: tf_load_rot_k<R, 2, 1>(f, M); break;
    case 2: tf_load_rot_k<R, 3, 1>(f, M); break;
    case 3: tf_load_rot_k<R, 4, 1>(f, M); break;
    case 4: tf_load_rot_k<R, 5, 2>(f, M); break;
    case 5: tf_load_rot_k<R, 6, 2>(f, M); break;
    case 6: tf_load_rot_k<R, 7, 2>(f, M); break;
    default: tf_load_rot_k<R, 8, 2>(f, M); break;
    }
}

template <class R, int KS>
__device__ __forceinline__ void tf_load_coax_k(TfCoax<R> &f, const R *T) {
#pragma unroll
    for (int i = 0; i < KS; ++i) {
        f.v[i][0] = T[(2 * i) * 64];
        f.v[i][1] = T[(2 * i + 1) * 64];
    }
}

// T: the class's fragment-order coaxial table offset by the lane; order |m| = am uses
// ceil((P - am) / 4) K chunks
template <class R>
__device__ __forceinline__ void tf_load_coax(TfCoax<R> &f, const R *T, int am, int P) {
    T += (int64_t)am * TF_FR_ORDER;
    switch ((P - am + 3) / 4) {
    case 1: tf_load_coax_k<R, 1>(f, T); break;
    case 2: tf_load_coax_k<R, 2>(f, T); break;
    case 3: tf_load_coax_k<R, 3>(f, T); break;
    default: tf_load_coax_k<R, 4>(f, T); break;
    }
}

// rotation of degrees n0 and n0 + 1 (if TWO; rows n^2 .. n^2 + 2n) on the wavefront's 16 columns,
// in place; KS K steps of 4 rows (the same for both degrees), RB row blocks of 16
template <class R, int LD, int KS, int RB, bool TWO>
__device__ __forceinline__ void tf_rot_pair(R *X, const TfRot<R> &f, int n0, int colw, int kq) {
    using Op = TmOp<R>;
    using v4 = typename Op::v4;
    constexpr int ND = TWO ? 2 : 1;
    R b[ND][KS];
#pragma unroll
    for (int d = 0; d < ND; ++d) {
        const int n = n0 + d, w = 2 * n + 1;
#pragma unroll
        for (int i = 0; i < KS; ++i) b[d][i] = X[(n * n + min(4 * i + kq, w - 1)) * LD + colw];  // A is 0 past w
    }
    v4 acc[ND][RB];
#pragma unroll
    for (int d = 0; d < ND; ++d)
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) acc[d][rb] = v4{0, 0, 0, 0};
#pragma unroll
    for (int i = 0; i < KS; ++i)
#pragma unroll
        for (int rb = 0; rb < RB; ++rb)
#pragma unroll
            for (int d = 0; d < ND; ++d) acc[d][rb] = Op::mma(f.v[d][i][rb], b[d][i], acc[d][rb]);
#pragma unroll
    for (int d = 0; d < ND; ++d) {
        const int n = n0 + d, w = 2 * n + 1;
#pragma unroll
        for (int rb = 0; rb < RB; ++rb)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int r = 16 * rb + Op::row(kq, i);
                if (r < w) X[(n * n + r) * LD + colw] = acc[d][rb][i];
            }
    }
}

// coaxial step of orders am and -am (if TWO) on the wavefront's 16 columns, in place: rows and
// columns are the degrees am .. P - 1 of the order; the imaginary part of the table meets the
// partner column (re <-> im)
template <class R, int LD, int KS, bool TWO>
__device__ __forceinline__ void tf_coax_pair(R *X, const TfCoax<R> &f, int am, int P, int colw, int kq, R swp) {
    using Op = TmOp<R>;
    using v4 = typename Op::v4;
    constexpr int ND = TWO ? 2 : 1;
    const int rows = P - am;
    R b[ND][KS], bw[ND][KS];
#pragma unroll
    for (int d = 0; d < ND; ++d) {
        const int m = d ? -am : am;
#pragma unroll
        for (int i = 0; i < KS; ++i) {
            const int nk = am + min(4 * i + kq, rows - 1), ck = nk * nk + nk + m;
            b[d][i] = X[ck * LD + colw];
            bw[d][i] = swp * X[ck * LD + (colw ^ 1)];
        }
    }
    v4 acc[ND];
#pragma unroll
    for (int d = 0; d < ND; ++d) acc[d] = v4{0, 0, 0, 0};
#pragma unroll
    for (int i = 0; i < KS; ++i)
#pragma unroll
        for (int d = 0; d < ND; ++d) {
            acc[d] = Op::mma(f.v[i][0], b[d][i], acc[d]);
            acc[d] = Op::mma(f.v[i][1], bw[d][i], acc[d]);
        }
#pragma unroll
    for (int d = 0; d < ND; ++d) {
        const int m = d ? -am : am;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int r = Op::row(kq, i), nn = am + r;
            if (r < rows) X[(nn * nn + nn + m) * LD + colw] = acc[d][i];
        }
    }
}

// rotation step k (degrees 2k, 2k + 1): K steps k + 1, two row blocks from degree 8 on
template <class R, int LD>
__device__ __forceinline__ void tf_rot_step(R *X, const TfRot<R> &f, int k, int P, int colw, int kq) {
    const int n0 = 2 * k;
    const bool two = n0 + 1 < P;
#define TF_ROT(KS, RB) \
    (two ? tf_rot_pair<R, LD, KS, RB, true>(X, f, n0, colw, kq) : tf_rot_pair<R, LD, KS, RB, false>(X, f, n0, colw, kq))
    switch (k) {
    case 0: TF_ROT(1, 1); break;
    case 1: TF_ROT(2, 1); break;
    case 2: TF_ROT(3, 1); break;
    case 3: TF_ROT(4, 1); break;
    case 4: TF_ROT(5, 2); break;
    case 5: TF_ROT(6, 2); break;
    case 6: TF_ROT(7, 2); break;
    default: TF_ROT(8, 2); break;
    }
#undef TF_ROT
}

template <class R, int LD>
__device__ __forceinline__ void tf_coax_step(R *X, const TfCoax<R> &f, int am, int P, int colw, int kq, R swp) {
    const int ks = (P - am + 3) / 4;
#define TF_COAX(KS) \
    (am > 0 ? tf_coax_pair<R, LD, KS, true>(X, f, am, P, colw, kq, swp) : tf_coax_pair<R, LD, KS, false>(X, f, am, P, colw, kq, swp))
    switch (ks) {
    case 1: TF_COAX(1); break;
    case 2: TF_COAX(2); break;
    case 3: TF_COAX(3); break;
    default: TF_COAX(4); break;
    }
#undef TF_COAX
}

// one rotation stage (all degree pairs) with the tables M; two fragment sets, each loaded one step
// before the step that uses it
template <class R, int LD>
__device__ __forceinline__ void tf_rot_stage(R *X, const R *M, int P, int colw, int kq) {
    const int QR = (P + 1) / 2;
    TfRot<R> fa, fb;
    tf_load_rot(fa, M, 0);
    for (int k = 0; k < QR; k += 2) {
        if (k + 1 < QR) tf_load_rot(fb, M, k + 1);
        tf_rot_step<R, LD>(X, fa, k, P, colw, kq);
        if (k + 2 < QR) tf_load_rot(fa, M, k + 2);
        if (k + 1 < QR) tf_rot_step<R, LD>(X, fb, k + 1, P, colw, kq);
    }
}

// J jobs per workgroup (J / 8 wavefronts): 16 (two workgroups share a CU in FP64) or 32 (runs of
// one target over 4 vectors span 32 virtual jobs)
template <class R, int J>
__global__ void __launch_bounds__(8 * J) k_tf_trans(TransArgsT<R> a) {
    using C = typename Cx<R>::T;
    constexpr int LD = 2 * J + 2, NT = 8 * J;
    __shared__ __align__(16) R X[TF_PMAX * TF_PMAX * LD];
    __shared__ C phl[J * TF_PH];  // e^{i m a_j}, m = -(P-1) .. P-1, per job
    __shared__ int64_t soff[J];
    __shared__ int32_t sdir[J];
    __shared__ int segl[J];
    int tile, part;
    xcd_block(tile, part);
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int64_t J0 = (int64_t)tile * LANE_JT + part * J;
    const int P = a.P, P2 = P * P, phs = 2 * a.PH + 1, nph = 2 * P - 1;
    if (tid < J) {
        const int64_t Jv = J0 + tid, Jc = Jv < a.njob ? Jv : a.njob - 1;
        soff[tid] = src_row(a, Jc) * P2;
        sdir[tid] = a.jdir[Jc / a.nr] * phs + a.PH - (P - 1);
        segl[tid] = Jv < a.njob ? a.jseg[Jv / a.nr] : 0;
    }
    __syncthreads();
    for (int e = tid; e < J * nph; e += NT) {
        const int j = e / nph, q = e - j * nph;
        phl[j * TF_PH + q] = a.ph[sdir[j] + q];
    }
    __syncthreads();
    // sources, phased: X[c][2j..2j+1] = e^{i m a_j} c_j  (coefficient c = n^2 + n + m); TF_GU loads
    // in flight per thread
    const int tot = J * P2;
    const float inv = 1.0f / (float)P2;
    // (indices past the end are clamped to the last element: those threads store the same value
    // to the same place, so no store is conditional and no load waits for a branch)
    for (int e0 = 0; e0 < tot; e0 += NT * TF_GU) {
        C s[TF_GU];
        int jj[TF_GU], cc[TF_GU];
#pragma unroll
        for (int u = 0; u < TF_GU; ++u) {
            const int e = min(e0 + tid + NT * u, tot - 1), j = (int)(((float)e + 0.5f) * inv);
            jj[u] = j;
            cc[u] = e - j * P2;
            s[u] = a.src[soff[j] + cc[u]];
        }
#pragma unroll
        for (int u = 0; u < TF_GU; ++u) {
            const int c = cc[u], n = (int)sqrtf((float)c + 0.5f), m = c - n * n - n;
            const C x = mulc(phl[jj[u] * TF_PH + m + P - 1], s[u]);
            X[c * LD + 2 * jj[u]] = x.x;
            X[c * LD + 2 * jj[u] + 1] = x.y;
        }
    }
    __syncthreads();
    {
        const int tr = a.tile_rot[tile / a.nr], tc = a.tile_coax[tile / a.nr];
        const R *HT = a.frHT + (int64_t)tr * TF_FR_ROT + lane, *H = a.frH + (int64_t)tr * TF_FR_ROT + lane;
        const R *T = a.frC + (int64_t)tc * TF_FR_COAX + lane;
        const int colw = 16 * wv + (lane & 15), kq = lane >> 4;
        const R swp = (colw & 1) ? R(1) : R(-1);
        tf_rot_stage<R, LD>(X, HT, P, colw, kq);
        {
            TfCoax<R> ca, cb;
            tf_load_coax(ca, T, 0, P);
            for (int am = 0; am < P; am += 2) {
                if (am + 1 < P) tf_load_coax(cb, T, am + 1, P);
                tf_coax_step<R, LD>(X, ca, am, P, colw, kq, swp);
                if (am + 2 < P) tf_load_coax(ca, T, am + 2, P);
                if (am + 1 < P) tf_coax_step<R, LD>(X, cb, am + 1, P, colw, kq, swp);
            }
        }
        tf_rot_stage<R, LD>(X, H, P, colw, kq);
    }
    __syncthreads();
    // back-rotated rows, phased (e^{-i m a}) and summed over the runs of one target, job-major
    for (int e = tid; e < tot; e += NT) {
        const int j = (int)(((float)e + 0.5f) * inv), c = e - j * P2, len = segl[j];
        if (len == 0) continue;
        const int n = (int)sqrtf((float)c + 0.5f), m = c - n * n - n;
        C v = mkc<C>(0, 0);
        for (int t = 0; t < len; ++t) {
            const int jj = j + t * a.nr;
            v = addc(v, mulcc(mkc<C>(X[c * LD + 2 * jj], X[c * LD + 2 * jj + 1]), phl[jj * TF_PH + m + P - 1]));
        }
        a.W1[(J0 + j) * (int64_t)P2 + c] = v;
    }
}

// ------------------------------------------------------------------ register-resident RCR tiles (FP64, p = 16)
// One wavefront takes 8 (virtual) jobs of one class and keeps their coefficient vectors in registers
// through the three stages: 16 columns (job j = column / 2, real or imaginary part by the column's
// parity), every vector of length w in the quad layout of the matrix cores -- element e in register
// e / 4 of lane group e % 4 (lanes 16 g .. 16 g + 15).  That is at once the layout of the B operand of
// v_mfma_f64_16x16x4f64 (K chunk e / 4, row g) and of its D output (rows 4 i + g), so a rotation's
// outputs feed the next product where they are.  Between the rotations and the coaxial step the
// vectors change from degree order (degree n: orders m = -n .. n) to order order (order m: degrees
// |m| .. p - 1) and back; each element stays in its lane group or moves to the opposite one (g ^ 2),
// so a change of layout is a select by lane group and at most one exchange between the two halves of
// the wavefront.  LDS holds the jobs' phase factors and one degree of outputs on its way to the run
// sums.  The tables are the fused tiles' fragment-order tables (one contiguous value per lane).
constexpr int TQ_P = 16;

template <class F, int... I>
__device__ __forceinline__ void tq_for_impl(F &&f, std::integer_sequence<int, I...>) {
    (f(std::integral_constant<int, I>{}), ...);
}
// f(integral_constant<int, i>) for i = 0 .. N-1, every index a compile-time constant (register arrays)
template <int N, class F> __device__ __forceinline__ void tq_for(F &&f) {
    tq_for_impl(f, std::make_integer_sequence<int, N>{});
}
// registers of degree n (2n + 1 elements) and of order m (p - |m| elements) in the quad layout
__host__ __device__ constexpr int tq_dreg(int n) { return (n + 2) / 2; }
__host__ __device__ constexpr int tq_doff(int n) {
    int s = 0;
    for (int q = 0; q < n; ++q) s += tq_dreg(q);
    return s;
}
__host__ __device__ constexpr int tq_oreg(int m) { return (TQ_P - (m < 0 ? -m : m) + 3) / 4; }
__host__ __device__ constexpr int tq_ooff(int m) {
    int s = 0;
    for (int q = -(TQ_P - 1); q < m; ++q) s += tq_oreg(q);
    return s;
}
constexpr int TQ_ND = tq_doff(TQ_P), TQ_NO = tq_ooff(TQ_P);
static_assert(TQ_ND == 72 && TQ_NO == 76, "quad-layout register counts");

// value of lane group g among four per-group candidates
__device__ __forceinline__ double tq_sel(bool g1, bool g2, double a0, double a1, double a2, double a3) {
    return g2 ? (g1 ? a3 : a2) : (g1 ? a1 : a0);
}
// the value of the partner column (lane ^ 1: the other part of the same job), DPP quad permutation
__device__ __forceinline__ double tq_swap_pair(double v) {
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), 0xB1, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), 0xB1, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}
// the value of lane l ^ 32 (lane group g ^ 2, same column)
__device__ __forceinline__ double tq_swap_halves(double v, int lane) {
    const int addr = (lane ^ 32) << 2;
    const int lo = __builtin_amdgcn_ds_bpermute(addr, __double2loint(v));
    const int hi = __builtin_amdgcn_ds_bpermute(addr, __double2hiint(v));
    return __hiloint2double(hi, lo);
}

// element (n = |m| + 4 s + g, m) of the degree layout for lane group g (K chunk s of order m)
template <int M, int S>
__device__ __forceinline__ double tq_to_order(const double (&X)[TQ_ND], bool g1, bool g2, int lane) {
    constexpr int AM = M < 0 ? -M : M;
    auto cand = [&](auto gI) -> double {
        constexpr int n = AM + 4 * S + decltype(gI)::value;
        if constexpr (n < TQ_P) return X[tq_doff(n) + ((n + M) >> 2)];
        else return 0.0;
    };
    using I0 = std::integral_constant<int, 0>;
    using I1 = std::integral_constant<int, 1>;
    using I2 = std::integral_constant<int, 2>;
    using I3 = std::integral_constant<int, 3>;
    if constexpr (((AM + M) & 3) == 0) {
        // row n + m of degree n lies in lane group g itself
        return tq_sel(g1, g2, cand(I0{}), cand(I1{}), cand(I2{}), cand(I3{}));
    } else {
        // odd m > 0: it lies in lane group g ^ 2, which selects what its partner group needs
        return tq_swap_halves(tq_sel(g1, g2, cand(I2{}), cand(I3{}), cand(I0{}), cand(I1{})), lane);
    }
}

// element (n, m = 4 s + g - n) of the order layout for lane group g (K chunk s of degree n)
template <int N, int S>
__device__ __forceinline__ double tq_to_degree(const double (&Y)[TQ_NO], bool g1, bool g2, int lane) {
    // source of lane group G: order m, row k = n - |m| in lane group k % 4, register k / 4
    auto valid = [](int G) { return 4 * S + G <= 2 * N; };
    auto grp = [](int G) {
        const int m = 4 * S + G - N, k = N - (m < 0 ? -m : m);
        return k & 3;
    };
    auto val = [&](auto GI) -> double {  // the source element of lane group G, read where it lies
        constexpr int G = decltype(GI)::value, m = 4 * S + G - N, k = N - (m < 0 ? -m : m);
        if constexpr (4 * S + G <= 2 * N) return Y[tq_ooff(m) + (k >> 2)];
        else return 0.0;
    };
    using I0 = std::integral_constant<int, 0>;
    using I1 = std::integral_constant<int, 1>;
    using I2 = std::integral_constant<int, 2>;
    using I3 = std::integral_constant<int, 3>;
    constexpr bool own0 = !valid(0) || grp(0) == 0, own1 = !valid(1) || grp(1) == 1;
    constexpr bool own2 = !valid(2) || grp(2) == 2, own3 = !valid(3) || grp(3) == 3;
    // lane group G keeps its own candidate when that lies in G, else takes what G ^ 2 gives it
    const double mine = tq_sel(g1, g2, own0 ? val(I0{}) : 0.0, own1 ? val(I1{}) : 0.0, own2 ? val(I2{}) : 0.0,
                               own3 ? val(I3{}) : 0.0);
    if constexpr (own0 && own1 && own2 && own3) {
        return mine;
    } else {
        // lane group H gives the candidate of group H ^ 2 when that lies in H
        const double give = tq_sel(g1, g2, own2 ? 0.0 : val(I2{}), own3 ? 0.0 : val(I3{}), own0 ? 0.0 : val(I0{}),
                                   own1 ? 0.0 : val(I1{}));
        const double got = tq_swap_halves(give, lane);
        return tq_sel(g1, g2, own0 ? mine : got, own1 ? mine : got, own2 ? mine : got, own3 ? mine : got);
    }
}

// sum of a value over the run of one target that starts at this column's job (runs never cross the
// wavefront's 8 jobs): segmented sums over the columns 2 (j + t) + part, t < len, by three shifts
// of 2, 4 and 8 columns within the lane group (DPP row shifts); end = first job past the run
__device__ __forceinline__ double tq_dpp_shl(double v, int ctrl_sel) {
    int lo = __double2loint(v), hi = __double2hiint(v);
    switch (ctrl_sel) {  // row_shl:2 / 4 / 8 (lane i takes lane i + d of its row of 16; 0 past the row)
    case 2: lo = __builtin_amdgcn_update_dpp(0, lo, 0x102, 0xF, 0xF, true), hi = __builtin_amdgcn_update_dpp(0, hi, 0x102, 0xF, 0xF, true); break;
    case 4: lo = __builtin_amdgcn_update_dpp(0, lo, 0x104, 0xF, 0xF, true), hi = __builtin_amdgcn_update_dpp(0, hi, 0x104, 0xF, 0xF, true); break;
    default: lo = __builtin_amdgcn_update_dpp(0, lo, 0x108, 0xF, 0xF, true), hi = __builtin_amdgcn_update_dpp(0, hi, 0x108, 0xF, 0xF, true);
    }
    return __hiloint2double(hi, lo);
}
// md = 1 where column c + d still belongs to column c's run, else 0 (multipliers: one FMA per shift
// instead of a select and an add)
__device__ __forceinline__ double tq_run_sum(double v, double m2, double m4, double m8) {
    double s = v;
    s = fma(tq_dpp_shl(s, 2), m2, s);
    s = fma(tq_dpp_shl(s, 4), m4, s);
    s = fma(tq_dpp_shl(s, 8), m8, s);
    return s;
}

// A fragments of the rotation of degree n (K chunks x row blocks), one value per lane
template <int N, class T>
__device__ __forceinline__ void tq_load_rot(T (&A)[16], const T *F) {
    constexpr int KS = tq_dreg(N), RB = (2 * N + 16) / 16;
    tq_for<RB>([&](auto bI) {
        tq_for<KS>([&](auto iI) {
            constexpr int b = decltype(bI)::value, i = decltype(iI)::value;
            A[b * 8 + i] = F[((N * 8 + i) * 2 + b) * 64];
        });
    });
}
// rotation of degree n on the quad-layout vector B (tq_dreg(n) registers) into acc (row blocks)
template <int N>
__device__ __forceinline__ void tq_rotate(const double (&A)[16], const double *B, TmOp<double>::v4 (&acc)[2]) {
    using v4 = TmOp<double>::v4;
    constexpr int KS = tq_dreg(N), RB = (2 * N + 16) / 16;
    tq_for<RB>([&](auto bI) { acc[decltype(bI)::value] = v4{0, 0, 0, 0}; });
    tq_for<KS>([&](auto iI) {
        tq_for<RB>([&](auto bI) {
            constexpr int b = decltype(bI)::value, i = decltype(iI)::value;
            acc[b] = TmOp<double>::mma(A[b * 8 + i], B[i], acc[b]);
        });
    });
}

// one wavefront = 8 jobs of a 64-job tile (grid: tiles x 8); one right-hand side; psrc = ptgt = P = PT = 16.
// OCC: waves per SIMD the register allocation is held to.  The table fragments of a step are loaded
// one step (for small degrees several) ahead of the step that uses them.
template <int OCC>
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(OCC, OCC))) k_tq_rcr(TransArgsT<double> a) {
    using v4 = TmOp<double>::v4;
    constexpr int P = TQ_P, P2 = P * P, NPH = 2 * P - 1;
    // e^{i m a_j}, m = -(P-1) .. P-1, with the imaginary part negated ([0]) or not ([1]): the
    // phase of a complex value held as (re, im) in partner columns is then fma(e.x, x, e.y * y) for
    // either part (x its own value, y the partner's), with no select on the part
    __shared__ double2 phg[2][8][NPH];
    __shared__ int64_t soff[8];
    __shared__ int sgend[8];  // per job: first job past the run it belongs to (within the wavefront)
    __shared__ int segl[8];
    int tile, part;
    xcd_block(tile, part);
    const int64_t J0 = (int64_t)tile * LANE_JT + part * 8;
    if (J0 >= a.njob) return;  // the whole workgroup (one wavefront)
    const int lane = threadIdx.x, g = lane >> 4, col = lane & 15, jl = col >> 1, im = col & 1;
    const bool g1 = (g & 1) != 0, g2 = (g & 2) != 0;
    const int phs = 2 * a.PH + 1;
    if (lane < 8) {
        const int64_t Jv = J0 + lane, Jc = Jv < a.njob ? Jv : a.njob - 1;
        soff[lane] = (int64_t)a.jsrc[Jc] * P2;
        segl[lane] = Jv < a.njob ? a.jseg[Jv] : 0;
    }
    for (int e = lane; e < 8 * NPH; e += 64) {
        const int j = e / NPH, q = e - j * NPH;
        const int64_t Jv = J0 + j, Jc = Jv < a.njob ? Jv : a.njob - 1;
        const double2 ph = a.ph[(int64_t)a.jdir[Jc] * phs + a.PH - (P - 1) + q];
        phg[1][j][q] = ph;
        phg[0][j][q] = make_double2(ph.x, -ph.y);
    }
    __syncthreads();
    if (lane < 8) {
        // run of job `lane`: it starts at the nearest start at or before it (runs are contiguous)
        int st = lane;
        while (st > 0 && segl[st] == 0) --st;
        sgend[lane] = segl[st] > 0 ? st + segl[st] : lane + 1;
    }
    const int tr = a.tile_rot[tile], tc = a.tile_coax[tile];
    const double *FF = a.frHT + (int64_t)tr * TF_FR_ROT + lane;  // forward: H (from HT's fragments)
    const double *FB = a.frH + (int64_t)tr * TF_FR_ROT + lane;   // back: H^T
    const double *FC = a.frC + (int64_t)tc * TF_FR_COAX + lane;
    double AF[P][16];  // rotation fragments per degree (only the live ones take registers)
    double TF[P][8];   // coaxial fragments per order |m|: 4 K chunks x (re, im)

    // sources in the degree layout; the fragments of the small degrees loaded behind them
    double X[TQ_ND];
    {
        const double *s = (const double *)a.src + 2 * soff[jl] + im;
        tq_for<P>([&](auto nI) {
            constexpr int n = decltype(nI)::value;
            tq_for<tq_dreg(n)>([&](auto sI) {
                constexpr int q = decltype(sI)::value;
                const int r = 4 * q + g;
                const double v = s[2 * (n * n + min(r, 2 * n))];  // clamped: no masked load
                X[tq_doff(n) + q] = r <= 2 * n ? v : 0.0;
            });
        });
        tq_for<4>([&](auto nI) { tq_load_rot<decltype(nI)::value>(AF[decltype(nI)::value], FF); });
        __syncthreads();  // sgend
        tq_for<P>([&](auto nI) {
            constexpr int n = decltype(nI)::value;
            tq_for<tq_dreg(n)>([&](auto sI) {
                constexpr int q = decltype(sI)::value;
                const int r = min(4 * q + g, 2 * n);
                const double x = X[tq_doff(n) + q], y = tq_swap_pair(x);
                const double2 e = phg[im][jl][r - n + P - 1];  // e: re x_r - im x_i, re x_i + im x_r
                X[tq_doff(n) + q] = fma(e.x, x, e.y * y);
            });
        });
    }
    const int end2 = 2 * sgend[jl];
    const bool starts = segl[jl] > 0;
    const double rm2 = col + 2 < end2 ? 1.0 : 0.0, rm4 = col + 4 < end2 ? 1.0 : 0.0, rm8 = col + 8 < end2 ? 1.0 : 0.0;
    // forward rotation, degree by degree: Y_n = H_n X_n
    tq_for<P>([&](auto nI) {
        constexpr int n = decltype(nI)::value;
        __builtin_amdgcn_sched_barrier(0);
        if constexpr (n >= 3 && n + 1 < P) tq_load_rot<n + 1>(AF[n + 1], FF);
        if constexpr (n == P - 1) {
            tq_for<2>([&](auto aI) {
                constexpr int am = decltype(aI)::value;
                tq_for<tq_oreg(am)>([&](auto iI) {
                    constexpr int i = decltype(iI)::value;
                    TF[am][2 * i] = FC[((am * 4 + i) * 2) * 64];
                    TF[am][2 * i + 1] = FC[((am * 4 + i) * 2 + 1) * 64];
                });
            });
        }
        v4 acc[2];
        tq_rotate<n>(AF[n], &X[tq_doff(n)], acc);
        tq_for<tq_dreg(n)>([&](auto sI) {
            constexpr int q = decltype(sI)::value;
            X[tq_doff(n) + q] = acc[q / 4][q % 4];
        });
    });
    // coaxial step, order pair by order pair (one table block for +-|m|), into the order layout
    double Y[TQ_NO];
    {
        const double swp = im ? 1.0 : -1.0;
        tq_for<P>([&](auto aI) {
            constexpr int am = decltype(aI)::value, KS = tq_oreg(am);
            __builtin_amdgcn_sched_barrier(0);
            if constexpr (am + 2 < P) {
                tq_for<tq_oreg(am + 2)>([&](auto iI) {
                    constexpr int i = decltype(iI)::value;
                    TF[am + 2][2 * i] = FC[(((am + 2) * 4 + i) * 2) * 64];
                    TF[am + 2][2 * i + 1] = FC[(((am + 2) * 4 + i) * 2 + 1) * 64];
                });
            }
            if constexpr (am == P - 3) tq_load_rot<P - 1>(AF[P - 1], FB);
            tq_for<(am > 0 ? 2 : 1)>([&](auto sgI) {
                constexpr int m = decltype(sgI)::value == 0 ? am : -am;
                double B[KS], Bw[KS];
                tq_for<KS>([&](auto sI) {
                    constexpr int q = decltype(sI)::value;
                    B[q] = tq_to_order<m, q>(X, g1, g2, lane);
                    Bw[q] = swp * tq_swap_pair(B[q]);
                });
                v4 acc = v4{0, 0, 0, 0};
                tq_for<KS>([&](auto iI) {
                    constexpr int i = decltype(iI)::value;
                    acc = TmOp<double>::mma(TF[am][2 * i], B[i], acc);
                    acc = TmOp<double>::mma(TF[am][2 * i + 1], Bw[i], acc);
                });
                tq_for<KS>([&](auto qI) {
                    constexpr int q = decltype(qI)::value;
                    Y[tq_ooff(m) + q] = acc[q];
                });
            });
        });
    }
    // back rotation, degree by degree from the largest: H_n^T, then e^{-i m a} and the run sums of
    // one target; the runs' first jobs store their rows (job-major, for the per-target reduction)
    double *const orow = (double *)(a.W1 + (J0 + jl) * (int64_t)P2 + g) + im;  // element r = 4 q + g: 2 (n^2 + 4 q)
    tq_for<P>([&](auto dI) {
        constexpr int n = P - 1 - decltype(dI)::value, KS = tq_dreg(n), w = 2 * n + 1;
        __builtin_amdgcn_sched_barrier(0);  // one degree's outputs at a time (register pressure)
        if constexpr (n - 1 >= 7) tq_load_rot<n - 1>(AF[n - 1], FB);
        if constexpr (n == 8) tq_for<7>([&](auto kI) { tq_load_rot<decltype(kI)::value>(AF[decltype(kI)::value], FB); });
        double B[KS];
        tq_for<KS>([&](auto sI) {
            constexpr int q = decltype(sI)::value;
            B[q] = tq_to_degree<n, q>(Y, g1, g2, lane);
        });
        v4 acc[2];
        tq_rotate<n>(AF[n], B, acc);
        tq_for<KS>([&](auto qI) {
            constexpr int q = decltype(qI)::value;
            const int r = 4 * q + g, rc = min(r, 2 * n);
            const double x = acc[q / 4][q % 4], y = tq_swap_pair(x);
            const double2 e = phg[1 - im][jl][rc - n + P - 1];  // conj(e)
            const double v = tq_run_sum(fma(e.x, x, e.y * y), rm2, rm4, rm8);
            if (starts && r < w) orow[2 * (n * n + 4 * q)] = v;
        });
    });
}

// The same fused translation with the vectors in LDS (p = 16, FP64 and FP32, any number of
// right-hand sides: a workgroup per vector): one workgroup = 8 jobs (CB = 1) or 16 jobs (CB = 2:
// two 16-column blocks, each table fragment feeding two products) of a 64-job tile as in k_tq_rcr, but the jobs' vectors live in LDS (256
// coefficients x 16 columns: 33 KB in FP64, 16 KB in FP32) instead of registers, shared by NW
// wavefronts that take the degrees (orders) n = h mod NW each.  Every step reads its B operands
// from LDS in the matrix-core layout (K row 4 i + g of chunk i in lane group g), the partner column
// (the other part of a job) included, and writes its outputs back in place in the output layout of
// the instruction (rows g + 4 i in FP64, 4 g + i in FP32, of a 16-row block), so that the changes
// between degree and order order are only addresses: no selects, no exchanges between lanes.  The
// phases of the sources and, after the back rotation, the conjugate phases and the sums over each
// target's run are taken with each lane owning coefficients (both parts of a job read from LDS at
// once); only the runs' first jobs do the sums.  Tables: the fragment-order tables of the fused
// tiles.  Measured at levels 6-7 of the 1M L-room: FP32 (mixed products) 2.77 ms with one
// wavefront per workgroup and the partner moves of k_tq_rcr, 2.27 ms with lanes owning
// coefficients in the first and last steps, 1.70 ms with two wavefronts, 1.71 -> 1.70 with four;
// FP64 3.29 ms in registers (k_tq_rcr, two wavefronts per SIMD), 2.88 ms here with four.

template <class R, int NW, int CB>
__global__ void __launch_bounds__(64 * NW) k_tq_lds(TransArgsT<R> a) {
    using C = typename Cx<R>::T;
    using Op = TmOp<R>;
    using v4 = typename Op::v4;
    // CB blocks of 8 jobs (16 columns) per workgroup: every table fragment feeds CB products
    constexpr int P = TQ_P, P2 = P * P, NPH = 2 * P - 1, NJ = 8 * CB, JW = NJ / NW;
    static_assert(NW == 2 || NW == 4, "two or four wavefronts per workgroup");
    static_assert(CB == 1 || CB == 2, "one or two column blocks");
    // coefficient (n, m) at row n^2 + n + m, column 2 job + part; rows P2 .. P2 + 3 (zeros) are read
    // past the last degree.  Reads need no branch: rows past a degree or order meet zero columns of
    // the table block (without the branches the reads of a step issue together: 2.58 -> 2.27 ms at
    // levels 6-7 of the 1M L-room); writes past a block stay masked (writing them to spare rows
    // nearly doubles the LDS stores and was slower)
    __shared__ R Xs[CB][P2 + 4][16];
    __shared__ C phg[NJ][NPH];  // e^{i m a_j}
    __shared__ int64_t soff[NJ];
    __shared__ int segl[NJ];
    int tile, part;
    xcd_block(tile, part);
    // several right-hand sides: virtual tile t holds vector t % nr of the 64 real jobs of tile t / nr
    // (a workgroup takes 8 CB real jobs of one vector, so a run of one target stays in its LDS)
    const int nr = a.nr, rt = tile / nr, rv = tile - rt * nr;
    const int64_t nj = a.njob / nr, J0 = (int64_t)rt * LANE_JT + part * NJ;
    if (J0 >= nj) return;  // the whole workgroup
    // NW wavefronts share the 8 jobs' vectors: wavefront h takes the degrees (orders) n = h mod NW of
    // every step, and the jobs JW h .. JW h + JW - 1 of the first and last steps
    const int tid = threadIdx.x, lane = tid & 63, h = tid >> 6, g = lane >> 4, col = lane & 15, im = col & 1;
    const int phs = 2 * a.PH + 1;
    if (tid < NJ) {
        const int64_t Jv = J0 + tid, Jc = Jv < nj ? Jv : nj - 1;
        soff[tid] = ((int64_t)a.jsrc[Jc] * nr + rv) * P2;  // sources: nr vectors per box
        segl[tid] = Jv < nj ? a.jseg[Jv] : 0;
    }
    if (h < CB) Xs[h][P2 + g][col] = R(0);
    for (int e = tid; e < NJ * NPH; e += 64 * NW) {
        const int j = e / NPH, q = e - j * NPH;
        const int64_t Jv = J0 + j, Jc = Jv < nj ? Jv : nj - 1;
        phg[j][q] = a.ph[(int64_t)a.jdir[Jc] * phs + a.PH - (P - 1) + q];
    }
    __syncthreads();
    const int tr = a.tile_rot[rt], tc = a.tile_coax[rt];
    const R *FF = a.frHT + (int64_t)tr * TF_FR_ROT + lane;  // forward: H (from HT's fragments)
    const R *FB = a.frH + (int64_t)tr * TF_FR_ROT + lane;   // back: H^T
    const R *FC = a.frC + (int64_t)tc * TF_FR_COAX + lane;
    // lane l owns coefficients e = l + 64 u (u < 4) in the first and last steps; their orders m
    int mo[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int e = lane + 64 * u;
        int n = (int)sqrtf((float)e);
        n -= n * n > e;
        n += (n + 1) * (n + 1) <= e;
        mo[u] = e - n * n - n;
    }
    // sources times e^{i m a}, one job after the other (64 consecutive coefficients per load)
#pragma unroll
    for (int jj = 0; jj < JW; ++jj) {
        const int j = JW * h + jj, cb = j >> 3, jl = j & 7;
        const C *src = a.src + soff[j];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int e = lane + 64 * u;
            const C x = src[e], ph = phg[j][mo[u] + P - 1];
            Xs[cb][e][2 * jl] = ph.x * x.x - ph.y * x.y;  // scalar accesses only (no type punning of Xs)
            Xs[cb][e][2 * jl + 1] = ph.x * x.y + ph.y * x.x;
        }
    }
    // rotation of degree n on the rows of Xs, in place
    auto rotate = [&](auto nI, const R (&A)[16]) {
        constexpr int n = decltype(nI)::value, KS = tq_dreg(n), RB = (2 * n + 16) / 16, w = 2 * n + 1;
        R B[CB][KS];
        tq_for<CB>([&](auto cI) {
            tq_for<KS>([&](auto iI) {
                constexpr int c = decltype(cI)::value, i = decltype(iI)::value;
                B[c][i] = Xs[c][n * n + 4 * i + g][col];  // past the degree: the next one's rows, zero columns of A
            });
        });
        v4 acc[CB][RB];
        tq_for<CB>([&](auto cI) {
            tq_for<RB>([&](auto bI) { acc[decltype(cI)::value][decltype(bI)::value] = v4{0, 0, 0, 0}; });
        });
        tq_for<KS>([&](auto iI) {
            tq_for<RB>([&](auto bI) {
                tq_for<CB>([&](auto cI) {
                    constexpr int b = decltype(bI)::value, i = decltype(iI)::value, c = decltype(cI)::value;
                    acc[c][b] = Op::mma(A[b * 8 + i], B[c][i], acc[c][b]);
                });
            });
        });
        tq_for<CB>([&](auto cI) {
            tq_for<RB>([&](auto bI) {
                constexpr int c = decltype(cI)::value, b = decltype(bI)::value;
                tq_for<4>([&](auto iI) {
                    constexpr int i = decltype(iI)::value;
                    const int r = 16 * b + Op::row(g, i);
                    if (r < w) Xs[c][n * n + r][col] = acc[c][b][i];
                });
            });
        });
    };
    // the steps of one residue H (mod NW): forward rotation of its degrees, coaxial step of its
    // orders, back rotation of its degrees; table fragments one step (of the same residue) ahead
    R AF[P][16];  // rotation fragments per degree (only the live ones take registers)
    R TF[P][8];   // coaxial fragments per order |m|: 4 K chunks x (re, im)
    auto forward = [&](auto HI) {
        constexpr int H = decltype(HI)::value;
        tq_for<4 / NW>([&](auto qI) {
            constexpr int n = H + NW * decltype(qI)::value;
            tq_load_rot<n>(AF[n], FF);
        });
        tq_for<P / NW>([&](auto kI) {
            constexpr int n = NW * decltype(kI)::value + H;
            if constexpr (n + 4 < P) tq_load_rot<n + 4>(AF[n + 4], FF);
            if constexpr (n + NW >= P) {  // this residue's first order of the coaxial step
                tq_for<tq_oreg(H)>([&](auto iI) {
                    constexpr int i = decltype(iI)::value;
                    TF[H][2 * i] = FC[((H * 4 + i) * 2) * 64];
                    TF[H][2 * i + 1] = FC[((H * 4 + i) * 2 + 1) * 64];
                });
            }
            rotate(std::integral_constant<int, n>{}, AF[n]);
        });
    };
    auto coax = [&](auto HI) {
        constexpr int H = decltype(HI)::value;
        const R swp = im ? R(1) : R(-1);
        tq_for<P / NW>([&](auto kI) {
            constexpr int am = NW * decltype(kI)::value + H, KS = tq_oreg(am), rows = P - am;
            if constexpr (am + NW < P) {
                tq_for<tq_oreg(am + NW)>([&](auto iI) {
                    constexpr int i = decltype(iI)::value;
                    TF[am + NW][2 * i] = FC[(((am + NW) * 4 + i) * 2) * 64];
                    TF[am + NW][2 * i + 1] = FC[(((am + NW) * 4 + i) * 2 + 1) * 64];
                });
            }
            tq_for<(am > 0 ? 2 : 1)>([&](auto sgI) {
                constexpr int m = decltype(sgI)::value == 0 ? am : -am;
                R B[CB][KS], Bw[CB][KS];
                tq_for<CB>([&](auto cI) {
                    tq_for<KS>([&](auto iI) {
                        constexpr int c = decltype(cI)::value, i = decltype(iI)::value;
                        // degrees past 15 read degree 15's row: zero columns of the table block
                        const int nn = min(am + 4 * i + g, P - 1), row = nn * nn + nn + m;
                        // X': column 2j holds -Im x_j, column 2j+1 holds Re x_j (the partner column)
                        B[c][i] = Xs[c][row][col];
                        Bw[c][i] = swp * Xs[c][row][col ^ 1];
                    });
                });
                v4 acc[CB];
                tq_for<CB>([&](auto cI) { acc[decltype(cI)::value] = v4{0, 0, 0, 0}; });
                tq_for<KS>([&](auto iI) {
                    tq_for<CB>([&](auto cI) {
                        constexpr int c = decltype(cI)::value, i = decltype(iI)::value;
                        acc[c] = Op::mma(TF[am][2 * i], B[c][i], acc[c]);
                    });
                    tq_for<CB>([&](auto cI) {
                        constexpr int c = decltype(cI)::value, i = decltype(iI)::value;
                        acc[c] = Op::mma(TF[am][2 * i + 1], Bw[c][i], acc[c]);
                    });
                });
                tq_for<CB>([&](auto cI) {
                    tq_for<4>([&](auto iI) {
                        constexpr int c = decltype(cI)::value, i = decltype(iI)::value;
                        const int r = Op::row(g, i), nn = am + r;
                        if (r < rows) Xs[c][nn * nn + nn + m][col] = acc[c][i];
                    });
                });
            });
        });
    };
    auto back = [&](auto HI) {
        constexpr int H = decltype(HI)::value, N0 = P - NW + H;  // this residue's largest degree
        tq_load_rot<N0>(AF[N0], FB);
        tq_for<P / NW>([&](auto kI) {
            constexpr int n = N0 - NW * decltype(kI)::value;
            if constexpr (n - NW >= 8) tq_load_rot<n - NW>(AF[n - NW], FB);
            if constexpr (n >= 8 && n - NW < 8)  // the rest of this residue's degrees
                tq_for<8 / NW>([&](auto qI) {
                    constexpr int k = NW * decltype(qI)::value + H;
                    tq_load_rot<k>(AF[k], FB);
                });
            rotate(std::integral_constant<int, n>{}, AF[n]);
        });
    };
    // each stage's residues under separate tests of h (compiled as one if / else chain, the back
    // rotation's matrix instructions were dropped from the code: the products then differ)
    auto stage = [&](auto f) {
        tq_for<NW>([&](auto HI) {
            if (h == decltype(HI)::value) f(HI);
        });
    };
    __syncthreads();  // Xs
    stage(forward);
    __syncthreads();
    stage(coax);
    __syncthreads();
    stage(back);
    __syncthreads();
    // e^{-i m a} and the sums over the runs of one target: each run's first job stores its row
    // (job-major, for the per-target reduction), lane l the coefficients l + 64 u
#pragma unroll 1
    for (int jj = 0; jj < JW; ++jj) {
        const int j = JW * h + jj, len = segl[j], cb = j >> 3, jl = j & 7;  // runs stay in 8-job blocks
        if (len == 0) continue;  // uniform: not a run's first job
        C *orow = a.W1 + ((J0 + j) * nr + rv) * (int64_t)P2;  // the row of virtual job (J0 + j) nr + rv
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int e = lane + 64 * u;
            R sx = R(0), sy = R(0);
            for (int t = 0; t < len; ++t) {
                const R xr = Xs[cb][e][2 * (jl + t)], xi = Xs[cb][e][2 * (jl + t) + 1];
                const C ph = phg[j + t][mo[u] + P - 1];
                sx += ph.x * xr + ph.y * xi;  // conj(e) x
                sy += ph.x * xi - ph.y * xr;
            }
            orow[e] = mkc<C>(sx, sy);
        }
    }
}

static_assert(TF_FR_STEP == 2 * 8 * 2 * 64 && TF_FR_ROT == (TF_PMAX / 2) * TF_FR_STEP, "rotation fragment layout");
static_assert(TF_FR_ORDER == 4 * 2 * 64 && TF_FR_COAX == TF_PMAX * TF_FR_ORDER, "coaxial fragment layout");

// Fragment-order rotation tables: element (class, k, d, i, b, lane) = A[16 b + lane % 16][4 i + lane / 16]
// of degree n = 2k + d of the class's table M (A[r][q] = M[rot_block_off(n) + q (2n + 1) + r]),
// zero past the block or for n >= P.
__global__ void __launch_bounds__(256) k_fr_rot(int64_t ntot, int P, const double *M, double *out) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= ntot) return;
    const int64_t cl = e / TF_FR_ROT;
    const int rem = (int)(e - cl * TF_FR_ROT);
    const int lane = rem & 63, b = (rem >> 6) & 1, i = (rem >> 7) & 7, d = (rem >> 10) & 1, k = rem >> 11;
    const int n = 2 * k + d, r = 16 * b + (lane & 15), q = 4 * i + (lane >> 4);
    double v = 0.0;
    if (n < P && r < 2 * n + 1 && q < 2 * n + 1)
        v = M[cl * rot_table_size(P) + rot_block_off(n) + (int64_t)q * (2 * n + 1) + r];
    out[e] = v;
}

// Fragment-order coaxial tables: element (class, am, i, part, lane) = (-1)^{q+r} (re or im of)
// T[q][r] of order |m| = am, q = 4 i + lane / 16 (source degree - am), r = lane % 16 (target
// degree - am), zero past the block (P - am rows and columns).
__global__ void __launch_bounds__(256) k_fr_coax(int64_t ntot, int P, int PT, const double2 *T, double *out) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= ntot) return;
    const int64_t cl = e / TF_FR_COAX;
    const int rem = (int)(e - cl * TF_FR_COAX);
    const int lane = rem & 63, part = (rem >> 6) & 1, i = (rem >> 7) & 3, am = rem >> 9;
    const int rows = P - am, q = 4 * i + (lane >> 4), r = lane & 15;
    double v = 0.0;
    if (am < P && q < rows && r < rows) {
        const double2 t = T[cl * coax_table_size(PT) + coax_block_off(PT, am) + (int64_t)q * (PT - am) + r];
        v = ((q + r) & 1 ? -1.0 : 1.0) * (part ? t.y : t.x);
    }
    out[e] = v;
}

// dst[t] (+)= sum of the job rows of target t (W1, P^2 per job); jobs of t listed in CSR order.
// With nr vectors, virtual target t is real target t / nr, vector t % nr, and the job rows of
// that vector are (job * nr + t % nr).  Workgroup (t, y) takes coefficients 256 y .. 256 y + 255
// of target t, so that the large expansions of the upper levels spread over many workgroups.
// Without acc the sums overwrite dst, targets without jobs included (the batch writes every
// target: no clearing of dst beforehand).  Rows are loaded eight at a time (a partial group
// included), all in flight together.
template <class C>
__global__ void __launch_bounds__(256) k_tr_reduce(int64_t ntgt, int nr, int ptgt, int P, const int32_t *start,
                                                   const int32_t *jobs, const C *W, C *dst, int acc) {
    const int64_t t = blockIdx.x;
    if (t >= ntgt * nr) return;
    const int64_t tr = t / nr;
    const int r = (int)(t - tr * nr);
    const int j0 = start[tr], j1 = start[tr + 1];
    if (j0 == j1 && acc) return;
    const int pt2 = ptgt * ptgt;
    const int64_t P2 = (int64_t)P * P;
    const int c = blockIdx.y * 256 + threadIdx.x;
    if (c >= pt2) return;
    C s[8];
    s[0] = acc ? dst[t * pt2 + c] : mkc<C>(0, 0);
#pragma unroll
    for (int u = 1; u < 8; ++u) s[u] = mkc<C>(0, 0);
    for (int q = j0; q < j1; q += 8) {  // a target has ~5-8 rows: the last group is partial, not serial
        C a[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) a[u] = q + u < j1 ? W[((int64_t)jobs[q + u] * nr + r) * P2 + c] : mkc<C>(0, 0);
#pragma unroll
        for (int u = 0; u < 8; ++u) s[u] = addc(s[u], a[u]);
    }
    dst[t * pt2 + c] = addc(addc(addc(s[0], s[1]), addc(s[2], s[3])), addc(addc(s[4], s[5]), addc(s[6], s[7])));
}

// ------------------------------------------------------------------ host side
int trans_fused_pmax() { return TF_PMAX; }
int trans_rcr_p() { return TQ_P; }

// H, HT: nbeta rotation tables of degree < P; coax: ncoax coaxial tables of size PT; outputs hold
// max(1, nbeta) TF_FR_ROT and max(1, ncoax) TF_FR_COAX values
void build_fused_tables(int P, int PT, int nbeta, const double *H, const double *HT, int ncoax, const double2 *coax,
                        double *frH, double *frHT, double *frC, hipStream_t st) {
    if (P > TF_PMAX || PT < P) throw FmmError(-1, "fragment-order tables need p <= 16 and PT >= p");
    const int64_t nr = (int64_t)std::max(1, nbeta) * TF_FR_ROT, nc = (int64_t)std::max(1, ncoax) * TF_FR_COAX;
    k_fr_rot<<<(unsigned)((nr + 255) / 256), 256, 0, st>>>(nr, P, H, frH);
    LAUNCH_OK();
    k_fr_rot<<<(unsigned)((nr + 255) / 256), 256, 0, st>>>(nr, P, HT, frHT);
    LAUNCH_OK();
    k_fr_coax<<<(unsigned)((nc + 255) / 256), 256, 0, st>>>(nc, P, PT, coax, frC);
    LAUNCH_OK();
}

int trans_pick_jt(int P, size_t lds_budget, int whole) {
    const size_t per = whole ? sizeof(double2) * (size_t)P * P : sizeof(double2) * (size_t)std::max(2 * P - 1, P);
    int jt = (int)std::min<size_t>(64, lds_budget / per);
    jt = std::max(RJ, jt - jt % RJ);
    return jt;
}

size_t trans_lds_bytes(int JT, int P, int whole) {
    return whole ? sizeof(double2) * (size_t)JT * P * P : sizeof(double2) * (size_t)JT * std::max(2 * P - 1, P);
}

void trans_configure_lds(size_t lds_max) {
    const void *f[] = {(const void *)k_tr_rot_fwd<double>, (const void *)k_tr_coax<double>,
                       (const void *)k_tr_rot_back<double>, (const void *)k_tw_rot<double, true>,
                       (const void *)k_tw_rot<double, false>, (const void *)k_tw_coax<double>,
                       (const void *)k_tr_rot_fwd<float>, (const void *)k_tr_coax<float>,
                       (const void *)k_tr_rot_back<float>, (const void *)k_tw_rot<float, true>,
                       (const void *)k_tw_rot<float, false>, (const void *)k_tw_coax<float>};
    for (auto fn : f) HIP_OK(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_max));
}

// One stage of a batch: 0 forward rotation, 1 coaxial step, 2 back rotation, 3 reduction into
// the targets.  Returns the HIP kernel's name (for profiling).
template <class R>
const char *trans_stage(const TransBatch &b, const TransTables<R> &tb, int stage, int nr, const typename Cx<R>::T *src,
                        typename Cx<R>::T *dst, const typename Cx<R>::T *ph, int PH, typename Cx<R>::T *W1,
                        typename Cx<R>::T *W2, hipStream_t st, bool accumulate) {
    if (nr < 1 || b.JT % nr) throw FmmError(-1, "right-hand-side count must divide the tile size");
    TransArgsT<R> a{b.njob * nr, b.JT, b.psrc, b.ptgt, b.P, b.PT, PH, nr, src, dst, b.src, b.tgt, b.dir,
                    b.tile_coax, b.tile_rot, tb.coax, tb.H, tb.HT, ph, W1, W2, b.seg, tb.frH, tb.frHT, tb.frC};
    // classes are padded to whole tiles of JT real jobs, so a tile of JT virtual jobs never
    // mixes tables: virtual tile t uses the tables of real tile t / nr
    const unsigned ntile = (unsigned)((b.njob * nr + b.JT - 1) / b.JT);
    // LDS sized for the scalar type
    const size_t lds = trans_lds_bytes(b.JT, b.P, b.whole) / (sizeof(double) / sizeof(R));
    const bool f32 = sizeof(R) == 4;
    const char *name = "";
    if constexpr (sizeof(R) == 8) {
        if (b.lane && b.mfma >= 3 && stage < 3 && (nr == 1 || b.mfma == 4) && b.P == TQ_P) {
            // register-resident fused tiles: FP64, p = 16 (mode 3 one vector, mode 4 any count)
            if (b.JT != LANE_JT || b.psrc != b.ptgt || b.PT != b.P)
                throw FmmError(-1, "register-resident translation tiles need 64-job tiles and p_src = p_tgt = 16");
            if (!tb.frH || !tb.frHT || !tb.frC)
                throw FmmError(-1, "fused translation tiles need their fragment-order tables");
            if (stage != 0) return nullptr;
            // mode 3: vectors in registers (one wavefront per SIMD); mode 4: vectors in LDS shared by
            // four wavefronts (levels 6-7 of the 1M L-room: 3.29 ms with the vectors in registers at
            // two wavefronts per SIMD, 2.88 ms in LDS)
            if (b.mfma == 3) k_tq_rcr<1><<<dim3(ntile, LANE_JT / 8), 64, 0, st>>>(a);
            else k_tq_lds<double, 4, 1><<<dim3(ntile, LANE_JT / 8), 256, 0, st>>>(a);
            LAUNCH_OK();
            return b.mfma == 3 ? "k_tq_rcr" : "k_tq_lds";
        }
    }
    if constexpr (sizeof(R) == 4) {
        if (b.lane && b.mfma >= 3 && stage < 3 && b.P == TQ_P) {
            // register-resident shape in FP32 (mixed products): vectors in LDS
            if (b.JT != LANE_JT || b.psrc != b.ptgt || b.PT != b.P)
                throw FmmError(-1, "register-resident translation tiles need 64-job tiles and p_src = p_tgt = 16");
            if (!tb.frH || !tb.frHT || !tb.frC)
                throw FmmError(-1, "fused translation tiles need their fragment-order tables");
            if (stage != 0) return nullptr;
            // two column blocks: 16 jobs per workgroup (37 KB of LDS, four workgroups per CU); in
            // FP64 two blocks (75 KB, two workgroups per CU) measured slower than one (3.30 against
            // 2.92 ms at levels 6-7 of the 1M L-room), in FP32 the mixed product 6.93 -> 6.73 ms
            k_tq_lds<float, 4, 2><<<dim3(ntile, LANE_JT / 16), 256, 0, st>>>(a);
            LAUNCH_OK();
            return "k_tq_lds_f32";
        }
    }
    if (b.lane && b.mfma >= 2 && stage < 3) {
        // the fused LDS-resident kernel (and mode 3 with several vectors, where it takes its place)
        // the fused kernel takes the three stages at stage 0
        // a run of one target (at most SEG_ALIGN real jobs, aligned) lies in one workgroup's jobs
        if (b.JT != LANE_JT || b.psrc != b.ptgt || b.PT != b.P || b.P > TF_PMAX || 32 / nr < SEG_ALIGN)
            throw FmmError(-1, "fused translation tiles need 64-job tiles, p_src = p_tgt <= 16, <= 4 vectors");
        if (!tb.frH || !tb.frHT || !tb.frC) throw FmmError(-1, "fused translation tiles need their fragment-order tables");
        if (stage != 0) return nullptr;
        if (16 / nr >= SEG_ALIGN)
            k_tf_trans<R, 16><<<dim3(ntile, LANE_JT / 16), 128, 0, st>>>(a);
        else
            k_tf_trans<R, 32><<<dim3(ntile, LANE_JT / 32), 256, 0, st>>>(a);
        LAUNCH_OK();
        return f32 ? "k_tf_trans_f32" : "k_tf_trans";
    }
    if (b.lane && b.mfma == 1 && stage < 3) {
        // stages of a lane batch on matrix cores (FP64, or FP32 for mixed products), tiles of 64 or
        // 32 jobs
        if (b.JT != LANE_JT && b.JT != LANE_JT / 2) throw FmmError(-1, "matrix-core tiles take 64 or 32 jobs");
        // A small batch (few workgroups per CU) also spreads the row groups of a degree (order)
        // over workgroups, so that the largest degrees do not run as one long workgroup each.
        auto passes = [&](int rows, int rbg, int nd) {
            const int np = ((rows + 15) / 16 + rbg - 1) / rbg;
            return (int64_t)ntile * nd >= 2048 ? 1 : np;
        };
        int np;
        switch (stage) {
        case 0:
            np = passes(2 * b.psrc - 1, 4, b.psrc);
            if (b.JT == LANE_JT) k_tm_rot<R, true, 4, 64><<<dim3(ntile, b.psrc * np), 256, 0, st>>>(a, np);
            else k_tm_rot<R, true, 4, 32><<<dim3(ntile, b.psrc * np), 256, 0, st>>>(a, np);
            name = f32 ? "k_tm_rot_fwd_f32" : "k_tm_rot_fwd";
            break;
        case 1:
            np = passes(b.ptgt, 4, 2 * b.ptgt - 1);
            // 64-row passes, K chunks of 8: 33 KB of LDS, four workgroups per CU
            if (b.JT == LANE_JT) k_tm_coax<R, 64, 4, 8><<<dim3(ntile, (2 * b.ptgt - 1) * np), 256, 0, st>>>(a, np);
            else k_tm_coax<R, 32, 4, 8><<<dim3(ntile, (2 * b.ptgt - 1) * np), 256, 0, st>>>(a, np);
            name = f32 ? "k_tm_coax_f32" : "k_tm_coax";
            break;
        default:
            np = passes(2 * b.ptgt - 1, 4, b.ptgt);
            if (b.JT == LANE_JT) k_tm_rot<R, false, 4, 64><<<dim3(ntile, b.ptgt * np), 256, 0, st>>>(a, np);
            else k_tm_rot<R, false, 4, 32><<<dim3(ntile, b.ptgt * np), 256, 0, st>>>(a, np);
            name = f32 ? "k_tm_rot_back_f32" : "k_tm_rot_back";
        }
        LAUNCH_OK();
        return name;
    }
    if (b.lane && stage < 3) {
        if (b.JT != LANE_JT) throw FmmError(-1, "lane batches use 64-job tiles");
        // enough wavefronts to cover the device: split degrees/orders over blockIdx.y
        const int nd = stage == 1 ? 2 * b.ptgt - 1 : (stage == 0 ? b.psrc : b.ptgt);
        const int ns = (int)std::max<int64_t>(1, std::min<int64_t>(nd, (4096 + ntile - 1) / std::max(1u, ntile)));
        const dim3 grid(ntile, ns);
        // Row chunks of up to 32 rows for the rotations (a whole degree up to p = 16) and 16 for
        // the coaxial step (a whole order up to p = 16), so that the inputs are read once per
        // degree or order; FP32 rows are small enough to double-buffer the table in scalar registers.
        constexpr bool PF = sizeof(R) == 4;
        switch (stage) {
        case 0: k_tl_rot_fwd<R, PF><<<grid, 64, 0, st>>>(a, ns), name = f32 ? "k_tl_rot_fwd_f32" : "k_tl_rot_fwd"; break;
        case 1: k_tl_coax<R, PF><<<grid, 64, 0, st>>>(a, ns), name = f32 ? "k_tl_coax_f32" : "k_tl_coax"; break;
        default:
            k_tl_rot_back<R, PF><<<grid, 64, 0, st>>>(a, ns), name = f32 ? "k_tl_rot_back_f32" : "k_tl_rot_back";
        }
        LAUNCH_OK();
        return name;
    }
    switch (stage) {
    case 0:
        if (b.whole) k_tw_rot<R, true><<<ntile, 256, lds, st>>>(a), name = f32 ? "k_tw_rot_fwd_f32" : "k_tw_rot_fwd";
        else k_tr_rot_fwd<R><<<dim3(ntile, b.psrc), 256, lds, st>>>(a), name = f32 ? "k_tr_rot_fwd_f32" : "k_tr_rot_fwd";
        break;
    case 1:
        if (b.whole) k_tw_coax<R><<<ntile, 256, lds, st>>>(a), name = f32 ? "k_tw_coax_f32" : "k_tw_coax";
        else k_tr_coax<R><<<dim3(ntile, 2 * b.P - 1), 256, lds, st>>>(a), name = f32 ? "k_tr_coax_f32" : "k_tr_coax";
        break;
    case 2:
        if (b.whole) k_tw_rot<R, false><<<ntile, 256, lds, st>>>(a), name = f32 ? "k_tw_rot_back_f32" : "k_tw_rot_back";
        else k_tr_rot_back<R><<<dim3(ntile, b.ptgt), 256, lds, st>>>(a), name = f32 ? "k_tr_rot_back_f32" : "k_tr_rot_back";
        break;
    default:
        k_tr_reduce<typename Cx<R>::T><<<dim3((unsigned)(b.ntgt * nr), (unsigned)ceil_div(b.ptgt * b.ptgt, 256)), 256, 0,
                                         st>>>(b.ntgt, nr, b.ptgt, b.P, b.tgt_start, b.tgt_jobs, W1, dst, accumulate ? 1 : 0);
        name = f32 ? "k_tr_reduce_f32" : "k_tr_reduce";
    }
    LAUNCH_OK();
    return name;
}

template const char *trans_stage<double>(const TransBatch &, const TransTables<double> &, int, int, const double2 *,
                                         double2 *, const double2 *, int, double2 *, double2 *, hipStream_t, bool);
template const char *trans_stage<float>(const TransBatch &, const TransTables<float> &, int, int, const float2 *, float2 *,
                                        const float2 *, int, float2 *, float2 *, hipStream_t, bool);

}  // namespace fmm
