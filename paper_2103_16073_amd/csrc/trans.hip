// Rotation - coaxial translation - back-rotation (Section 3.3) for tiles of translations.
//
// A translation job moves one expansion (multipole of a source box, or local of a parent) into
// another frame: coefficient vectors are rotated so that the translation vector t points along
// +z, translated coaxially by |t| (block-diagonal in m), rotated back, and added into the target.
// Jobs are grouped in tiles of JT jobs that share |t|, so every table entry read from memory is
// used JT times: the rotation matrices Delta^n are shared by all jobs (only the z-rotation phases
// differ per direction) and the coaxial block (E|F)^{|m|} by all jobs of the tile.
//
//  k_trans_fused : the JT coefficient vectors stay in LDS through all three steps (p up to the
//                  LDS budget); the result is accumulated into the target with FP64 atomics.
//  k_stage_rot / k_stage_coax : the same steps for large p, one step per launch, vectors in a
//                  global work buffer (one row of P^2 coefficients per job), per-degree (or
//                  per-order) slices of the tile staged in LDS.
//
// Rotation conventions (see fmm.hip): forward  c <- A_m c, Delta^T, B_m, Delta;
//                                     back     Delta^T, conj(B_m), Delta, conj(A_m)
// with A_m = e^{i m alpha} (-i)^m and B_m = e^{i m beta} tabulated per direction.
#include "internal.h"

namespace fmm {

struct TransArgs {
    int64_t njob;
    int JT, psrc, ptgt, P, PT, PH;
    const double2 *src;      // source expansions (psrc^2 per box)
    double2 *dst;            // target expansions (ptgt^2 per box), accumulated
    const int32_t *jsrc, *jtgt;  // per job; jtgt < 0 marks padding
    const int16_t *jdir;
    const int32_t *tile_tab;     // table index per tile
    const double2 *tables;       // coaxial tables, coax_table_size(PT) each
    const double2 *phA, *phB;    // per-direction phases, 2*PH+1 per direction
    const double *D, *DT;        // Delta^n and its transpose
};

__device__ inline int isqrt_c(int c) {
    int n = (int)sqrtf((float)c);
    while (n * n > c) --n;
    while ((n + 1) * (n + 1) <= c) ++n;
    return n;
}

// out[j][mp] = phase(j, mp) * sum_m Dn[m][mp] in[j][m], for j < nj, mp < w.
// in/out are LDS slices with per-job strides is/os; Dn is the row-major (2n+1)^2 block.
template <bool CONJ>
__device__ inline void rot_half(int nj, int w, int n, const double *Dn, const double2 *in, int is, double2 *out, int os,
                                const double2 *ph, int phs, const int16_t *dirs, int PH) {
    for (int e = threadIdx.x; e < nj * w; e += blockDim.x) {
        const int j = e / w, mp = e - j * w;
        const double2 *x = in + j * is;
        double sr = 0.0, si = 0.0;
#pragma unroll 4
        for (int m = 0; m < w; ++m) {
            const double d = Dn[m * w + mp];
            const double2 v = x[m];
            sr = fma(d, v.x, sr);
            si = fma(d, v.y, si);
        }
        double2 s = cmk(sr, si);
        if (ph) {
            const double2 f = ph[(int64_t)dirs[j] * phs + PH + (mp - n)];
            s = CONJ ? cmulc(s, f) : cmul(s, f);
        }
        out[j * os + mp] = s;
    }
}

// Register-blocked variant: each thread produces column mp for R jobs, so every table value read
// (from LDS here) feeds 2R fused multiply-adds.
template <bool CONJ, int R>
__device__ inline void rot_half_b(int nj, int w, int n, const double *Dn, const double2 *in, int is, double2 *out,
                                  int os, const double2 *ph, int phs, const int16_t *dirs, int PH) {
    const int ngrp = (nj + R - 1) / R;
    for (int e = threadIdx.x; e < ngrp * w; e += blockDim.x) {
        const int g = e / w, mp = e - g * w;
        const double2 *x[R];
        double sr[R], si[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            x[r] = in + min(g * R + r, nj - 1) * is;
            sr[r] = 0.0;
            si[r] = 0.0;
        }
        for (int m = 0; m < w; ++m) {
            const double d = Dn[m * w + mp];
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const double2 v = x[r][m];
                sr[r] = fma(d, v.x, sr[r]);
                si[r] = fma(d, v.y, si[r]);
            }
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int j = g * R + r;
            if (j >= nj) break;
            double2 s = cmk(sr[r], si[r]);
            if (ph) {
                const double2 f = ph[(int64_t)dirs[j] * phs + PH + (mp - n)];
                s = CONJ ? cmulc(s, f) : cmul(s, f);
            }
            out[j * os + mp] = s;
        }
    }
}

// ------------------------------------------------------------------ fused kernel
__global__ void __launch_bounds__(256) k_trans_fused(TransArgs a) {
    extern __shared__ double2 lds[];
    const int JT = a.JT, P2 = a.P * a.P, TW = 2 * a.P;
    double2 *X = lds;                 // JT * P2
    double2 *tmp = X + JT * P2;       // JT * TW
    double *DL = (double *)(tmp + JT * TW);  // Delta^n and its transpose, (2P-1)^2 each
    const int DW = (2 * a.P - 1) * (2 * a.P - 1);
    __shared__ int16_t sdir[64];
    __shared__ int32_t stgt[64];
    const int64_t t0 = (int64_t)blockIdx.x * JT;
    const int nj = (int)min((int64_t)JT, a.njob - t0);
    const int ps2 = a.psrc * a.psrc, pt2 = a.ptgt * a.ptgt;
    const int phs = 2 * a.PH + 1;
    for (int j = threadIdx.x; j < nj; j += blockDim.x) {
        sdir[j] = a.jdir[t0 + j];
        stgt[j] = a.jtgt[t0 + j];
    }
    __syncthreads();
    // gather with the first phase A_m
    for (int e = threadIdx.x; e < nj * P2; e += blockDim.x) {
        const int j = e / P2, c = e - j * P2;
        double2 v = cmk(0, 0);
        if (c < ps2) {
            const int n = isqrt_c(c), m = c - n * n - n;
            v = cmul(a.phA[(int64_t)sdir[j] * phs + a.PH + m], a.src[(int64_t)a.jsrc[t0 + j] * ps2 + c]);
        }
        X[j * P2 + c] = v;
    }
    __syncthreads();
    // forward rotation
    for (int n = 0; n < a.psrc; ++n) {
        const int w = 2 * n + 1;
        for (int e = threadIdx.x; e < w * w; e += blockDim.x) {
            DL[e] = a.D[rot_block_off(n) + e];
            DL[DW + e] = a.DT[rot_block_off(n) + e];
        }
        __syncthreads();
        rot_half_b<false, 4>(nj, w, n, DL, X + n * n, P2, tmp, TW, a.phB, phs, sdir, a.PH);
        __syncthreads();
        rot_half_b<false, 4>(nj, w, n, DL + DW, tmp, TW, X + n * n, P2, nullptr, 0, sdir, a.PH);
        __syncthreads();
    }
    // coaxial translation, order by order (in place through tmp)
    const double2 *T = a.tables + (int64_t)a.tile_tab[blockIdx.x] * coax_table_size(a.PT);
    const int pm = min(a.psrc, a.ptgt);
    for (int m = -(pm - 1); m <= pm - 1; ++m) {
        const int am = m < 0 ? -m : m;
        const int rows = a.ptgt - am, B = a.PT - am;
        const double2 *Tm = T + coax_block_off(a.PT, am);
        constexpr int R = 4;
        const int ngrp = (nj + R - 1) / R;
        for (int e = threadIdx.x; e < ngrp * rows; e += blockDim.x) {
            const int g = e / rows, nn = am + (e - g * rows);
            const double2 *x[R];
            double sr[R], si[R];
#pragma unroll
            for (int r = 0; r < R; ++r) {
                x[r] = X + min(g * R + r, nj - 1) * P2;
                sr[r] = 0.0;
                si[r] = 0.0;
            }
            for (int n = am; n < a.psrc; ++n) {
                double2 t = Tm[(n - am) * B + (nn - am)];
                if ((n + nn) & 1) t = cmk(-t.x, -t.y);
                const int c = n * n + n + m;
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const double2 v = x[r][c];
                    sr[r] = fma(t.x, v.x, fma(-t.y, v.y, sr[r]));
                    si[r] = fma(t.x, v.y, fma(t.y, v.x, si[r]));
                }
            }
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const int j = g * R + r;
                if (j < nj) tmp[j * TW + nn] = cmk(sr[r], si[r]);
            }
        }
        __syncthreads();
        for (int e = threadIdx.x; e < nj * rows; e += blockDim.x) {
            const int j = e / rows, nn = am + (e - j * rows);
            X[j * P2 + nn * nn + nn + m] = tmp[j * TW + nn];
        }
        __syncthreads();
    }
    // back rotation
    for (int n = 0; n < a.ptgt; ++n) {
        const int w = 2 * n + 1;
        for (int e = threadIdx.x; e < w * w; e += blockDim.x) {
            DL[e] = a.D[rot_block_off(n) + e];
            DL[DW + e] = a.DT[rot_block_off(n) + e];
        }
        __syncthreads();
        rot_half_b<true, 4>(nj, w, n, DL, X + n * n, P2, tmp, TW, a.phB, phs, sdir, a.PH);
        __syncthreads();
        rot_half_b<true, 4>(nj, w, n, DL + DW, tmp, TW, X + n * n, P2, a.phA, phs, sdir, a.PH);
        __syncthreads();
    }
    // accumulate into the targets
    for (int e = threadIdx.x; e < nj * pt2; e += blockDim.x) {
        const int j = e / pt2, c = e - j * pt2;
        const int t = stgt[j];
        if (t < 0) continue;
        const double2 v = X[j * P2 + c];
        double *d = (double *)(a.dst + (int64_t)t * pt2 + c);
        unsafeAtomicAdd(d, v.x);
        unsafeAtomicAdd(d + 1, v.y);
    }
}

// ------------------------------------------------------------------ staged kernels (large p)
// Rotation of one degree n (= blockIdx.y) for a tile of jobs.  forward: gather from a.src (phase
// A) -> W (row P^2 per job).  back: W -> atomically into a.dst (final phase conj(A)).
__global__ void __launch_bounds__(256) k_stage_rot(TransArgs a, int forward, const double2 *Win, double2 *Wout) {
    extern __shared__ double2 lds[];
    const int JT = a.JT, TW = 2 * a.P, P2 = a.P * a.P;
    double2 *xs = lds, *tmp = lds + JT * TW;
    __shared__ int16_t sdir[64];
    __shared__ int32_t stgt[64];
    __shared__ int32_t ssrc[64];
    const int n = blockIdx.y;
    if (n >= (forward ? a.psrc : a.ptgt)) return;
    const int64_t t0 = (int64_t)blockIdx.x * JT;
    const int nj = (int)min((int64_t)JT, a.njob - t0);
    const int phs = 2 * a.PH + 1;
    const int ps2 = a.psrc * a.psrc, pt2 = a.ptgt * a.ptgt;
    for (int j = threadIdx.x; j < nj; j += blockDim.x) {
        sdir[j] = a.jdir[t0 + j];
        stgt[j] = a.jtgt[t0 + j];
        ssrc[j] = a.jsrc[t0 + j];
    }
    __syncthreads();
    const int w = 2 * n + 1;
    for (int e = threadIdx.x; e < nj * w; e += blockDim.x) {
        const int j = e / w, m = e - j * w - n;
        double2 v;
        if (forward)
            v = cmul(a.phA[(int64_t)sdir[j] * phs + a.PH + m], a.src[(int64_t)ssrc[j] * ps2 + n * n + n + m]);
        else
            v = Win[(t0 + j) * (int64_t)P2 + n * n + n + m];
        xs[j * TW + m + n] = v;
    }
    __syncthreads();
    if (forward) {
        rot_half_b<false, 4>(nj, w, n, a.D + rot_block_off(n), xs, TW, tmp, TW, a.phB, phs, sdir, a.PH);
        __syncthreads();
        rot_half_b<false, 4>(nj, w, n, a.DT + rot_block_off(n), tmp, TW, xs, TW, nullptr, 0, sdir, a.PH);
    } else {
        rot_half_b<true, 4>(nj, w, n, a.D + rot_block_off(n), xs, TW, tmp, TW, a.phB, phs, sdir, a.PH);
        __syncthreads();
        rot_half_b<true, 4>(nj, w, n, a.DT + rot_block_off(n), tmp, TW, xs, TW, a.phA, phs, sdir, a.PH);
    }
    __syncthreads();
    for (int e = threadIdx.x; e < nj * w; e += blockDim.x) {
        const int j = e / w, m = e - j * w - n;
        const double2 v = xs[j * TW + m + n];
        if (forward) {
            Wout[(t0 + j) * (int64_t)P2 + n * n + n + m] = v;
        } else {
            const int t = stgt[j];
            if (t >= 0) {
                double *d = (double *)(a.dst + (int64_t)t * pt2 + n * n + n + m);
                unsafeAtomicAdd(d, v.x);
                unsafeAtomicAdd(d + 1, v.y);
            }
        }
    }
}

// Coaxial step of one order m = blockIdx.y - (P-1) for a tile: Wout rows (ptgt^2 valid) from Win
// rows (psrc^2 valid); orders |m| >= min(psrc, ptgt) have no source and are written as zero.
__global__ void __launch_bounds__(256) k_stage_coax(TransArgs a, const double2 *Win, double2 *Wout) {
    extern __shared__ double2 lds[];
    const int JT = a.JT, TW = 2 * a.P, P2 = a.P * a.P;
    double2 *col = lds;  // JT * TW
    const int m = (int)blockIdx.y - (a.P - 1);
    const int am = m < 0 ? -m : m;
    if (am >= a.ptgt) return;
    const int64_t t0 = (int64_t)blockIdx.x * JT;
    const int nj = (int)min((int64_t)JT, a.njob - t0);
    const int pm = min(a.psrc, a.ptgt);
    const int rows = a.ptgt - am;
    if (am >= pm) {
        for (int e = threadIdx.x; e < nj * rows; e += blockDim.x) {
            const int j = e / rows, nn = am + (e - j * rows);
            Wout[(t0 + j) * (int64_t)P2 + nn * nn + nn + m] = cmk(0, 0);
        }
        return;
    }
    const double2 *T = a.tables + (int64_t)a.tile_tab[blockIdx.x] * coax_table_size(a.PT);
    const int B = a.PT - am;
    const double2 *Tm = T + coax_block_off(a.PT, am);
    const int cin = a.psrc - am;
    for (int e = threadIdx.x; e < nj * cin; e += blockDim.x) {
        const int j = e / cin, n = am + (e - j * cin);
        col[j * TW + n] = Win[(t0 + j) * (int64_t)P2 + n * n + n + m];
    }
    __syncthreads();
    for (int e = threadIdx.x; e < nj * rows; e += blockDim.x) {
        const int j = e / rows, nn = am + (e - j * rows);
        const double2 *x = col + j * TW;
        double sr = 0.0, si = 0.0;
        for (int n = am; n < a.psrc; ++n) {
            const double2 t = Tm[(int64_t)(n - am) * B + (nn - am)];
            const double2 v = x[n];
            const double sg = ((n + nn) & 1) ? -1.0 : 1.0;
            sr = fma(sg, t.x * v.x - t.y * v.y, sr);
            si = fma(sg, t.x * v.y + t.y * v.x, si);
        }
        Wout[(t0 + j) * (int64_t)P2 + nn * nn + nn + m] = cmk(sr, si);
    }
}

// ------------------------------------------------------------------ host side
static size_t fused_table_bytes(int P) { return sizeof(double) * 2 * (size_t)(2 * P - 1) * (2 * P - 1); }

size_t trans_lds_bytes(int fused, int JT, int P) {
    return fused ? sizeof(double2) * (size_t)JT * ((size_t)P * P + 2 * P) + fused_table_bytes(P)
                 : sizeof(double2) * (size_t)JT * 4 * P;
}

int trans_pick_jt(int fused, int P, size_t lds_max) {
    const size_t fixed = fused ? fused_table_bytes(P) : 0;
    if (lds_max <= fixed) return 0;
    const size_t per = fused ? sizeof(double2) * ((size_t)P * P + 2 * P) : sizeof(double2) * 4 * (size_t)P;
    int jt = (int)std::min<size_t>(64, (lds_max - fixed) / per);
    if (!fused) jt = std::min(jt, 64);
    return jt;
}

void trans_configure_lds(size_t lds_max) {
    HIP_OK(hipFuncSetAttribute((const void *)k_trans_fused, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_max));
    HIP_OK(hipFuncSetAttribute((const void *)k_stage_rot, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_max));
    HIP_OK(hipFuncSetAttribute((const void *)k_stage_coax, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_max));
}

void trans_launch(const TransBatch &b, const double2 *src, double2 *dst, const double2 *tables, const double2 *phA,
                  const double2 *phB, int PH, const double *D, const double *DT, double2 *W1, double2 *W2,
                  hipStream_t st) {
    if (b.njob == 0) return;
    TransArgs a{b.njob, b.JT, b.psrc, b.ptgt, b.P, b.PT, PH, src, dst, b.src, b.tgt, b.dir, b.tile_tab, tables,
                phA, phB, D, DT};
    const unsigned ntile = (unsigned)((b.njob + b.JT - 1) / b.JT);
    if (b.fused) {
        k_trans_fused<<<ntile, 256, trans_lds_bytes(1, b.JT, b.P), st>>>(a);
        LAUNCH_OK();
    } else {
        k_stage_rot<<<dim3(ntile, b.psrc), 256, trans_lds_bytes(0, b.JT, b.P), st>>>(a, 1, nullptr, W1);
        LAUNCH_OK();
        k_stage_coax<<<dim3(ntile, 2 * b.P - 1), 256, (size_t)sizeof(double2) * b.JT * 2 * b.P, st>>>(a, W1, W2);
        LAUNCH_OK();
        k_stage_rot<<<dim3(ntile, b.ptgt), 256, trans_lds_bytes(0, b.JT, b.P), st>>>(a, 0, W2, nullptr);
        LAUNCH_OK();
    }
}

}  // namespace fmm
