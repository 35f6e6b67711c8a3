// Learned preconditioner: a small MLP applied per chunk of up to 64 consecutive unknowns of one
// octree leaf, on top of the near-field block inverse.  FGMRES admits it because its
// preconditioner may change from step to step (Section 4.3 uses flexible GMRES).
//
//   input  (140): the chunk's residual divided by its norm (64 complex, zero padded), k times
//                 the leaf side, occupancy, mean and spread of the element normals, mean
//                 admittance, a constant 1
//   layers       : 140 -> 128 -> 128 -> 128 (ReLU) -> 128 (linear)
//   output (128): correction d (64 complex); z = P_near(v) + |v_chunk| d on the chunk
//
// Weights are kept in FP32 (training master copy) and FP16 (forward); every product
// accumulates in FP32.  Training minimises the mean squared distance between the output and
// (e - P_near r) / |r| on the chunk, for residual/error pairs (r, e) of the plain solver.
#include "internal.h"

#include <hip/hip_fp16.h>

namespace fmm {

// ------------------------------------------------------------------ features and application
// chunk c covers tree-order unknowns [cs[c], cs[c] + cn[c]) of leaf cl[c]
__global__ void __launch_bounds__(64) k_mlp_features(int64_t nchunk, const int32_t *cs, const int32_t *cn,
                                                     const int32_t *cl, const int32_t *perm, const double2 *v,
                                                     const double4 *en, const double2 *beta, const double *leaf_ka,
                                                     float *X, float *scale) {
    const int64_t c = blockIdx.x;
    if (c >= nchunk) return;
    const int tid = threadIdx.x, s = cs[c], cnt = cn[c];
    __shared__ double red[64];
    __shared__ double acc[10][64];
    double2 val = cmk(0, 0);
    double4 nv = make_double4(0, 0, 0, 0);
    double2 bt = cmk(0, 0);
    if (tid < cnt) {
        val = v[perm[s + tid]];
        nv = en[s + tid];
        bt = beta[s + tid];
    }
    red[tid] = val.x * val.x + val.y * val.y;
    const double q[10] = {nv.x, nv.y, nv.z, nv.x * nv.x, nv.y * nv.y, nv.z * nv.z, sqrt(bt.x * bt.x + bt.y * bt.y),
                          bt.x, bt.y, 0.0};
    for (int i = 0; i < 10; ++i) acc[i][tid] = q[i];
    __syncthreads();
    for (int w = 32; w > 0; w >>= 1) {
        if (tid < w) {
            red[tid] += red[tid + w];
            for (int i = 0; i < 9; ++i) acc[i][tid] += acc[i][tid + w];
        }
        __syncthreads();
    }
    const double nrm = sqrt(red[0]);
    const double inv = nrm > 0 ? 1.0 / nrm : 0.0;
    float *x = X + c * MLP_IN;
    x[2 * tid] = (float)(val.x * inv);
    x[2 * tid + 1] = (float)(val.y * inv);
    if (tid == 0) {
        const double ic = 1.0 / cnt;
        const double mx = acc[0][0] * ic, my = acc[1][0] * ic, mz = acc[2][0] * ic;
        float *g = x + 128;
        g[0] = (float)leaf_ka[cl[c]];
        g[1] = (float)(cnt / 64.0);
        g[2] = (float)mx;
        g[3] = (float)my;
        g[4] = (float)mz;
        g[5] = (float)sqrt(fmax(acc[3][0] * ic - mx * mx, 0.0));
        g[6] = (float)sqrt(fmax(acc[4][0] * ic - my * my, 0.0));
        g[7] = (float)sqrt(fmax(acc[5][0] * ic - mz * mz, 0.0));
        g[8] = (float)(acc[6][0] * ic);
        g[9] = (float)(acc[7][0] * ic);
        g[10] = (float)(acc[8][0] * ic);
        g[11] = 1.0f;
        scale[c] = (float)nrm;
    }
}

// z[perm[s + q]] += scale * (Y[2q] + i Y[2q+1]) for the chunk's unknowns
__global__ void __launch_bounds__(64) k_mlp_apply(int64_t nchunk, const int32_t *cs, const int32_t *cn,
                                                  const int32_t *perm, const float *Y, const float *scale,
                                                  double2 *z) {
    const int64_t c = blockIdx.x;
    if (c >= nchunk) return;
    const int tid = threadIdx.x;
    if (tid >= cn[c]) return;
    const int u = perm[cs[c] + tid];
    const double sc = scale[c];
    const float *y = Y + c * MLP_OUT;
    z[u] = cadd(z[u], cmk(sc * y[2 * tid], sc * y[2 * tid + 1]));
}

// training target: T = (e - z0) / |r| on the chunk, zero padded (z0 = P_near r)
__global__ void __launch_bounds__(64) k_mlp_target(int64_t nchunk, const int32_t *cs, const int32_t *cn,
                                                   const int32_t *perm, const double2 *e, const double2 *z0,
                                                   const float *scale, float *T) {
    const int64_t c = blockIdx.x;
    if (c >= nchunk) return;
    const int tid = threadIdx.x;
    float *t = T + c * MLP_OUT;
    double2 d = cmk(0, 0);
    const double sc = scale[c];
    if (tid < cn[c] && sc > 0) {
        const int u = perm[cs[c] + tid];
        d = cscale(csub(e[u], z0[u]), 1.0 / sc);
    }
    t[2 * tid] = (float)d.x;
    t[2 * tid + 1] = (float)d.y;
}

// ------------------------------------------------------------------ dense layers
constexpr int LT_M = 64;  // rows per workgroup

// Y[M x NO] = act(X[M x K] W[K x NO] + b) on matrix cores (the forward pass: the solve's
// preconditioner and training): v_mfma_f32_16x16x16f16 takes FP16 inputs (the layer's input rounded to FP16) and FP16 weights
// and accumulates in FP32.  Wt holds W transposed, NO x Kp with Kp = K rounded up to 16 and zeros
// past K, so that a lane's four consecutive K values are one 8-byte load.  Operand layouts of the
// instruction, lane l = 16 g + c: A[c][4 g + j] and B[4 g + j][c] (j = 0..3), D[4 g + i][c].
// 64 rows per workgroup, wavefront w rows 16 w .. 16 w + 15 and all NO = 128 columns (8 blocks).
typedef _Float16 mlp_h4 __attribute__((ext_vector_type(4)));
typedef float mlp_f4 __attribute__((ext_vector_type(4)));
__global__ void __launch_bounds__(256) k_lin_fwd_mfma(int64_t M, int K, int Kp, const float *X, const __half *Wt,
                                                      const float *b, float *Y, int relu) {
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, g = lane >> 4, c = lane & 15;
    const int64_t r0 = (int64_t)blockIdx.x * LT_M + 16 * wv, ra = r0 + c;
    const _Float16 *W = (const _Float16 *)Wt;
    mlp_f4 acc[MLP_H / 16];
#pragma unroll
    for (int cb = 0; cb < MLP_H / 16; ++cb) acc[cb] = mlp_f4{0.f, 0.f, 0.f, 0.f};
    for (int k0 = 0; k0 < Kp; k0 += 16) {
        const int kk = k0 + 4 * g;  // K % 4 == 0: the four values lie on the same side of K
        mlp_h4 a = {0, 0, 0, 0};
        if (ra < M && kk < K) {
            const float4 x = *(const float4 *)(X + ra * K + kk);
            a = mlp_h4{(_Float16)x.x, (_Float16)x.y, (_Float16)x.z, (_Float16)x.w};
        }
#pragma unroll
        for (int cb = 0; cb < MLP_H / 16; ++cb) {
            const mlp_h4 bv = *(const mlp_h4 *)(W + (int64_t)(16 * cb + c) * Kp + kk);
            acc[cb] = __builtin_amdgcn_mfma_f32_16x16x16f16(a, bv, acc[cb], 0, 0, 0);
        }
    }
#pragma unroll
    for (int cb = 0; cb < MLP_H / 16; ++cb)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int64_t m = r0 + 4 * g + i;
            const int o = 16 * cb + c;
            if (m >= M) continue;
            float v = acc[cb][i] + b[o];
            if (relu) v = fmaxf(v, 0.f);
            Y[m * MLP_H + o] = v;
        }
}

// the transposed, padded FP16 copy of one layer: Wt[o][k] = W[k][o] (k < K), 0 (K <= k < Kp)
__global__ void k_half_t(int K, int Kp, int NO, const float *W, __half *Wt) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)NO * Kp) return;
    const int o = (int)(i / Kp), k = (int)(i % Kp);
    Wt[i] = __float2half(k < K ? W[(int64_t)k * NO + o] : 0.f);
}

// dX[M x K] = (dY[M x NO] W^T) masked by (Xact > 0) when mask is set (ReLU of the layer below)
__global__ void __launch_bounds__(256) k_lin_bwd_x(int64_t M, int K, int NO, const float *dY, const __half *W,
                                                   const float *Xact, int mask, float *dX) {
    __shared__ float ds[LT_M][MLP_H + 1];
    const int tid = threadIdx.x;
    const int64_t m0 = (int64_t)blockIdx.x * LT_M;
    for (int e = tid; e < LT_M * MLP_H; e += 256) {
        const int r = e / MLP_H, o = e % MLP_H;
        const int64_t m = m0 + r;
        ds[r][o] = (m < M && o < NO) ? dY[m * NO + o] : 0.f;
    }
    __syncthreads();
    for (int e = tid; e < LT_M * K; e += 256) {
        const int r = e / K, kk = e % K;
        const int64_t m = m0 + r;
        if (m >= M) continue;
        float s = 0.f;
        const __half *wr = W + (int64_t)kk * NO;
        for (int o = 0; o < NO; ++o) s = fmaf(ds[r][o], __half2float(wr[o]), s);
        if (mask && !(Xact[m * K + kk] > 0.f)) s = 0.f;
        dX[m * K + kk] = s;
    }
}

// partial weight gradients over row chunks: P[chunk][K+1][NO] (row K holds the bias gradient)
constexpr int GW_ROWS = 512;
__global__ void __launch_bounds__(256) k_lin_bwd_w(int64_t M, int K, int NO, const float *X, const float *dY,
                                                   float *P) {
    const int64_t r0 = (int64_t)blockIdx.x * GW_ROWS;
    const int64_t r1 = min(M, r0 + GW_ROWS);
    float *out = P + (int64_t)blockIdx.x * (K + 1) * NO;
    for (int e = threadIdx.x; e < (K + 1) * NO; e += blockDim.x) {
        const int kk = e / NO, o = e % NO;
        float s = 0.f;
        for (int64_t m = r0; m < r1; ++m) s = fmaf(kk < K ? X[m * K + kk] : 1.f, dY[m * NO + o], s);
        out[e] = s;
    }
}

__global__ void k_sum_partials(int nchunk, int64_t len, const float *P, float *g) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= len) return;
    float s = 0.f;
    for (int c = 0; c < nchunk; ++c) s += P[(int64_t)c * len + e];
    g[e] = s;
}

// loss = sum (Y - T)^2 / M per block partial; dY = 2 (Y - T) / M
__global__ void __launch_bounds__(256) k_mse(int64_t M, int NO, const float *Y, const float *T, float *dY,
                                             float *partial) {
    __shared__ float red[256];
    float s = 0.f;
    const int64_t total = M * NO;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const float d = Y[e] - T[e];
        dY[e] = 2.f * d / (float)M;
        s += d * d;
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = red[0] / (float)M;
}

__global__ void k_adam(int64_t n, float *w, const float *g, float *m1, float *m2, float lr, float b1, float b2,
                       float eps, float c1, float c2, __half *w16) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float a = b1 * m1[i] + (1.f - b1) * gi, v = b2 * m2[i] + (1.f - b2) * gi * gi;
    m1[i] = a;
    m2[i] = v;
    const float wi = w[i] - lr * (a / c1) / (sqrtf(v / c2) + eps);
    w[i] = wi;
    w16[i] = __float2half(wi);
}

__global__ void k_gather_rows(int64_t B, int width, const int64_t *idx, const float *src, float *dst) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= B * width) return;
    const int64_t r = e / width;
    dst[e] = src[idx[r] * width + (e - r * width)];
}

__global__ void k_vsub(int64_t n, const double2 *a, const double2 *b, double2 *out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = csub(a[i], b[i]);
}

__global__ void k_to_half(int64_t n, const float *a, __half *b) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) b[i] = __float2half(a[i]);
}

// ------------------------------------------------------------------ host side
// packed parameter layout: for each layer l: W_l (in_l x out_l, row-major), then b_l (out_l)
static const int LAYER_IN[4] = {MLP_IN, MLP_H, MLP_H, MLP_H};
static const int LAYER_OUT[4] = {MLP_H, MLP_H, MLP_H, MLP_OUT};

int64_t mlp_param_count() {
    int64_t s = 0;
    for (int l = 0; l < 4; ++l) s += (int64_t)LAYER_IN[l] * LAYER_OUT[l] + LAYER_OUT[l];
    return s;
}
static int64_t layer_w_off(int l) {
    int64_t s = 0;
    for (int q = 0; q < l; ++q) s += (int64_t)LAYER_IN[q] * LAYER_OUT[q] + LAYER_OUT[q];
    return s;
}
static int layer_kp(int l) { return (LAYER_IN[l] + 15) / 16 * 16; }
static int64_t layer_wt_off(int l) {  // offsets in the transposed FP16 copy
    int64_t s = 0;
    for (int q = 0; q < l; ++q) s += (int64_t)LAYER_OUT[q] * layer_kp(q);
    return s;
}
static void make_half_t(const float *w32, __half *w16t, hipStream_t st) {
    for (int l = 0; l < 4; ++l) {
        const int64_t n = (int64_t)LAYER_OUT[l] * layer_kp(l);
        k_half_t<<<ceil_div(n, 256), 256, 0, st>>>(LAYER_IN[l], layer_kp(l), LAYER_OUT[l], w32 + layer_w_off(l),
                                                   w16t + layer_wt_off(l));
        LAUNCH_OK();
    }
}

void Mlp::init(DeviceBuffers &buf, uint64_t seed, hipStream_t st) {
    const int64_t np = mlp_param_count();
    std::vector<float> h(np, 0.f);
    // He-uniform initialisation from a counter-based generator (SplitMix64)
    auto mix = [](uint64_t z) {
        z += 0x9E3779B97F4A7C15ull;
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        return z ^ (z >> 31);
    };
    for (int l = 0; l < 4; ++l) {
        const int64_t off = layer_w_off(l);
        const double lim = (l == 3 ? 0.1 : 1.0) * std::sqrt(6.0 / LAYER_IN[l]);
        for (int64_t i = 0; i < (int64_t)LAYER_IN[l] * LAYER_OUT[l]; ++i) {
            const double u = (mix(seed * 0x100000001B3ull + off + i) >> 11) * (1.0 / 9007199254740992.0);
            h[off + i] = (float)((2.0 * u - 1.0) * lim);
        }
    }
    w32 = dget<float>(buf, "mlp_w32", np);
    w16 = dget<__half>(buf, "mlp_w16", np);
    w16t = dget<__half>(buf, "mlp_w16t", layer_wt_off(4 - 1) + (int64_t)LAYER_OUT[3] * layer_kp(3));
    m1 = dget<float>(buf, "mlp_m1", np);
    m2 = dget<float>(buf, "mlp_m2", np);
    h2d_now(w32, h.data(), sizeof(float) * np, st);  // h is a temporary
    HIP_OK(hipMemsetAsync(m1, 0, sizeof(float) * np, st));
    HIP_OK(hipMemsetAsync(m2, 0, sizeof(float) * np, st));
    sync_half(st);
    step = 0;
    ready = true;
}

void Mlp::sync_half(hipStream_t st) {
    const int64_t np = mlp_param_count();
    k_to_half<<<ceil_div(np, 256), 256, 0, st>>>(np, w32, w16);
    LAUNCH_OK();
    make_half_t(w32, w16t, st);
}

// forward over M samples; A[l] receives the output of layer l (A[3] = network output)
void Mlp::forward(int64_t M, const float *X, float *const A[4], hipStream_t st) const {
    const float *in = X;
    for (int l = 0; l < 4; ++l) {
        const int64_t off = layer_w_off(l);
        const float *b = w32 + off + (int64_t)LAYER_IN[l] * LAYER_OUT[l];
        static_assert(MLP_IN % 4 == 0 && MLP_H % 4 == 0 && MLP_OUT == MLP_H, "matrix-core layer shapes");
        k_lin_fwd_mfma<<<ceil_div(M, LT_M), 256, 0, st>>>(M, LAYER_IN[l], layer_kp(l), in, w16t + layer_wt_off(l), b,
                                                          A[l], l < 3 ? 1 : 0);
        LAUNCH_OK();
        in = A[l];
    }
}

// gradient of the mean squared error over M samples into grad (packed like the parameters);
// returns nothing on the host: the loss goes to loss_dev[0] after the partial sum
void Mlp::backward(int64_t M, const float *X, float *const A[4], const float *T, float *grad, float *loss_dev,
                   DeviceBuffers &scr, hipStream_t st) const {
    float *dA = dget<float>(scr, "mlp_dA", (size_t)M * MLP_H);
    float *dB = dget<float>(scr, "mlp_dB", (size_t)M * MLP_H);
    const int nb = 256;
    float *part = dget<float>(scr, "mlp_lpart", nb);
    k_mse<<<nb, 256, 0, st>>>(M, MLP_OUT, A[3], T, dA, part);
    LAUNCH_OK();
    k_sum_partials<<<1, 1, 0, st>>>(nb, 1, part, loss_dev);
    LAUNCH_OK();
    const int nch = ceil_div(M, GW_ROWS);
    float *P = dget<float>(scr, "mlp_gpart", (size_t)nch * (MLP_IN + 1) * MLP_H);
    float *dcur = dA, *dnext = dB;
    for (int l = 3; l >= 0; --l) {
        const int K = LAYER_IN[l], NO = LAYER_OUT[l];
        const float *in = l == 0 ? X : A[l - 1];
        const int64_t off = layer_w_off(l);
        k_lin_bwd_w<<<nch, 256, 0, st>>>(M, K, NO, in, dcur, P);
        LAUNCH_OK();
        const int64_t len = (int64_t)(K + 1) * NO;  // W then b: the packed layout
        k_sum_partials<<<ceil_div(len, 256), 256, 0, st>>>(nch, len, P, grad + off);
        LAUNCH_OK();
        if (l > 0) {
            k_lin_bwd_x<<<ceil_div(M, LT_M), 256, 0, st>>>(M, K, NO, dcur, w16 + off, A[l - 1], 1, dnext);
            LAUNCH_OK();
            std::swap(dcur, dnext);
        }
    }
}

void Mlp::adam_step(const float *grad, float lr, hipStream_t st) {
    const int64_t np = mlp_param_count();
    ++step;
    const float b1 = 0.9f, b2 = 0.999f;
    const float c1 = 1.f - std::pow(b1, (float)step), c2 = 1.f - std::pow(b2, (float)step);
    k_adam<<<ceil_div(np, 256), 256, 0, st>>>(np, w32, grad, m1, m2, lr, b1, b2, 1e-8f, c1, c2, w16);
    LAUNCH_OK();
    make_half_t(w32, w16t, st);
}

void gather_rows(int64_t B, int width, const int64_t *idx, const float *src, float *dst, hipStream_t st) {
    if (B == 0) return;
    k_gather_rows<<<ceil_div(B * width, 256), 256, 0, st>>>(B, width, idx, src, dst);
    LAUNCH_OK();
}

__global__ void k_vadd(int64_t n, const double2 *a, const double2 *b, double2 *out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = cadd(a[i], b[i]);
}

void vec_add(int64_t n, const double2 *a, const double2 *b, double2 *out, hipStream_t st) {
    k_vadd<<<ceil_div(n, 256), 256, 0, st>>>(n, a, b, out);
    LAUNCH_OK();
}

void vec_sub(int64_t n, const double2 *a, const double2 *b, double2 *out, hipStream_t st) {
    k_vsub<<<ceil_div(n, 256), 256, 0, st>>>(n, a, b, out);
    LAUNCH_OK();
}

void mlp_features(int64_t nchunk, const int32_t *cs, const int32_t *cn, const int32_t *cl, const int32_t *perm,
                  const double2 *v, const double4 *en, const double2 *beta, const double *leaf_ka, float *X,
                  float *scale, hipStream_t st) {
    if (nchunk == 0) return;
    k_mlp_features<<<(unsigned)nchunk, 64, 0, st>>>(nchunk, cs, cn, cl, perm, v, en, beta, leaf_ka, X, scale);
    LAUNCH_OK();
}

void mlp_apply(int64_t nchunk, const int32_t *cs, const int32_t *cn, const int32_t *perm, const float *Y,
               const float *scale, double2 *z, hipStream_t st) {
    if (nchunk == 0) return;
    k_mlp_apply<<<(unsigned)nchunk, 64, 0, st>>>(nchunk, cs, cn, perm, Y, scale, z);
    LAUNCH_OK();
}

void mlp_target(int64_t nchunk, const int32_t *cs, const int32_t *cn, const int32_t *perm, const double2 *e,
                const double2 *z0, const float *scale, float *T, hipStream_t st) {
    if (nchunk == 0) return;
    k_mlp_target<<<(unsigned)nchunk, 64, 0, st>>>(nchunk, cs, cn, perm, e, z0, scale, T);
    LAUNCH_OK();
}

}  // namespace fmm
