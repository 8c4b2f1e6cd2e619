// HIP kernels of the learned correction (see gnn.h): BF16 weights and
// activations, FP32 accumulation, deterministic gradient reductions.
#include <hip/hip_runtime.h>

#include "gnn.h"

namespace bido {
namespace {

constexpr int BLOCK = 256;
constexpr int WAVE = 64;

__device__ __forceinline__ float bf2f(uint16_t u) { return __uint_as_float((uint32_t)u << 16); }
__device__ __forceinline__ uint16_t f2bf(float f) {   // round to nearest even
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)(u >> 16);   // inf / nan
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

unsigned blocks_for(int64_t threads) {
    int64_t g = (threads + BLOCK - 1) / BLOCK;
    return (unsigned)(g < 1 ? 1 : g);
}

// f[i][0] = t_i / rms(t) with rms(t) = sqrt(tn2 / n), f[i][1..15] = static features
__global__ void k_input(int64_t n, const double* __restrict__ t, const double* __restrict__ tn2,
                        const float* __restrict__ that, const float* __restrict__ stat,
                        uint16_t* __restrict__ f) {
    const int64_t id = blockIdx.x * (int64_t)BLOCK + threadIdx.x;
    if (id >= n * GNN_F) return;
    const int64_t i = id / GNN_F;
    const int j = (int)(id % GNN_F);
    float v;
    if (j == 0) {
        if (that) {
            v = that[i];
        } else if (!t) {
            v = 1.0f;                      // embedding mode: constant channel
        } else {
            const double rms = sqrt(*tn2 / (double)n);
            v = rms > 0.0 ? (float)(t[i] / rms) : 0.0f;
        }
    } else {
        v = stat[i * GNN_F + j];
    }
    f[id] = f2bf(v);
}

// out_i = sum_j a_ij in_j  (W features per vertex)
template <int W>
__global__ void k_agg(int64_t n, const int64_t* __restrict__ ptr, const int32_t* __restrict__ col,
                      const float* __restrict__ val, const uint16_t* __restrict__ in,
                      uint16_t* __restrict__ out) {
    const int64_t id = blockIdx.x * (int64_t)BLOCK + threadIdx.x;
    if (id >= n * W) return;
    const int64_t i = id / W;
    const int k = (int)(id % W);
    float s = 0.0f;
    for (int64_t p = ptr[i]; p < ptr[i + 1]; ++p) s += val[p] * bf2f(in[(int64_t)col[p] * W + k]);
    out[id] = f2bf(s);
}

// r_i = o_i - y_i * yinv
__global__ void k_resid(int64_t n, const float* __restrict__ o, const float* __restrict__ y, float yinv,
                        float* __restrict__ r) {
    const int64_t i = blockIdx.x * (int64_t)BLOCK + threadIdx.x;
    if (i < n) r[i] = o[i] - y[i] * yinv;
}

// energy-norm loss r^T W r: d o = 2 W r, per-block loss partials
__global__ __launch_bounds__(BLOCK) void k_energy(int64_t n, const int64_t* __restrict__ wptr,
                                                  const int32_t* __restrict__ wcol,
                                                  const float* __restrict__ wval,
                                                  const float* __restrict__ r, float* __restrict__ dout,
                                                  float* __restrict__ loss_part) {
    __shared__ float red[BLOCK];
    const int64_t i = blockIdx.x * (int64_t)BLOCK + threadIdx.x;
    float l = 0.0f;
    if (i < n) {
        float wr = 0.0f;
        for (int64_t p = wptr[i]; p < wptr[i + 1]; ++p) wr += wval[p] * r[wcol[p]];
        dout[i] = 2.0f * wr;
        l = r[i] * wr;
    }
    red[threadIdx.x] = l;
    __syncthreads();
    for (int k = BLOCK / 2; k > 0; k >>= 1) {
        if (threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) loss_part[blockIdx.x] = red[0];
}

// dz2 = d o_i * w3 * [h2 > 0]
__global__ __launch_bounds__(BLOCK) void k_bwd_out(int64_t n, const float* __restrict__ dout,
                                                   const uint16_t* __restrict__ h2,
                                                   const uint16_t* __restrict__ wbf,
                                                   float* __restrict__ dz2) {
    const int64_t id = blockIdx.x * (int64_t)BLOCK + threadIdx.x;
    const int64_t i = id / GNN_H;
    const int a = (int)(id % GNN_H);
    if (i < n) dz2[id] = bf2f(h2[id]) > 0.0f ? dout[i] * bf2f(wbf[GNN_OFF_W3 + a]) : 0.0f;
}

// g_i = W2n^T dz2_i
__global__ __launch_bounds__(BLOCK) void k_bwd_g(int64_t n, const float* __restrict__ dz2,
                                                 const uint16_t* __restrict__ wbf, float* __restrict__ g) {
    __shared__ float wn[GNN_H * GNN_H];
    __shared__ float ds[BLOCK / GNN_H][GNN_H];
    for (int k = threadIdx.x; k < GNN_H * GNN_H; k += BLOCK) wn[k] = bf2f(wbf[GNN_OFF_W2N + k]);
    const int nl = threadIdx.x / GNN_H, k = threadIdx.x % GNN_H;
    const int64_t i = blockIdx.x * (int64_t)(BLOCK / GNN_H) + nl;
    if (i < n) ds[nl][k] = dz2[i * GNN_H + k];
    __syncthreads();
    if (i >= n) return;
    float s = 0.0f;
    for (int a = 0; a < GNN_H; ++a) s += wn[a * GNN_H + k] * ds[nl][a];
    g[i * GNN_H + k] = s;
}

// dh1_i = W2s^T dz2_i + sum_j (A^T)_ij g_j ;  dz1 = dh1 * [h1 > 0]
__global__ __launch_bounds__(BLOCK) void k_bwd_hidden(int64_t n, const float* __restrict__ dz2,
                                                      const float* __restrict__ g,
                                                      const int64_t* __restrict__ tptr,
                                                      const int32_t* __restrict__ tcol,
                                                      const float* __restrict__ tval,
                                                      const uint16_t* __restrict__ h1,
                                                      const uint16_t* __restrict__ wbf,
                                                      float* __restrict__ dz1) {
    __shared__ float wsm[GNN_H * GNN_H];
    __shared__ float ds[BLOCK / GNN_H][GNN_H];
    for (int k = threadIdx.x; k < GNN_H * GNN_H; k += BLOCK) wsm[k] = bf2f(wbf[GNN_OFF_W2S + k]);
    const int nl = threadIdx.x / GNN_H, k = threadIdx.x % GNN_H;
    const int64_t i = blockIdx.x * (int64_t)(BLOCK / GNN_H) + nl;
    if (i < n) ds[nl][k] = dz2[i * GNN_H + k];
    __syncthreads();
    if (i >= n) return;
    float s = 0.0f;
    for (int a = 0; a < GNN_H; ++a) s += wsm[a * GNN_H + k] * ds[nl][a];
    for (int64_t p = tptr[i]; p < tptr[i + 1]; ++p) s += tval[p] * g[(int64_t)tcol[p] * GNN_H + k];
    dz1[i * GNN_H + k] = bf2f(h1[i * GNN_H + k]) > 0.0f ? s : 0.0f;
}

// Weight-gradient partials: block b sums over its vertex range
//   P[b][off_w + a*IN + k] = sum_i G[i][a] X[i][k],   P[b][off_b + a] = sum_i G[i][a]
// with GW rows of G per vertex (GW = 32, or 1 for the readout).
template <int GW, int IN>
__global__ void k_wgrad(int64_t n, const float* __restrict__ G, const uint16_t* __restrict__ X,
                        float* __restrict__ part, int off_w, int off_b) {
    const int64_t per = (n + gridDim.x - 1) / gridDim.x;
    const int64_t i0 = blockIdx.x * per, i1 = min(n, i0 + per);
    float* P = part + (int64_t)blockIdx.x * GNN_P;
    for (int e = threadIdx.x; e < GW * IN; e += blockDim.x) {
        const int a = e / IN, k = e % IN;
        float s = 0.0f;
        for (int64_t i = i0; i < i1; ++i) s += G[i * GW + a] * bf2f(X[i * IN + k]);
        P[off_w + e] = s;
    }
    if (off_b >= 0)
        for (int a = threadIdx.x; a < GW; a += blockDim.x) {
            float s = 0.0f;
            for (int64_t i = i0; i < i1; ++i) s += G[i * GW + a];
            P[off_b + a] = s;
        }
}

// The same weight-gradient partials on the matrix cores: the product
// G^T X (32 x IN) is a sum over vertices, so each wave runs FP32 MFMA
// 32x32x2 steps (two vertices per step: lane l feeds G[v][l % 32] and
// X[v][l % 32] of vertex v = v0 + l / 32), the four waves of the block add
// their 32 x 32 tiles in LDS, and the bias (sum over vertices of G[v][a])
// rides in column IN when IN < 32, else in a per-lane sum.  X is BF16 and
// widened exactly to FP32; accumulation is FP32 as in k_wgrad.
typedef float floatx16 __attribute__((ext_vector_type(16)));

template <int IN>
__global__ __launch_bounds__(256) void k_wgrad_mfma(int64_t n, const float* __restrict__ G,
                                                    const uint16_t* __restrict__ X, float* __restrict__ part,
                                                    int off_w, int off_b) {
    __shared__ float tile[4][32 * 33];
    __shared__ float bsum[4][32];
    const int lane = threadIdx.x % WAVE, wave = threadIdx.x / WAVE;
    const int64_t per = (n + gridDim.x - 1) / gridDim.x;
    const int64_t b0 = blockIdx.x * per, b1 = min(n, b0 + per);
    const int64_t wper = (b1 - b0 + 3) / 4;
    const int64_t w0 = b0 + wave * wper, w1 = min(b1, w0 + wper);
    const int a = lane % 32, half = lane / 32;
    floatx16 acc = {};
    float bs = 0.0f;
    for (int64_t v0 = w0; v0 < w1; v0 += 2) {
        const int64_t v = v0 + half;
        const bool in = v < w1;
        const int64_t vc = in ? v : w0;
        const float g = in ? G[vc * 32 + a] : 0.0f;
        float x;
        if (a < IN) x = in ? bf2f(X[vc * IN + a]) : 0.0f;
        else x = (a == IN && in) ? 1.0f : 0.0f;
        bs += g;
        acc = __builtin_amdgcn_mfma_f32_32x32x2f32(g, x, acc, 0, 0, 0);
    }
    // D[row][col], row = 8 (r / 4) + 4 (lane / 32) + r % 4, col = lane % 32
#pragma unroll
    for (int r = 0; r < 16; ++r) tile[wave][(8 * (r / 4) + 4 * half + (r % 4)) * 33 + a] = acc[r];
    const float bo = __shfl_down(bs, 32, WAVE);
    if (lane < 32) bsum[wave][lane] = bs + bo;
    __syncthreads();
    float* P = part + (int64_t)blockIdx.x * GNN_P;
    for (int e = threadIdx.x; e < 32 * IN; e += blockDim.x) {
        const int row = e / IN, col = e % IN;
        P[off_w + e] = tile[0][row * 33 + col] + tile[1][row * 33 + col] + tile[2][row * 33 + col] +
                       tile[3][row * 33 + col];
    }
    if (off_b >= 0 && threadIdx.x < 32) {
        const int row = threadIdx.x;
        P[off_b + row] = IN < 32 ? tile[0][row * 33 + IN] + tile[1][row * 33 + IN] + tile[2][row * 33 + IN] +
                                       tile[3][row * 33 + IN]
                                 : bsum[0][row] + bsum[1][row] + bsum[2][row] + bsum[3][row];
    }
}

// sum of squares of a float vector into per-block partials
__global__ void k_sumsq_f(int64_t n, const float* __restrict__ a, float* __restrict__ part) {
    __shared__ float red[BLOCK];
    float s = 0.0f;
    for (int64_t i = blockIdx.x * (int64_t)BLOCK + threadIdx.x; i < n; i += (int64_t)gridDim.x * BLOCK)
        s += a[i] * a[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int k = BLOCK / 2; k > 0; k >>= 1) {
        if (threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// grad[p] += sum_b part[b][p] (fixed order); loss += sum of loss partials
__global__ void k_reduce_grad(int nb, const float* __restrict__ part, float* __restrict__ grad,
                              const float* __restrict__ loss_part, int nlp, double* loss) {
    const int p = blockIdx.x * BLOCK + threadIdx.x;
    if (grad && p < GNN_P) {
        float s = 0.0f;
        for (int b = 0; b < nb; ++b) s += part[(int64_t)b * GNN_P + p];
        grad[p] += s;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0 && loss) {
        double l = 0.0;
        for (int b = 0; b < nlp; ++b) l += loss_part[b];
        *loss += l;
    }
}

__global__ void k_adam(float* theta, float* m, float* v, const float* grad, float scale, float lr,
                       float c1, float c2, uint16_t* wbf) {
    const int p = blockIdx.x * BLOCK + threadIdx.x;
    if (p >= GNN_P) return;
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    const float g = grad[p] * scale;
    const float mm = b1 * m[p] + (1.0f - b1) * g;
    const float vv = b2 * v[p] + (1.0f - b2) * g * g;
    m[p] = mm;
    v[p] = vv;
    const float th = theta[p] - lr * (mm / c1) / (sqrtf(vv / c2) + eps);
    theta[p] = th;
    wbf[p] = f2bf(th);
}

__global__ void k_to_bf16(const float* theta, uint16_t* wbf) {
    const int p = blockIdx.x * BLOCK + threadIdx.x;
    if (p < GNN_P) wbf[p] = f2bf(theta[p]);
}

__global__ void k_store_sample(int64_t n, const double* __restrict__ t, const double* __restrict__ tn2,
                               float* __restrict__ that) {
    const int64_t i = blockIdx.x * (int64_t)BLOCK + threadIdx.x;
    if (i >= n) return;
    const double rms = sqrt(*tn2 / (double)n);
    that[i] = rms > 0.0 ? (float)(t[i] / rms) : 0.0f;
}

__global__ void k_pending(int64_t n, const double* __restrict__ xv, const double* __restrict__ z2,
                          double* __restrict__ d) {
    const int64_t i = blockIdx.x * (int64_t)BLOCK + threadIdx.x;
    if (i < n) d[i] = xv[i] + z2[i];
}

__global__ void k_finish_targets(int64_t n, const double* __restrict__ vstar, const double* __restrict__ d,
                                 const double* __restrict__ tn2, float* __restrict__ y) {
    const int64_t i = blockIdx.x * (int64_t)BLOCK + threadIdx.x;
    if (i >= n) return;
    const double rms = sqrt(*tn2 / (double)n);
    y[i] = rms > 0.0 ? (float)((vstar[i] - d[i]) / rms) : 0.0f;
}

// One layer, h_i = relu(Ws x_i + Wn m_i + b); with READOUT also
// o_i = w3 . h_i + b3, added (times rms(t) * out_scale) to z2 in inference
// mode.  On the matrix cores: each wave computes a tile of 32 vertices x 32
// units as X Ws^T + M Wn^T with FP32 MFMA 32x32x2 steps
// (lane l feeds A = X[v0 + l % 32][k0 + l / 32] from the wave's LDS copy of
// the tile's inputs and B = Ws[l % 32][k0 + l / 32], held in registers for
// every k0), BF16 inputs widened exactly to FP32, FP32 accumulation.
// D[row][col]: row = 8 (r / 4) + 4 (l / 32) + r % 4 (vertex),
// col = l % 32 (unit).  The readout sums the 32 units of a vertex across
// the lanes of one half-wave.  Workgroups of four waves take 128 vertices
// per round (a round count uniform over the workgroup).
template <int IN, bool READOUT>
__global__ __launch_bounds__(256) void k_layer_mfma(int64_t n, const uint16_t* __restrict__ x,
                                                    const uint16_t* __restrict__ m,
                                                    const uint16_t* __restrict__ wbf, int off_ws, int off_wn,
                                                    int off_b, uint16_t* __restrict__ h, float* __restrict__ o,
                                                    const double* __restrict__ tn2, double* __restrict__ z2,
                                                    float out_scale) {
    __shared__ float xs[4][32][IN + 1], ms[4][32][IN + 1];
    const int lane = threadIdx.x % WAVE, wave = threadIdx.x / WAVE;
    const int a = lane % 32, half = lane / 32;
    float wsr[IN / 2], wnr[IN / 2];
#pragma unroll
    for (int j = 0; j < IN / 2; ++j) {
        wsr[j] = bf2f(wbf[off_ws + a * IN + 2 * j + half]);
        wnr[j] = bf2f(wbf[off_wn + a * IN + 2 * j + half]);
    }
    const float bias = bf2f(wbf[off_b + a]);
    const float w3 = READOUT ? bf2f(wbf[GNN_OFF_W3 + a]) : 0.0f;
    const float b3 = READOUT ? bf2f(wbf[GNN_OFF_B3]) : 0.0f;
    const double zscale = (READOUT && z2) ? sqrt(*tn2 / (double)n) * (double)out_scale : 0.0;
    for (int64_t base = (int64_t)blockIdx.x * 128; base < n; base += (int64_t)gridDim.x * 128) {
        const int64_t v0 = base + wave * 32;
        for (int e = lane; e < 32 * IN; e += WAVE) {
            const int r = e / IN, k = e % IN;
            const int64_t v = v0 + r;
            xs[wave][r][k] = v < n ? bf2f(x[v * IN + k]) : 0.0f;
            ms[wave][r][k] = v < n ? bf2f(m[v * IN + k]) : 0.0f;
        }
        __syncthreads();
        floatx16 acc = {};
#pragma unroll
        for (int j = 0; j < IN / 2; ++j) {
            acc = __builtin_amdgcn_mfma_f32_32x32x2f32(xs[wave][a][2 * j + half], wsr[j], acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_32x32x2f32(ms[wave][a][2 * j + half], wnr[j], acc, 0, 0, 0);
        }
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int row = 8 * (r / 4) + 4 * half + (r % 4);
            const int64_t v = v0 + row;
            const float z = acc[r] + bias;
            const uint16_t hb = f2bf(z > 0.0f ? z : 0.0f);
            if (h && v < n) h[v * GNN_H + a] = hb;
            if (READOUT) {
                float s = w3 * bf2f(hb);
#pragma unroll
                for (int msk = 16; msk > 0; msk >>= 1) s += __shfl_xor(s, msk, 32);
                if (a == 0 && v < n) {
                    const float ov = s + b3;
                    if (o) o[v] = ov;
                    if (z2) z2[v] += zscale * (double)ov;
                }
            }
        }
        __syncthreads();
    }
}

void forward_common(hipStream_t s, int64_t n, const GnnGraph& A, const uint16_t* wbf, GnnAct& a, int mode,
                    const double* tn2, double* z2, float out_scale) {
    k_agg<GNN_F><<<blocks_for(n * GNN_F), BLOCK, 0, s>>>(n, A.ptr, A.col, A.val, a.f, a.m0);
    const unsigned gb = (unsigned)std::min<int64_t>((n + 127) / 128, 16384);
    k_layer_mfma<GNN_F, false><<<gb, 256, 0, s>>>(n, a.f, a.m0, wbf, GNN_OFF_W1S, GNN_OFF_W1N, GNN_OFF_B1, a.h1,
                                                   nullptr, nullptr, nullptr, 1.0f);
    k_agg<GNN_H><<<blocks_for(n * GNN_H), BLOCK, 0, s>>>(n, A.ptr, A.col, A.val, a.h1, a.m1);
    k_layer_mfma<GNN_H, true><<<gb, 256, 0, s>>>(n, a.h1, a.m1, wbf, GNN_OFF_W2S, GNN_OFF_W2N, GNN_OFF_B2,
                                                  mode == 1 ? a.h2 : nullptr, mode == 1 ? a.o : nullptr,
                                                  tn2, mode == 0 ? z2 : nullptr, out_scale);
}

}  // namespace

void launch_gnn_forward(hipStream_t s, int64_t n, const double* t, const double* tn2, const float* stat,
                        const GnnGraph& A, const uint16_t* wbf, GnnAct& a, int mode, double* z2,
                        float out_scale) {
    if (n <= 0) return;
    k_input<<<blocks_for(n * GNN_F), BLOCK, 0, s>>>(n, t, tn2, nullptr, stat, a.f);
    forward_common(s, n, A, wbf, a, mode, tn2, z2, out_scale);
}

void launch_gnn_forward_sample(hipStream_t s, int64_t n, const float* that, const float* stat,
                               const GnnGraph& A, const uint16_t* wbf, GnnAct& a) {
    if (n <= 0) return;
    k_input<<<blocks_for(n * GNN_F), BLOCK, 0, s>>>(n, nullptr, nullptr, that, stat, a.f);
    forward_common(s, n, A, wbf, a, 1, nullptr, nullptr, 1.0f);
}

void launch_gnn_backward(hipStream_t s, int64_t n, const float* y, const GnnGraph& W, const GnnGraph& At,
                         const uint16_t* wbf, GnnAct& a, float* partials, float* grad, double* loss,
                         float yinv) {
    if (n <= 0) return;
    const unsigned gb = blocks_for(n * GNN_H);
    const unsigned nb = blocks_for(n);
    float* loss_part = partials + (int64_t)GNN_WG_BLOCKS * GNN_P;
    k_resid<<<nb, BLOCK, 0, s>>>(n, a.o, y, yinv, a.res);
    k_energy<<<nb, BLOCK, 0, s>>>(n, W.ptr, W.col, W.val, a.res, a.dout, loss_part);
    k_bwd_out<<<gb, BLOCK, 0, s>>>(n, a.dout, a.h2, wbf, a.dz2);
    k_bwd_g<<<gb, BLOCK, 0, s>>>(n, a.dz2, wbf, a.g2);
    k_bwd_hidden<<<gb, BLOCK, 0, s>>>(n, a.dz2, a.g2, At.ptr, At.col, At.val, a.h1, wbf, a.dz1);
    const int wb = GNN_WG_BLOCKS;
    k_wgrad<1, GNN_H><<<wb, BLOCK, 0, s>>>(n, a.dout, a.h2, partials, GNN_OFF_W3, GNN_OFF_B3);
    k_wgrad_mfma<GNN_H><<<wb, 256, 0, s>>>(n, a.dz2, a.h1, partials, GNN_OFF_W2S, GNN_OFF_B2);
    k_wgrad_mfma<GNN_H><<<wb, 256, 0, s>>>(n, a.dz2, a.m1, partials, GNN_OFF_W2N, -1);
    k_wgrad_mfma<GNN_F><<<wb, 256, 0, s>>>(n, a.dz1, a.f, partials, GNN_OFF_W1S, GNN_OFF_B1);
    k_wgrad_mfma<GNN_F><<<wb, 256, 0, s>>>(n, a.dz1, a.m0, partials, GNN_OFF_W1N, -1);
    k_reduce_grad<<<(GNN_P + BLOCK - 1) / BLOCK, BLOCK, 0, s>>>(GNN_WG_BLOCKS, partials, grad, loss_part,
                                                                 (int)nb, loss);
}

void launch_gnn_loss(hipStream_t s, int64_t n, const float* y, const GnnGraph& W, GnnAct& a,
                     float* partials, double* loss, float yinv) {
    if (n <= 0) return;
    const unsigned nb = blocks_for(n);
    float* loss_part = partials + (int64_t)GNN_WG_BLOCKS * GNN_P;
    k_resid<<<nb, BLOCK, 0, s>>>(n, a.o, y, yinv, a.res);
    k_energy<<<nb, BLOCK, 0, s>>>(n, W.ptr, W.col, W.val, a.res, a.dout, loss_part);
    k_reduce_grad<<<1, BLOCK, 0, s>>>(0, partials, nullptr, loss_part, (int)nb, loss);
}

void launch_gnn_sumsq(hipStream_t s, int64_t n, const float* y, float* partials, double* out) {
    if (n <= 0) return;
    float* lp = partials + (int64_t)GNN_WG_BLOCKS * GNN_P;
    k_sumsq_f<<<256, BLOCK, 0, s>>>(n, y, lp);
    k_reduce_grad<<<1, BLOCK, 0, s>>>(0, partials, nullptr, lp, 256, out);
}

void launch_gnn_energy0(hipStream_t s, int64_t n, const float* y, const GnnGraph& W, GnnAct& a,
                        float* partials, double* out, float yinv) {
    // loss of the zero output: (-y)^T W (-y)
    if (n <= 0) return;
    const unsigned nb = blocks_for(n);
    float* loss_part = partials + (int64_t)GNN_WG_BLOCKS * GNN_P;
    k_resid<<<nb, BLOCK, 0, s>>>(n, a.zero, y, yinv, a.res);
    k_energy<<<nb, BLOCK, 0, s>>>(n, W.ptr, W.col, W.val, a.res, a.dout, loss_part);
    k_reduce_grad<<<1, BLOCK, 0, s>>>(0, partials, nullptr, loss_part, (int)nb, out);
}

// ---------------------------------------------------------------------------
// Learned Schur-complement stencil C^_p = sum_a w3_a h2_ia h2_ja + b3 [i==j]
// on the stored pattern of S_m (entry p = (row[p], col[p]), tpos[p] = index
// of (col[p], row[p])).
// ---------------------------------------------------------------------------
__global__ void k_cvals(int64_t nnz, const int32_t* __restrict__ row, const int32_t* __restrict__ col,
                        const uint16_t* __restrict__ h2, const uint16_t* __restrict__ wbf,
                        float* __restrict__ cval) {
    __shared__ float w3[GNN_H];
    if (threadIdx.x < GNN_H) w3[threadIdx.x] = bf2f(wbf[GNN_OFF_W3 + threadIdx.x]);
    __syncthreads();
    const int64_t p = blockIdx.x * (int64_t)BLOCK + threadIdx.x;
    if (p >= nnz) return;
    const int64_t i = row[p], j = col[p];
    float s = (i == j) ? bf2f(wbf[GNN_OFF_B3]) : 0.0f;
#pragma unroll 8
    for (int a = 0; a < GNN_H; ++a) s += w3[a] * bf2f(h2[i * GNN_H + a]) * bf2f(h2[j * GNN_H + a]);
    cval[p] = s;
}

// r = C^ z - b, loss partial |r|^2
__global__ __launch_bounds__(BLOCK) void k_cspmv(int64_t n, const int64_t* __restrict__ ptr,
                                                 const int32_t* __restrict__ col, const float* __restrict__ cval,
                                                 const float* __restrict__ z, const float* __restrict__ b,
                                                 float* __restrict__ r, float* __restrict__ loss_part) {
    __shared__ float red[BLOCK];
    const int64_t i = blockIdx.x * (int64_t)BLOCK + threadIdx.x;
    float l = 0.0f;
    if (i < n) {
        float s = -b[i];
        for (int64_t p = ptr[i]; p < ptr[i + 1]; ++p) s += cval[p] * z[col[p]];
        r[i] = s;
        l = s * s;
    }
    red[threadIdx.x] = l;
    __syncthreads();
    for (int k = BLOCK / 2; k > 0; k >>= 1) {
        if (threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) loss_part[blockIdx.x] = red[0];
}

// G_p += 2 r_i z_j
__global__ void k_gacc(int64_t nnz, const int32_t* __restrict__ row, const int32_t* __restrict__ col,
                       const float* __restrict__ r, const float* __restrict__ z, float* __restrict__ G) {
    const int64_t p = blockIdx.x * (int64_t)BLOCK + threadIdx.x;
    if (p < nnz) G[p] += 2.0f * r[row[p]] * z[col[p]];
}

// dz2_ia = [h2_ia > 0] w3_a sum_{p in row i} (G_p + G_tpos[p]) h2_{col p, a}
__global__ __launch_bounds__(BLOCK) void k_dh2(int64_t n, const int64_t* __restrict__ ptr,
                                               const int32_t* __restrict__ col, const int32_t* __restrict__ tpos,
                                               const float* __restrict__ G, const uint16_t* __restrict__ h2,
                                               const uint16_t* __restrict__ wbf, float* __restrict__ dz2) {
    const int64_t id = blockIdx.x * (int64_t)BLOCK + threadIdx.x;
    const int64_t i = id / GNN_H;
    const int a = (int)(id % GNN_H);
    if (i >= n) return;
    float s = 0.0f;
    for (int64_t p = ptr[i]; p < ptr[i + 1]; ++p)
        s += (G[p] + G[tpos[p]]) * bf2f(h2[(int64_t)col[p] * GNN_H + a]);
    dz2[id] = bf2f(h2[id]) > 0.0f ? s * bf2f(wbf[GNN_OFF_W3 + a]) : 0.0f;
}

// partials of d/dw3_a = sum_p G_p h2_ia h2_ja and d/db3 = sum_{diag} G_p, by
// rows: block b takes a range of rows, 8 rows at a time (32 lanes per row,
// lane a), then the 8 row slots are summed in LDS in a fixed order.
__global__ __launch_bounds__(256) void k_w3grad(int64_t n, const int64_t* __restrict__ ptr,
                                                const int32_t* __restrict__ col, const float* __restrict__ G,
                                                const uint16_t* __restrict__ h2, float* __restrict__ part) {
    __shared__ float red[8][GNN_H + 1];
    const int a = threadIdx.x % GNN_H, slot = threadIdx.x / GNN_H;
    const int64_t per = (n + gridDim.x - 1) / gridDim.x;
    const int64_t i0 = blockIdx.x * per, i1 = min(n, i0 + per);
    float s = 0.0f, sd = 0.0f;
    for (int64_t i = i0 + slot; i < i1; i += 8) {
        const float hi = bf2f(h2[i * GNN_H + a]);
        float q = 0.0f;
        for (int64_t p = ptr[i]; p < ptr[i + 1]; ++p) {
            const int32_t j = col[p];
            q += G[p] * bf2f(h2[(int64_t)j * GNN_H + a]);
            if (j == i) sd += G[p];
        }
        s += hi * q;
    }
    red[slot][a] = s;
    if (a == 0) red[slot][GNN_H] = sd;
    __syncthreads();
    float* P = part + (int64_t)blockIdx.x * GNN_P;
    if (threadIdx.x <= GNN_H) {
        float t = 0.0f;
        for (int k = 0; k < 8; ++k) t += red[k][threadIdx.x];
        P[threadIdx.x < GNN_H ? GNN_OFF_W3 + threadIdx.x : GNN_OFF_B3] = t;
    }
}

// zero-correction loss |b|^2 and the samples of one solve:
// zh = z / rms(z), bh = (t - K_m z) / (dbar rms(z)), z = V* - V_k
__global__ void k_stencil_sample(int64_t n, const int64_t* __restrict__ kptr, const int32_t* __restrict__ kcol,
                                 const double* __restrict__ kval, const double* __restrict__ z,
                                 const double* __restrict__ zz, const double* __restrict__ t, double dbar,
                                 float* __restrict__ zh, float* __restrict__ bh) {
    const int64_t i = blockIdx.x * (int64_t)BLOCK + threadIdx.x;
    if (i >= n) return;
    const double rms = sqrt(*zz / (double)n);
    double kz = 0.0;
    for (int64_t p = kptr[i]; p < kptr[i + 1]; ++p) kz += kval[p] * z[kcol[p]];
    zh[i] = rms > 0.0 ? (float)(z[i] / rms) : 0.0f;
    bh[i] = rms > 0.0 ? (float)((t[i] - kz) / (dbar * rms)) : 0.0f;
}

__global__ void k_sub(int64_t n, const double* __restrict__ a, const double* __restrict__ b,
                      double* __restrict__ out) {
    const int64_t i = blockIdx.x * (int64_t)BLOCK + threadIdx.x;
    if (i < n) out[i] = a[i] - b[i];
}

void launch_gnn_adam(hipStream_t s, float* theta, float* m, float* v, const float* grad, float scale,
                     float lr, int step, uint16_t* wbf) {
    const float c1 = 1.0f - powf(0.9f, (float)step), c2 = 1.0f - powf(0.999f, (float)step);
    k_adam<<<(GNN_P + BLOCK - 1) / BLOCK, BLOCK, 0, s>>>(theta, m, v, grad, scale, lr, c1, c2, wbf);
}

void launch_gnn_embed(hipStream_t s, int64_t n, const float* stat, const GnnGraph& A, const uint16_t* wbf,
                      GnnAct& a) {
    if (n <= 0) return;
    k_input<<<blocks_for(n * GNN_F), BLOCK, 0, s>>>(n, nullptr, nullptr, nullptr, stat, a.f);
    forward_common(s, n, A, wbf, a, 1, nullptr, nullptr, 1.0f);
}

void launch_stencil_values(hipStream_t s, const StencilPattern& P, const uint16_t* h2, const uint16_t* wbf,
                           float* cval) {
    if (P.nnz > 0) k_cvals<<<blocks_for(P.nnz), BLOCK, 0, s>>>(P.nnz, P.row, P.col, h2, wbf, cval);
}

void launch_stencil_sample_loss(hipStream_t s, const StencilPattern& P, const float* cval, const float* zh,
                                const float* bh, float* r, float* G, float* partials, double* loss) {
    const int64_t n = P.n;
    if (n <= 0) return;
    const unsigned nb = blocks_for(n);
    float* loss_part = partials + (int64_t)GNN_WG_BLOCKS * GNN_P;
    k_cspmv<<<nb, BLOCK, 0, s>>>(n, P.ptr, P.col, cval, zh, bh, r, loss_part);
    if (G) k_gacc<<<blocks_for(P.nnz), BLOCK, 0, s>>>(P.nnz, P.row, P.col, r, zh, G);
    k_reduce_grad<<<1, BLOCK, 0, s>>>(0, partials, nullptr, loss_part, (int)nb, loss);
}

void launch_stencil_backward(hipStream_t s, const StencilPattern& P, const GnnGraph& At, const float* G,
                             const uint16_t* wbf, GnnAct& a, float* partials, float* grad) {
    const int64_t n = P.n;
    if (n <= 0) return;
    const unsigned gb = blocks_for(n * GNN_H);
    const int wb = GNN_WG_BLOCKS;
    k_dh2<<<gb, BLOCK, 0, s>>>(n, P.ptr, P.col, P.tpos, G, a.h2, wbf, a.dz2);
    k_w3grad<<<wb, 256, 0, s>>>(n, P.ptr, P.col, G, a.h2, partials);
    k_bwd_g<<<gb, BLOCK, 0, s>>>(n, a.dz2, wbf, a.g2);
    k_bwd_hidden<<<gb, BLOCK, 0, s>>>(n, a.dz2, a.g2, At.ptr, At.col, At.val, a.h1, wbf, a.dz1);
    k_wgrad_mfma<GNN_H><<<wb, 256, 0, s>>>(n, a.dz2, a.h1, partials, GNN_OFF_W2S, GNN_OFF_B2);
    k_wgrad_mfma<GNN_H><<<wb, 256, 0, s>>>(n, a.dz2, a.m1, partials, GNN_OFF_W2N, -1);
    k_wgrad_mfma<GNN_F><<<wb, 256, 0, s>>>(n, a.dz1, a.f, partials, GNN_OFF_W1S, GNN_OFF_B1);
    k_wgrad_mfma<GNN_F><<<wb, 256, 0, s>>>(n, a.dz1, a.m0, partials, GNN_OFF_W1N, -1);
    k_reduce_grad<<<(GNN_P + BLOCK - 1) / BLOCK, BLOCK, 0, s>>>(wb, partials, grad, nullptr, 0, nullptr);
}

void launch_gnn_sub(hipStream_t s, int64_t n, const double* a, const double* b, double* out) {
    if (n > 0) k_sub<<<blocks_for(n), BLOCK, 0, s>>>(n, a, b, out);
}

void launch_stencil_sample(hipStream_t s, int64_t n, const StencilKm& K, const double* z, const double* zz,
                           const double* t, double dbar, float* zh, float* bh) {
    if (n > 0) k_stencil_sample<<<blocks_for(n), BLOCK, 0, s>>>(n, K.ptr, K.col, K.val, z, zz, t, dbar, zh, bh);
}

void launch_gnn_to_bf16(hipStream_t s, const float* theta, uint16_t* wbf) {
    k_to_bf16<<<(GNN_P + BLOCK - 1) / BLOCK, BLOCK, 0, s>>>(theta, wbf);
}

void launch_gnn_store_sample(hipStream_t s, int64_t n, const double* t, const double* tn2, float* that) {
    if (n > 0) k_store_sample<<<blocks_for(n), BLOCK, 0, s>>>(n, t, tn2, that);
}

void launch_gnn_finish_targets(hipStream_t s, int64_t n, const double* vstar, const double* d,
                               const double* tn2, float* y) {
    if (n > 0) k_finish_targets<<<blocks_for(n), BLOCK, 0, s>>>(n, vstar, d, tn2, y);
}

void launch_gnn_pending(hipStream_t s, int64_t n, const double* xv, const double* z2, double* d) {
    if (n > 0) k_pending<<<blocks_for(n), BLOCK, 0, s>>>(n, xv, z2, d);
}

}  // namespace bido
