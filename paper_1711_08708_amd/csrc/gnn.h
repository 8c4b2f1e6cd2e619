// Learned correction of the Schur-complement solve: a two-layer message
// passing network on the heart vertices (hidden width 32), BF16 weights and
// activations with FP32 accumulation.  Parameter vector layout (FP32 master
// copy and BF16 working copy share it):
//   W1s (32x16) W1n (32x16) b1 (32) W2s (32x32) W2n (32x32) b2 (32) w3 (32) b3 (1)
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace bido {

constexpr int GNN_F = 16;
constexpr int GNN_H = 32;
constexpr int GNN_OFF_W1S = 0;
constexpr int GNN_OFF_W1N = GNN_OFF_W1S + GNN_H * GNN_F;
constexpr int GNN_OFF_B1 = GNN_OFF_W1N + GNN_H * GNN_F;
constexpr int GNN_OFF_W2S = GNN_OFF_B1 + GNN_H;
constexpr int GNN_OFF_W2N = GNN_OFF_W2S + GNN_H * GNN_H;
constexpr int GNN_OFF_B2 = GNN_OFF_W2N + GNN_H * GNN_H;
constexpr int GNN_OFF_W3 = GNN_OFF_B2 + GNN_H;
constexpr int GNN_OFF_B3 = GNN_OFF_W3 + GNN_H;
constexpr int GNN_P = GNN_OFF_B3 + 1;          // 3169 parameters
constexpr int GNN_WG_BLOCKS = 1024;            // partial-sum blocks of the weight gradients

struct GnnGraph {                 // row-normalised neighbour weights (internal v order)
    int64_t n = 0;
    int64_t* ptr = nullptr;
    int32_t* col = nullptr;
    float* val = nullptr;
};

struct StencilPattern {           // stored pattern of S_m, internal v order
    int64_t n = 0, nnz = 0;
    int64_t* ptr = nullptr;
    int32_t* col = nullptr;
    int32_t* row = nullptr;       // row of each entry
    int32_t* tpos = nullptr;      // entry of the transposed position
};

struct StencilKm {                // K_m = gamma M_H + S_m, FP64, internal v order
    int64_t* ptr = nullptr;
    int32_t* col = nullptr;
    double* val = nullptr;
};

struct GnnAct {                   // activations of one forward pass
    uint16_t *f = nullptr, *m0 = nullptr, *h1 = nullptr, *m1 = nullptr, *h2 = nullptr;  // bf16
    float* o = nullptr;
    float* dout = nullptr;        // d loss / d o
    float* res = nullptr;         // o - target
    float* zero = nullptr;        // all zeros (loss of the zero correction)
    float *dz2 = nullptr, *g2 = nullptr, *dz1 = nullptr;
};

// forward: features from t (|t|^2 at *tn2; input t / rms(t), rms = |t| / sqrt(n)),
// both layers, readout.  mode 0: z2[i] += rms(t) * out_scale * o_i (inference);
// mode 1: keep o (training)
void launch_gnn_forward(hipStream_t s, int64_t n, const double* t, const double* tn2, const float* stat,
                        const GnnGraph& A, const uint16_t* wbf, GnnAct& a, int mode, double* z2,
                        float out_scale);
// sample input from a stored feature column (t / |t| already, FP32)
void launch_gnn_forward_sample(hipStream_t s, int64_t n, const float* that, const float* stat,
                               const GnnGraph& A, const uint16_t* wbf, GnnAct& a);
// backward of the energy loss r^T W r, r = o - y * yinv: loss partials and
// weight-gradient partials (GNN_WG_BLOCKS x GNN_P), then `grad += sum of
// partials` and loss += sum.  At is the transposed neighbour graph.
void launch_gnn_backward(hipStream_t s, int64_t n, const float* y, const GnnGraph& W, const GnnGraph& At,
                         const uint16_t* wbf, GnnAct& a, float* partials, float* grad, double* loss,
                         float yinv);
void launch_gnn_loss(hipStream_t s, int64_t n, const float* y, const GnnGraph& W, GnnAct& a,
                     float* partials, double* loss, float yinv);
void launch_gnn_sumsq(hipStream_t s, int64_t n, const float* y, float* partials, double* out);
void launch_gnn_energy0(hipStream_t s, int64_t n, const float* y, const GnnGraph& W, GnnAct& a,
                        float* partials, double* out, float yinv);
void launch_gnn_adam(hipStream_t s, float* theta, float* m, float* v, const float* grad, float scale,
                     float lr, int step, uint16_t* wbf);
void launch_gnn_to_bf16(hipStream_t s, const float* theta, uint16_t* wbf);

// learned Schur-complement stencil (K_m + C, Sec. 5.2): embeddings from the
// static features, stencil values, per-sample residual/loss (G += dloss/dC
// when G is given), backward from G to the weight gradient, sample targets
void launch_gnn_embed(hipStream_t s, int64_t n, const float* stat, const GnnGraph& A, const uint16_t* wbf,
                      GnnAct& a);
void launch_stencil_values(hipStream_t s, const StencilPattern& P, const uint16_t* h2, const uint16_t* wbf,
                           float* cval);
void launch_stencil_sample_loss(hipStream_t s, const StencilPattern& P, const float* cval, const float* zh,
                                const float* bh, float* r, float* G, float* partials, double* loss);
void launch_stencil_backward(hipStream_t s, const StencilPattern& P, const GnnGraph& At, const float* G,
                             const uint16_t* wbf, GnnAct& a, float* partials, float* grad);
void launch_gnn_sub(hipStream_t s, int64_t n, const double* a, const double* b, double* out);
void launch_stencil_sample(hipStream_t s, int64_t n, const StencilKm& K, const double* z, const double* zz,
                           const double* t, double dbar, float* zh, float* bh);
void launch_gnn_store_sample(hipStream_t s, int64_t n, const double* t, const double* tn2, float* that);
void launch_gnn_finish_targets(hipStream_t s, int64_t n, const double* vstar, const double* d,
                               const double* tn2, float* y);
void launch_gnn_pending(hipStream_t s, int64_t n, const double* xv, const double* z2, double* d);

}  // namespace bido
