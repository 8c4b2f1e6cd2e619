// HIP kernels for gfx950 (CDNA4, 64-lane wavefronts).
//
//   tri_*               sweeps of the multifrontal Cholesky inner solves
//                       P_1^-1, P_K^-1 (Def. 2, Sec. 5.3): subtree phase,
//                       level phases with their combine launches, top
//                       (dense or hierarchical inverse of the top Schur
//                       complement)
//   spmv_*              Lambda products (Sec. 3.2, eq. (system)) and the
//                       S_i Pi / Pi^T S_i products of the preconditioner
//   pcg_*, p_update,    FP64 CG recurrences; each reduction leaves one partial
//   combine_dot         per block and the kernel that needs the total sums
//                       the partials itself, in a fixed order (no fences)
//   ionic_rhs           Steps 1 and 3 of the resolution algorithm
//   dot_reduce,         normalisation (M U, 1) = 0 of Prop. 1 (the last
//   gather_out          block reduces: once per step)
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>

#include "kernels.h"
#include "launch.h"
#include "rows.h"

namespace bido {

constexpr int BLOCK = 256;
constexpr int WAVE = 64;

// ---------------------------------------------------------------------------
// reductions
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = WAVE / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, WAVE);
    return v;
}

// Sum over the block (BLOCK threads); result valid in every thread.
__device__ __forceinline__ double block_sum(double v, double* sh) {
    v = wave_sum(v);
    const int lane = threadIdx.x % WAVE, w = threadIdx.x / WAVE;
    __syncthreads();
    if (lane == 0) sh[w] = v;
    __syncthreads();
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < BLOCK / WAVE; ++i) s += sh[i];
    return s;
}

// Store this block's partials; the last block to arrive sums all partials in
// block order (deterministic) and writes them to out[0..K).
template <int K>
__device__ void finish_reduce(const double (&part)[K], double* partials, unsigned* counter,
                              double* out, double* sh) {
    __shared__ bool last;
    if (threadIdx.x == 0) {
        for (int k = 0; k < K; ++k) partials[(size_t)k * gridDim.x + blockIdx.x] = part[k];
        __threadfence();
        unsigned t = atomicAdd(counter, 1u);
        last = (t == gridDim.x - 1);
    }
    __syncthreads();
    if (!last) return;
    __threadfence();
    for (int k = 0; k < K; ++k) {
        double s = 0.0;
        for (unsigned b = threadIdx.x; b < gridDim.x; b += BLOCK)
            s += partials[(size_t)k * gridDim.x + b];
        s = block_sum(s, sh);
        if (threadIdx.x == 0) out[k] = s;
    }
    if (threadIdx.x == 0) *counter = 0u;
}

// ---------------------------------------------------------------------------
// simple vector kernels
// ---------------------------------------------------------------------------
__global__ void k_fill(int64_t n, double* x, double v) {
    for (int64_t i = blockIdx.x * (int64_t)BLOCK + threadIdx.x; i < n; i += (int64_t)gridDim.x * BLOCK)
        x[i] = v;
}

__global__ void k_add2(int64_t n, const double* __restrict__ a, const double* __restrict__ b,
                       double* __restrict__ out) {
    for (int64_t i = blockIdx.x * (int64_t)BLOCK + threadIdx.x; i < n; i += (int64_t)gridDim.x * BLOCK)
        out[i] = a[i] + b[i];
}

// y = A x for a dense n x n row-major A: one wave per row, the lanes stride
// the row (coalesced), a wave reduction.
template <typename V>
__global__ __launch_bounds__(BLOCK) void k_dense_gemv(int64_t n, const double* __restrict__ A,
                                                      const V* __restrict__ x, V* __restrict__ y) {
    const int lane = threadIdx.x % WAVE;
    const int64_t nw = (int64_t)gridDim.x * (BLOCK / WAVE);
    for (int64_t r = (blockIdx.x * (int64_t)BLOCK + threadIdx.x) / WAVE; r < n; r += nw) {
        const double* a = A + r * n;
        double s = 0.0;
        for (int64_t j = lane; j < n; j += WAVE) s += a[j] * (double)x[j];
        s = wave_sum(s);
        if (lane == 0) y[r] = (V)s;
    }
}

__global__ void k_axpy(int64_t n, double a, const double* __restrict__ x, double* __restrict__ y) {
    for (int64_t i = blockIdx.x * (int64_t)BLOCK + threadIdx.x; i < n; i += (int64_t)gridDim.x * BLOCK)
        y[i] += a * x[i];
}

// dst[pos[i]] = src[i]
__global__ void k_scatter_in(int64_t n, const int64_t* __restrict__ pos,
                             const double* __restrict__ src, double* __restrict__ dst) {
    for (int64_t i = blockIdx.x * (int64_t)BLOCK + threadIdx.x; i < n; i += (int64_t)gridDim.x * BLOCK)
        dst[pos[i]] = src[i];
}

// float variant
__global__ void k_scatter_in_f(int64_t n, const int64_t* __restrict__ pos, const float* __restrict__ src,
                               float* __restrict__ dst) {
    for (int64_t i = blockIdx.x * (int64_t)BLOCK + threadIdx.x; i < n; i += (int64_t)gridDim.x * BLOCK)
        dst[pos[i]] = src[i];
}

__global__ void k_gather_f(int64_t n, const int64_t* __restrict__ pos, const float* __restrict__ src,
                           float* __restrict__ dst) {
    for (int64_t i = blockIdx.x * (int64_t)BLOCK + threadIdx.x; i < n; i += (int64_t)gridDim.x * BLOCK)
        dst[i] = src[pos[i]];
}

// dst[i] = src[pos[i]] - (shift ? *shift_num / shift_den : 0)
__global__ void k_gather_out(int64_t n, const int64_t* __restrict__ pos,
                             const double* __restrict__ src, double* __restrict__ dst,
                             const double* __restrict__ sc, int shift_slot, double shift_den) {
    const double s = shift_slot >= 0 ? sc[shift_slot] / shift_den : 0.0;
    for (int64_t i = blockIdx.x * (int64_t)BLOCK + threadIdx.x; i < n; i += (int64_t)gridDim.x * BLOCK)
        dst[i] = src[pos[i]] - s;
}

// dst[i] = src[pos[i]] for the new potential V^{n+1}, and the activation
// time of vertex i: the first time its potential reaches v_act, linearly
// interpolated between t_n (V^n = the old dst[i]) and t_n + dt; act < 0
// marks a vertex not reached yet
__global__ void k_gather_v_act(int64_t n, const int64_t* __restrict__ pos, const double* __restrict__ src,
                               double* __restrict__ dst, double* __restrict__ act, double v_act, double t_n,
                               double dt) {
    for (int64_t i = blockIdx.x * (int64_t)BLOCK + threadIdx.x; i < n; i += (int64_t)gridDim.x * BLOCK) {
        const double vo = dst[i], vn = src[pos[i]], a = act[i];
        dst[i] = vn;
        if (a < 0.0 && vn >= v_act) act[i] = vo >= v_act ? t_n : t_n + dt * (v_act - vo) / (vn - vo);
    }
}

// out[q] = sum_k w[q][k] u[id[q][k]]: the P1 interpolant of u at probe q
__global__ void k_probe(int np, int nv, const int64_t* __restrict__ ids, const double* __restrict__ wts,
                        const double* __restrict__ u, double* __restrict__ out) {
    const int q = blockIdx.x * BLOCK + threadIdx.x;
    if (q >= np) return;
    double s = 0.0;
    for (int k = 0; k < nv; ++k) s += wts[q * nv + k] * u[ids[q * nv + k]];
    out[q] = s;
}

// (M U, 1) for the normalisation, and optionally sum of a second vector
__global__ void k_dot_reduce(int64_t n, const double* __restrict__ a, const double* __restrict__ b,
                             double* partials, unsigned* counter, double* out) {
    __shared__ double sh[BLOCK / WAVE];
    double s = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)BLOCK + threadIdx.x; i < n; i += (int64_t)gridDim.x * BLOCK)
        s += b ? a[i] * b[i] : a[i];
    s = block_sum(s, sh);
    double part[1] = {s};
    finish_reduce<1>(part, partials, counter, out, sh);
}

// ---------------------------------------------------------------------------
// Initial guess of a step's solve: the Lambda-orthogonal projection of the
// solution onto the span of the states W_k the last steps started from
// (Fischer's projection for a sequence of right-hand sides): x0 = W c with
// (W^T Lambda W) c = W^T Y.  The Gram matrix G is kept by ring slot and gets
// one new row per step; everything stays on the device.
// ---------------------------------------------------------------------------
// out[k] = W_k . y for k < W.m (out[k] = 0 beyond).  The m sums of a block
// are reduced wave by wave with shuffles and combined after one barrier;
// the last block to finish (a counter) sums the blocks' partials, one wave
// per sum (the counter is reset for the next call).
__global__ void k_multidot(int64_t n, GuessList W, const double* __restrict__ y, double* partials,
                           unsigned* counter, double* out) {
    constexpr int NW = BLOCK / WAVE;
    __shared__ double sh[GUESS_MAX][NW];
    __shared__ bool last;
    const int m = W.m, lane = threadIdx.x % WAVE, wv = threadIdx.x / WAVE;
    double part[GUESS_MAX];
#pragma unroll
    for (int k = 0; k < GUESS_MAX; ++k) part[k] = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)BLOCK + threadIdx.x; i < n; i += (int64_t)gridDim.x * BLOCK) {
        const double yi = y[i];
#pragma unroll
        for (int k = 0; k < GUESS_MAX; ++k)
            if (k < m) part[k] += W.v[k][i] * yi;
    }
#pragma unroll
    for (int k = 0; k < GUESS_MAX; ++k)
        if (k < m) {
            const double v = wave_sum(part[k]);
            if (lane == 0) sh[k][wv] = v;
        }
    __syncthreads();
    if ((int)threadIdx.x < m) {
        double s = 0.0;
#pragma unroll
        for (int w = 0; w < NW; ++w) s += sh[threadIdx.x][w];
        partials[(size_t)threadIdx.x * gridDim.x + blockIdx.x] = s;
    }
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) last = atomicAdd(counter, 1u) == gridDim.x - 1;
    __syncthreads();
    if (!last) return;
    __threadfence();
    for (int k = wv; k < GUESS_MAX; k += NW) {
        double s = 0.0;
        if (k < m)
            for (unsigned b = lane; b < gridDim.x; b += WAVE) s += partials[(size_t)k * gridDim.x + b];
        s = wave_sum(s);
        if (lane == 0) out[k] = k < m ? s : 0.0;
    }
    if (threadIdx.x == 0) *counter = 0u;
}

// One workgroup: the new Gram row (d[k] = W_k . Lambda W_0, W_0 the newest,
// at ring slot W.slot[0]) into G (ld GUESS_MAX, by slot), then, when b is
// given, c from (G_W + delta I) c = b by Cholesky, delta = 1e-13 times the
// largest diagonal entry (the states are close to dependent); a failed
// factorisation keeps x0 = W_0 (c = e_0).  The threads stage G_W in LDS;
// one thread factors and solves there.
__global__ void k_guess_solve(GuessList W, const double* __restrict__ d, double* G, const double* __restrict__ b,
                              double* __restrict__ c) {
    __shared__ double L[GUESS_MAX][GUESS_MAX];
    __shared__ double z[GUESS_MAX];
    const int m = W.m, t = threadIdx.x;
    if (d && t < m) {
        G[W.slot[0] * GUESS_MAX + W.slot[t]] = d[t];
        G[W.slot[t] * GUESS_MAX + W.slot[0]] = d[t];
    }
    if (!b) return;
    __syncthreads();
    for (int e = t; e < m * m; e += blockDim.x) {
        const int i = e / m, k = e - i * m;
        L[i][k] = G[W.slot[i] * GUESS_MAX + W.slot[k]];
    }
    if (t < m) z[t] = b[t];
    __syncthreads();
    if (t != 0) return;
    double dmax = 0.0;
    for (int k = 0; k < m; ++k) dmax = fmax(dmax, L[k][k]);
    const double delta = 1e-13 * dmax;
    bool ok = dmax > 0.0;
    for (int i = 0; i < m && ok; ++i)                 // lower triangle in place
        for (int j = 0; j <= i; ++j) {
            double s = L[i][j] + (i == j ? delta : 0.0);
            for (int k = 0; k < j; ++k) s -= L[i][k] * L[j][k];
            if (i == j) {
                if (!(s > 0.0)) { ok = false; break; }
                L[i][i] = sqrt(s);
            } else {
                L[i][j] = s / L[j][j];
            }
        }
    if (!ok) {
        for (int k = 0; k < m; ++k) c[k] = k == 0 ? 1.0 : 0.0;
        return;
    }
    for (int i = 0; i < m; ++i) {                      // L z = b
        double s = z[i];
        for (int k = 0; k < i; ++k) s -= L[i][k] * z[k];
        z[i] = s / L[i][i];
    }
    for (int i = m - 1; i >= 0; --i) {                 // L^T c = z, c kept in z
        double s = z[i];
        for (int k = i + 1; k < m; ++k) s -= L[k][i] * z[k];
        z[i] = s / L[i][i];
    }
    for (int k = 0; k < m; ++k) c[k] = z[k];
}

// x = sum_k c[k] W_k
__global__ void k_guess_combine(int64_t n, GuessList W, const double* __restrict__ c, double* __restrict__ x) {
    double ck[GUESS_MAX];
#pragma unroll
    for (int k = 0; k < GUESS_MAX; ++k) ck[k] = k < W.m ? c[k] : 0.0;
    for (int64_t i = blockIdx.x * (int64_t)BLOCK + threadIdx.x; i < n; i += (int64_t)gridDim.x * BLOCK) {
        double s = 0.0;
#pragma unroll
        for (int k = 0; k < GUESS_MAX; ++k)
            if (k < W.m) s += ck[k] * W.v[k][i];
        x[i] = s;
    }
}

// x[i] -= sc[slot] / den   for i < n
__global__ void k_shift(int64_t n, double* x, const double* sc, int slot, double den) {
    const double s = sc[slot] / den;
    for (int64_t i = blockIdx.x * (int64_t)BLOCK + threadIdx.x; i < n; i += (int64_t)gridDim.x * BLOCK)
        x[i] -= s;
}

// ---------------------------------------------------------------------------
// Steps 1 and 3 (Mitchell-Schaeffer), heart-local order in, internal out.
// ---------------------------------------------------------------------------
__global__ void k_ionic_rhs(int64_t nh, const double* __restrict__ v, double* __restrict__ h,
                            const double* __restrict__ stim, double stim_on,
                            const double* __restrict__ mh, const int64_t* __restrict__ pos,
                            double* __restrict__ y2, double* __restrict__ x2,
                            const double* __restrict__ sub, IonicConst c) {
    for (int64_t k = blockIdx.x * (int64_t)BLOCK + threadIdx.x; k < nh; k += (int64_t)gridDim.x * BLOCK) {
        const double V = v[k], hk = h[k];
        const double vt = V * c.inv_dv;
        const double iion = c.cm * c.dv * (-hk * vt * vt * (1.0 - vt) * c.inv_tau_in + vt * c.inv_tau_out);
        const double ist = stim[k] * stim_on;
        const int64_t p = pos[k];
        y2[p] = c.scale * mh[k] * (c.gamma * V - c.reaction * c.chi * (iion - ist)) - (sub ? sub[p] : 0.0);
        x2[p] = V;
        if (c.reaction != 0.0) {
            const double g = (vt < c.v_gate) ? (1.0 - hk) * c.inv_tau_open : -hk * c.inv_tau_close;
            h[k] = hk + c.dt * g;
        }
    }
}

// Strang splitting: the reaction c dV/dt = I_st - I_ion(V, h), dh/dt = g(V, h)
// advanced pointwise by Heun's method over tau = dt/2 before and after the
// diffusion step
__device__ __forceinline__ void ms_rates(double V, double hk, double ist, const IonicConst& c, double& dv,
                                         double& dh) {
    const double vt = V * c.inv_dv;
    const double iion = c.cm * c.dv * (-hk * vt * vt * (1.0 - vt) * c.inv_tau_in + vt * c.inv_tau_out);
    dv = (ist - iion) / c.cm;
    dh = (vt < c.v_gate) ? (1.0 - hk) * c.inv_tau_open : -hk * c.inv_tau_close;
}
__device__ __forceinline__ void ms_heun(double& V, double& hk, double ist, double tau, const IonicConst& c) {
    double a1, b1, a2, b2;
    ms_rates(V, hk, ist, c, a1, b1);
    ms_rates(V + tau * a1, hk + tau * b1, ist, c, a2, b2);
    V += 0.5 * tau * (a1 + a2);
    hk += 0.5 * tau * (b1 + b2);
}
// first half-step from (V^n, h^n): vs = V*, h <- h*  (heart-local order)
__global__ void k_strang_in(int64_t nh, const double* __restrict__ v, double* __restrict__ h,
                            const double* __restrict__ stim, double stim_on, double tau, IonicConst c,
                            double* __restrict__ vs) {
    for (int64_t k = blockIdx.x * (int64_t)BLOCK + threadIdx.x; k < nh; k += (int64_t)gridDim.x * BLOCK) {
        double V = v[k], hk = h[k];
        ms_heun(V, hk, stim[k] * stim_on, tau, c);
        vs[k] = V;
        h[k] = hk;
    }
}
// second half-step from (V**, h*), V** = x2[pos[k]] the diffusion step's
// output: v <- V^{n+1}, h <- h^{n+1}; with act, the activation time of the
// step (V^n = the old v, linear in time between t_n and t_n + dt)
__global__ void k_strang_out(int64_t nh, const int64_t* __restrict__ pos, const double* __restrict__ x2,
                             double* __restrict__ v, double* __restrict__ h, const double* __restrict__ stim,
                             double stim_on, double tau, IonicConst c, double* __restrict__ act, double v_act,
                             double t_n, double dt) {
    for (int64_t k = blockIdx.x * (int64_t)BLOCK + threadIdx.x; k < nh; k += (int64_t)gridDim.x * BLOCK) {
        const double vo = v[k];
        double V = x2[pos[k]], hk = h[k];
        ms_heun(V, hk, stim[k] * stim_on, tau, c);
        v[k] = V;
        h[k] = hk;
        if (act && act[k] < 0.0 && V >= v_act) act[k] = vo >= v_act ? t_n : t_n + dt * (v_act - vo) / (V - vo);
    }
}

// ---------------------------------------------------------------------------
// Lambda products.  Rows handled by groups of G lanes.
// ---------------------------------------------------------------------------

// mode 0: q = A p, block partial of p.q            (region PP_PQ)
// mode 1: r = y - A x, block partials of |r|^2, |y|^2 (PP_RR, PP_YY)
template <int G, int MODE>
__global__ __launch_bounds__(BLOCK) void k_spmv_lambda(int64_t n, const int64_t* __restrict__ ptr,
                                                       const int32_t* __restrict__ col,
                                                       const double* __restrict__ val,
                                                       const double* __restrict__ x,
                                                       const double* __restrict__ y,
                                                       double* __restrict__ out, double* __restrict__ pp) {
    __shared__ double sh[BLOCK / WAVE];
    constexpr int RU = SPMV_RU;
    constexpr int GPB = BLOCK / G;    // lane groups per workgroup
    const int lane = threadIdx.x % G;
    const RowRange rr = block_rows(n);
    double acc0 = 0.0, acc1 = 0.0;
    for (int64_t rb = rr.r0 + threadIdx.x / G; rb < rr.r1; rb += RU * GPB) {
        int64_t row[RU];
        bool ok[RU];
        double own[RU];   // x[row] (p.q) or y[row] (residual), loaded with the rows
#pragma unroll
        for (int u = 0; u < RU; ++u) {
            row[u] = rb + u * GPB;
            ok[u] = row[u] < rr.r1;
            own[u] = (MODE == 0 ? x : y)[ok[u] ? row[u] : rb];
        }
        double s[RU];
        csr_rows<G, RU>(ptr, col, val, x, row, ok, lane, s);
        if (lane == 0) {
#pragma unroll
            for (int u = 0; u < RU; ++u) {
                if (!ok[u]) continue;
                if (MODE == 0) {
                    out[row[u]] = s[u];
                    acc0 += s[u] * own[u];
                } else {
                    const double rv = own[u] - s[u];
                    out[row[u]] = rv;
                    acc0 += rv * rv;
                    acc1 += own[u] * own[u];
                }
            }
        }
    }
    acc0 = block_sum(acc0, sh);
    if (MODE == 0) {
        if (threadIdx.x == 0) pp[pp_offset(PP_PQ) + blockIdx.x] = acc0;
    } else {
        acc1 = block_sum(acc1, sh);
        if (threadIdx.x == 0) {
            pp[pp_offset(PP_RR) + blockIdx.x] = acc0;
            pp[pp_offset(PP_YY) + blockIdx.x] = acc1;
        }
    }
}

// The same products on the blocked form of Lambda (Pi = I, one order for u
// and v): row k gives the u output k and the v output N + k from one pass
// over its positions (column, {S_1, S_i}), gathering x_u and x_v at each
// column; partials as in k_spmv_lambda.
template <int G, int K, int MODE, typename C>
__global__ __launch_bounds__(BLOCK) void k_spmv_lam_blk(int64_t n, const int64_t* __restrict__ ptr,
                                                        const C* __restrict__ col,
                                                        const int32_t* __restrict__ cb,
                                                        const double2* __restrict__ val,
                                                        const double* __restrict__ gm,
                                                        const double* __restrict__ x,
                                                        const double* __restrict__ y,
                                                        double* __restrict__ out, double* __restrict__ pp) {
    __shared__ double sh[BLOCK / WAVE];
    constexpr int RU = 2;               // (four: 5.8 ms per step on the 128^3 slab, two: 5.4)
    constexpr int GPB = BLOCK / G;
    const int lane = threadIdx.x % G;
    const double* __restrict__ xv = x + n;
    const RowRange rr = block_rows(n);
    double acc0 = 0.0, acc1 = 0.0;
    for (int64_t rb = rr.r0 + threadIdx.x / G; rb < rr.r1; rb += RU * GPB) {
        int64_t row[RU], pb[RU], pe[RU];
        int32_t c0[RU];
        bool ok[RU];
        double su[RU], sv[RU];
#pragma unroll
        for (int u = 0; u < RU; ++u) {
            row[u] = rb + u * GPB;
            ok[u] = row[u] < rr.r1;
            const int64_t r = ok[u] ? row[u] : rb;
            pb[u] = ptr[r];
            pe[u] = ptr[r + 1];
            if constexpr (sizeof(C) == 2) c0[u] = cb[r];     // 16-bit offsets from the row's base
            else c0[u] = 0;
            su[u] = 0.0;
            sv[u] = 0.0;
        }
        // K unconditional passes (an entry past the row's end rereads
        // position 0 and is dropped by a select), then the rest of the row
#pragma unroll
        for (int k = 0; k < K; ++k)
#pragma unroll
            for (int u = 0; u < RU; ++u) {
                const int64_t q = pb[u] + lane + k * G;
                const bool in = q < pe[u];
                const int64_t qc = in ? q : 0;
                const int32_t c = c0[u] + (int32_t)col[qc];
                const double2 w = val[qc];
                const double a = x[c], b = xv[c];
                su[u] += in ? w.x * a + w.y * b : 0.0;
                sv[u] += in ? w.y * (a + b) : 0.0;
            }
#pragma unroll
        for (int u = 0; u < RU; ++u)
            for (int64_t q = pb[u] + lane + K * G; q < pe[u]; q += G) {
                const int32_t c = c0[u] + (int32_t)col[q];
                const double2 w = val[q];
                const double a = x[c], b = xv[c];
                su[u] += w.x * a + w.y * b;
                sv[u] += w.y * (a + b);
            }
#pragma unroll
        for (int u = 0; u < RU; ++u) {
            su[u] = lane_group_sum<G>(su[u]);
            sv[u] = lane_group_sum<G>(sv[u]);
        }
        if (lane == 0) {
#pragma unroll
            for (int u = 0; u < RU; ++u) {
                if (!ok[u]) continue;
                const int64_t k = row[u];
                const double yu = su[u], yv = sv[u] + gm[k] * xv[k];
                if (MODE == 0) {
                    out[k] = yu;
                    out[n + k] = yv;
                    acc0 += yu * x[k] + yv * xv[k];
                } else {
                    const double bu = y[k], bv = y[n + k];
                    const double ru = bu - yu, rv = bv - yv;
                    out[k] = ru;
                    out[n + k] = rv;
                    acc0 += ru * ru + rv * rv;
                    acc1 += bu * bu + bv * bv;
                }
            }
        }
    }
    acc0 = block_sum(acc0, sh);
    if (MODE == 0) {
        if (threadIdx.x == 0) pp[pp_offset(PP_PQ) + blockIdx.x] = acc0;
    } else {
        acc1 = block_sum(acc1, sh);
        if (threadIdx.x == 0) {
            pp[pp_offset(PP_RR) + blockIdx.x] = acc0;
            pp[pp_offset(PP_YY) + blockIdx.x] = acc1;
        }
    }
}

// y = b - A x  (b may be null: y = A x), rows of a CSR block (one row per
// group at a time: Pi^T S_i has mostly empty rows, the torso vertices)
template <int G>
__global__ __launch_bounds__(BLOCK) void k_spmv_csr(int64_t n, const int64_t* __restrict__ ptr,
                                                    const int32_t* __restrict__ col,
                                                    const double* __restrict__ val,
                                                    const double* __restrict__ x,
                                                    const double* __restrict__ b,
                                                    double* __restrict__ y) {
    const int lane = threadIdx.x % G;
    const RowRange rr = block_rows(n);
    for (int64_t r = rr.r0 + threadIdx.x / G; r < rr.r1; r += BLOCK / G) {
        double s = 0.0;
        for (int64_t p = ptr[r] + lane; p < ptr[r + 1]; p += G) s += val[p] * x[col[p]];
        s = lane_group_sum<G>(s);
        if (lane == 0) y[r] = b ? b[r] - s : s;
    }
}

// ---------------------------------------------------------------------------
// P_K by Chebyshev acceleration of the Jacobi iteration on K_m (z_0 = 0):
// d_0 = z = D^-1 t / theta, then per step r -= K_m d, d <- c1 d + c2 D^-1 r,
// z += d (coefficients from the spectral interval, set up on the host)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(BLOCK) void k_cheb_init(int64_t n, const double* __restrict__ t,
                                                     const double* __restrict__ dinv, double inv_theta,
                                                     double* __restrict__ d, double* __restrict__ z) {
    for (int64_t i = blockIdx.x * (int64_t)BLOCK + threadIdx.x; i < n; i += (int64_t)gridDim.x * BLOCK) {
        const double v = inv_theta * dinv[i] * t[i];
        d[i] = v;
        z[i] = v;
    }
}

// r = r_in - K dp ; dn = c1 dp + c2 D^-1 r ; z += dn.  r_in and r may be one
// array (a row reads and writes only its own entry); dp and dn differ, since
// other rows gather dp.  The last step writes z only.
template <int G>
__global__ __launch_bounds__(BLOCK) void k_cheb_step(int64_t n, const int64_t* __restrict__ ptr,
                                                     const int32_t* __restrict__ col,
                                                     const double* __restrict__ val,
                                                     const double* __restrict__ dinv, const double* r_in,
                                                     double* r, const double* __restrict__ dp,
                                                     double* __restrict__ dn, double* __restrict__ z,
                                                     double c1, double c2, int last) {
    constexpr int RU = SPMV_RU;
    constexpr int GPB = BLOCK / G;
    const int lane = threadIdx.x % G;
    const RowRange rr = block_rows(n);
    for (int64_t rb = rr.r0 + threadIdx.x / G; rb < rr.r1; rb += RU * GPB) {
        int64_t row[RU];
        bool ok[RU];
        double rv[RU], dv[RU], di[RU], zv[RU];   // the rows' own entries, loaded with the rows
#pragma unroll
        for (int u = 0; u < RU; ++u) {
            row[u] = rb + u * GPB;
            ok[u] = row[u] < rr.r1;
            const int64_t i = ok[u] ? row[u] : rb;
            rv[u] = r_in[i];
            dv[u] = dp[i];
            di[u] = dinv[i];
            zv[u] = z[i];
        }
        double s[RU];
        csr_rows<G, RU>(ptr, col, val, dp, row, ok, lane, s);
        if (lane == 0) {
#pragma unroll
            for (int u = 0; u < RU; ++u) {
                if (!ok[u]) continue;
                const double rn = rv[u] - s[u];
                const double d = c1 * dv[u] + c2 * di[u] * rn;
                z[row[u]] = zv[u] + d;
                if (!last) {
                    r[row[u]] = rn;
                    dn[row[u]] = d;
                }
            }
        }
    }
}

// ---------------------------------------------------------------------------
// PCG vector recurrences
// ---------------------------------------------------------------------------
// Sum of nb block partials, in the same order in every block.
__device__ __forceinline__ double sum_partials(const double* __restrict__ part, int nb, double* sh) {
    double s = 0.0;
    for (int b = threadIdx.x; b < nb; b += BLOCK) s += part[b];
    return block_sum(s, sh);
}

// alpha = rho / p.q (p.q from the SpMV's nb_pq partials); x += alpha p ;
// r -= alpha q ; block partials of |r|^2.  Block 0 records p.q and alpha.
__global__ __launch_bounds__(BLOCK) void k_pcg_update(int64_t n, double* __restrict__ x,
                                                      double* __restrict__ r,
                                                      double* __restrict__ r_old,
                                                      const double* __restrict__ p,
                                                      const double* __restrict__ q,
                                                      double* __restrict__ pp, int nb_pq, int rho_slot) {
    __shared__ double sh[BLOCK / WAVE];
    const double pq = sum_partials(pp + pp_offset(PP_PQ), nb_pq, sh);
    const double alpha = pp[rho_slot] / pq;
    double acc = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)BLOCK + threadIdx.x; i < n; i += (int64_t)gridDim.x * BLOCK) {
        x[i] += alpha * p[i];
        if (r_old) r_old[i] = r[i];
        const double ri = r[i] - alpha * q[i];
        r[i] = ri;
        acc += ri * ri;
    }
    acc = block_sum(acc, sh);
    if (threadIdx.x == 0) {
        pp[pp_offset(PP_RR) + blockIdx.x] = acc;
        if (blockIdx.x == 0) {
            pp[S_PQ] = pq;
            pp[S_ALPHA] = alpha;
        }
    }
}

// z1 = a - b over the first n1 entries (z2 already in place); block
// partials of r.z (PP_RZ) and, with flexible CG, of r_old.z (PP_ZRO).
__global__ __launch_bounds__(BLOCK) void k_combine_dot(int64_t n1, int64_t n, double* __restrict__ z,
                                                       const double* __restrict__ a,
                                                       const double* __restrict__ b,
                                                       const double* __restrict__ r,
                                                       const double* __restrict__ r_old,
                                                       double* __restrict__ pp) {
    __shared__ double sh[BLOCK / WAVE];
    double acc = 0.0, acc2 = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)BLOCK + threadIdx.x; i < n; i += (int64_t)gridDim.x * BLOCK) {
        double zi;
        if (i < n1) {
            zi = a[i] - b[i];
            z[i] = zi;
        } else {
            zi = z[i];
        }
        acc += r[i] * zi;
        if (r_old) acc2 += r_old[i] * zi;
    }
    acc = block_sum(acc, sh);
    if (r_old) acc2 = block_sum(acc2, sh);
    if (threadIdx.x == 0) {
        pp[pp_offset(PP_RZ) + blockIdx.x] = acc;
        if (r_old) pp[pp_offset(PP_ZRO) + blockIdx.x] = acc2;
    }
}

// rho_new = r.z (summed from nb partials); beta = rho_new / rho_old, or the
// flexible (Polak-Ribiere) (r.z - r_old.z) / rho_old; p = z + beta p.  Block
// 0 stores rho_new in slot rho_new_slot (never the slot read here).
__global__ __launch_bounds__(BLOCK) void k_p_update(int64_t n, const double* __restrict__ z, double* __restrict__ p,
                                                    double* __restrict__ pp, int nb, int first, int flexible,
                                                    int rho_old_slot, int rho_new_slot) {
    __shared__ double sh[BLOCK / WAVE];
    const double rz = sum_partials(pp + pp_offset(PP_RZ), nb, sh);
    double beta = 0.0;
    if (!first) {
        const double zro = flexible ? sum_partials(pp + pp_offset(PP_ZRO), nb, sh) : 0.0;
        beta = (rz - zro) / pp[rho_old_slot];
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) pp[rho_new_slot] = rz;
    // the first direction is z itself: p may hold stale bits (0 * NaN = NaN)
    for (int64_t i = blockIdx.x * (int64_t)BLOCK + threadIdx.x; i < n; i += (int64_t)gridDim.x * BLOCK)
        p[i] = first ? z[i] : z[i] + beta * p[i];
}

// ---------------------------------------------------------------------------
// Hierarchical-Cholesky sweeps
//
// Node t owns the panel P_t = [L_tt^-1 ; L_Bt L_tt^-1].  Forward: w_t = b_t -
// (children's updates at I_t), [y_t ; c_t] = P_t w_t, c_t also collects the
// children's updates at B(t).  Backward: x_t = P_t^T [y_t ; -x_B].
// Forward threads own rows and read the column-major copy; backward threads
// own columns and read the row-major copy (see TriNode).
// ---------------------------------------------------------------------------
constexpr int SUB_BLOCK = 1024;    // subtree phase: 16 waves per workgroup
constexpr int SUB_NW = SUB_BLOCK / WAVE;
constexpr int SUB_MAXW = 256;      // max own size of a node below the cut
constexpr int SUB_MAXF = 384;      // max panel rows of a node below the cut
constexpr int FWD_ROWS = 64;       // forward row tile of the level phase

__device__ __forceinline__ int64_t panel_row_off(int64_t r, int64_t nI) {
    return r < nI ? r * (r + 1) / 2 : nI * (nI + 1) / 2 + (r - nI) * nI;
}
__device__ __forceinline__ int64_t panel_col_off(int64_t c, int64_t nI, int64_t nB) {
    return c * (nI + nB) - c * (c - 1) / 2;
}

__device__ __forceinline__ int pow2_ceil64(int n) {
    int g = 1;
    while (g < n && g < 64) g <<= 1;
    return g;
}

// Staging steps issue every load before using any: entry 0 of the update
// workspace is always 0.0 (no node's update vector starts there) and stands in
// for a missing child update, the boundary index array ends with a spare
// entry, lanes past the end of a range reread its last entry, and their
// results go to a spare LDS slot.  A staging step then costs two memory
// latencies (indices, then values) instead of two per element.

// w[i - ibase] = b[off+i] - children's updates at own position i (ground ->
// 0), for i = i0 + t + stride k < i1 (k < K)
template <int K>
__device__ __forceinline__ void stage_w(const TriNode& nd, int t, int stride, int i0, int i1, int ibase,
                                        const Ea* __restrict__ ea, const double* __restrict__ b,
                                        const double* upd, int64_t u0, int64_t u1, double* w, int spare) {
    if (i1 <= i0) return;
    Ea m[K];
#pragma unroll
    for (int k = 0; k < K; ++k) m[k] = ea[nd.ea + min(i0 + t + stride * k, i1 - 1)];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int i = i0 + t + stride * k, ic = min(i, i1 - 1);
        const double v = b[nd.off + ic] - upd[m[k].a >= 0 ? u0 + m[k].a : 0] - upd[m[k].b >= 0 ? u1 + m[k].b : 0];
        w[i < i1 ? i - ibase : spare] = v * (ic == nd.gi ? 0.0 : 1.0);
    }
}

// z[r - zbase] = y_t[r] (own rows) or -x[B(t)[r - nI]] (boundary rows), for
// r = r0 + t + stride k < r1 (k < K)
template <int K>
__device__ __forceinline__ void stage_z(const TriNode& nd, int t, int stride, int r0, int r1, int zbase,
                                        const int64_t* __restrict__ bidx, const double* __restrict__ y,
                                        const double* x, double* z, int spare) {
    if (r1 <= r0) return;
    const int nI = nd.nI;
    int64_t xi[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int rc = min(r0 + t + stride * k, r1 - 1);
        xi[k] = bidx[nd.bidx + (rc >= nI ? rc - nI : 0)];
    }
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int r = r0 + t + stride * k, rc = min(r, r1 - 1);
        const double v = *(rc < nI ? y + nd.off + rc : x + xi[k]);
        z[r < r1 ? r - zbase : spare] = rc < nI ? v : -v;
    }
}

// the children's updates at row r of P_t w_t (0.0 for own rows), loaded
// ahead of the row's products
__device__ __forceinline__ double row_add(const TriNode& nd, int r, const Ea* __restrict__ ea, const double* upd,
                                          int64_t u0, int64_t u1) {
    const Ea m = ea[nd.ea + r];
    const bool bnd = r >= nd.nI;
    return upd[bnd && m.a >= 0 ? u0 + m.a : 0] + upd[bnd && m.b >= 0 ? u1 + m.b : 0];
}

// store row r of P_t w_t (its additions included): own rows to y, boundary
// rows to the update vector of the node
__device__ __forceinline__ void store_row(const TriNode& nd, int r, double s, double* __restrict__ y, double* upd) {
    if (r < nd.nI) y[nd.off + r] = s;
    else upd[nd.upd + (r - nd.nI)] = s;
}

// Independent loads in flight per lane in the sweeps' inner loops.
constexpr int SWEEP_ILP = 8;
__device__ __forceinline__ double sum_ilp(const double (&a)[SWEEP_ILP]) {
    double s[SWEEP_ILP / 2];
#pragma unroll
    for (int k = 0; k < SWEEP_ILP / 2; ++k) s[k] = a[2 * k] + a[2 * k + 1];
#pragma unroll
    for (int w = SWEEP_ILP / 4; w >= 1; w >>= 1)
#pragma unroll
        for (int k = 0; k < w; ++k) s[k] = s[2 * k] + s[2 * k + 1];
    return s[0];
}

// sum_{c in [cs, ce), c <= r if r < nI} P(r, c) w[c - cs]   (column-major copy).
// Entry (r, c) sits at col_off(c) + r - c; moving to column c+1 adds
// nI + nB - c - 1.  SWEEP_ILP independent accumulators keep that many loads
// in flight.
template <typename T>
__device__ __forceinline__ double row_part(const T* __restrict__ Pc, int nI, int nB, int r, int cs,
                                           int ce, const double* w) {
    const int cend = r < nI ? min(ce, r + 1) : ce;
    const int nF = nI + nB;
    int64_t off = panel_col_off(cs, nI, nB) + (r - cs);
    double a[SWEEP_ILP];
#pragma unroll
    for (int k = 0; k < SWEEP_ILP; ++k) a[k] = 0.0;
    int c = cs;
    for (; c + SWEEP_ILP <= cend; c += SWEEP_ILP) {
#pragma unroll
        for (int k = 0; k < SWEEP_ILP; ++k) {
            a[k] += (double)Pc[off] * w[c + k - cs];
            off += nF - (c + k) - 1;
        }
    }
    // remainder (< SWEEP_ILP columns): every lane issues all its loads at
    // once (a finished lane reads the panel's first entry and drops it), so
    // the tail costs one memory latency instead of one per column
    int64_t offs[SWEEP_ILP - 1];
#pragma unroll
    for (int k = 0; k < SWEEP_ILP - 1; ++k) {
        offs[k] = off;
        off += nF - (c + k) - 1;
    }
#pragma unroll
    for (int k = 0; k < SWEEP_ILP - 1; ++k) {
        const bool ok = c + k < cend;
        const double v = (double)Pc[ok ? offs[k] : 0] * w[ok ? c + k - cs : 0];
        a[k] += v * (ok ? 1.0 : 0.0);      // (a select would let the load sink into a branch)
    }
    return sum_ilp(a);
}

// Offset of row r in a packed row-major panel, in 32-bit arithmetic (a
// single node's panel stays far below 2^31 entries).
__device__ __forceinline__ int row_off32(int r, int nI) {
    return r < nI ? (r * (r + 1)) >> 1 : ((nI * (nI + 1)) >> 1) + (r - nI) * nI;
}

// sum over rows r = r0, r0+S, ... < re of P(r, c) z[r - z0] (row-major copy),
// skipping the unstored entries c > r of the triangle.  All lanes of a wave
// walk the same rows, so each row is read as one contiguous segment.  S is a
// power of two (2^lgS); row offsets advance by additions only: in the
// triangle off(r+S) = off(r) + S r + S(S+1)/2, below it off(r+S) = off(r) + S nI.
template <typename T>
__device__ __forceinline__ double col_part(const T* __restrict__ P, int nI, int c, int r0, int re, int S,
                                           const double* z, int z0) {
    const int lgS = __ffs(S) - 1;
    const int SS = (S * (S + 1)) >> 1;
    double a[SWEEP_ILP];
#pragma unroll
    for (int k = 0; k < SWEEP_ILP; ++k) a[k] = 0.0;
    int r = r0;
    int off = row_off32(r, nI);
    const int te = min(re, nI);
    // triangle: the loads are unconditional (entry (rr, c > rr) is not
    // stored, but off + c still lies inside the triangle) and the unstored
    // products are dropped, so all SWEEP_ILP loads are in flight together
    for (; r + (SWEEP_ILP - 1) * S < te; r += SWEEP_ILP * S) {
#pragma unroll
        for (int q = 0; q < SWEEP_ILP; ++q) {
            const int rr = r + q * S;
            const double v = (double)P[off + c] * z[rr - z0];
            a[q] += c <= rr ? v : 0.0;
            off = rr + S <= nI ? off + (rr << lgS) + SS : row_off32(rr + S, nI);
        }
    }
    // triangle tail: rows past te read the panel's first entry, dropped
    int offs[SWEEP_ILP - 1];
#pragma unroll
    for (int q = 0; q < SWEEP_ILP - 1; ++q) {
        const int rr = r + q * S;
        offs[q] = off;
        const int nxt = rr + S <= nI ? off + (rr << lgS) + SS : row_off32(rr + S, nI);
        off = rr < te ? nxt : off;
    }
#pragma unroll
    for (int q = 0; q < SWEEP_ILP - 1; ++q) {
        const int rr = r + q * S;
        const bool ok = rr < te;
        const double v = (double)P[ok ? offs[q] + c : 0] * z[ok ? rr - z0 : 0];
        a[q] += v * (ok && c <= rr ? 1.0 : 0.0);
    }
    if (r < te) r += ((te - r + S - 1) >> lgS) << lgS;   // first row of the sequence at or past te
    const int step = S * nI;
    for (; r + (SWEEP_ILP - 1) * S < re; r += SWEEP_ILP * S) {
#pragma unroll
        for (int q = 0; q < SWEEP_ILP; ++q) a[q] += (double)P[off + q * step + c] * z[r + q * S - z0];
        off += SWEEP_ILP * step;
    }
#pragma unroll
    for (int q = 0; q < SWEEP_ILP - 1; ++q) {
        const bool ok = r + q * S < re;
        const double v = (double)P[ok ? off + q * step + c : 0] * z[ok ? r + q * S - z0 : 0];
        a[q] += v * (ok ? 1.0 : 0.0);
    }
    return sum_ilp(a);
}

// Subtree phases: workgroup s walks its subtree one height at a time, each
// wave taking whole nodes.  In the forward phase a height with 8 or fewer
// nodes (the upper ones of a subtree) gives every node a group of
// g = 16 / (nodes) waves (rounded down to a power of two) that split its
// rows.  (The backward phase stays one wave per node: its upper nodes are
// thin, a few columns over many rows that the row streams of one wave
// already cover, and a group's reductions cost more than they save.)

// waves per node at a height with n < SUB_NW nodes
__device__ __forceinline__ int sub_group(int n) {
    int g = SUB_NW;
    while (g * n > SUB_NW) g >>= 1;
    return g;
}

// The node records and index maps a wave needs at a height do not depend on
// the heights before it, so they are loaded before the barrier that ends the
// previous height; after it only the values that do (x of the ancestors,
// the children's updates) remain to be fetched.
constexpr int SUB_KW = SUB_MAXW / WAVE;   // columns of w per lane (one wave per node)
constexpr int SUB_KF = SUB_MAXF / WAVE;   // rows of z per lane

// this wave's share of height h of a subtree: its first node k (-1: none),
// the group size g and the thread's index t within the group
struct SubSlot {
    int k, g, t;
};
__device__ __forceinline__ SubSlot fwd_slot(const int32_t* hoff, int h, int wave, int lane) {
    const int k0 = hoff[h], n = hoff[h + 1] - k0;
    SubSlot sl;
    if (n > SUB_NW / 2) {
        sl.g = 1;
        sl.t = lane;
        sl.k = wave < n ? k0 + wave : -1;
    } else {
        sl.g = n > 0 ? sub_group(n) : 1;
        const int grp = wave / sl.g;
        sl.t = (wave % sl.g) * WAVE + lane;
        sl.k = grp < n ? k0 + grp : -1;
    }
    return sl;
}

struct FwdPre {
    TriNode nd;
    Ea mw[SUB_KW];   // maps of the thread's columns of w (stride g * WAVE)
    Ea mr;           // map of the thread's first row
};
__device__ __forceinline__ void fwd_load(const TriNode* __restrict__ sub_tn, const Ea* __restrict__ ea, int k,
                                         int t, int stride, FwdPre& p) {
    p.nd = sub_tn[__builtin_amdgcn_readfirstlane(k)];
    const int nI = p.nd.nI, nF = nI + p.nd.nB;
#pragma unroll
    for (int q = 0; q < SUB_KW; ++q) p.mw[q] = ea[p.nd.ea + max(0, min(t + stride * q, nI - 1))];
    p.mr = ea[p.nd.ea + max(0, min(t, nF - 1))];
}
// w from prefetched maps: w[i] = b[off+i] - children's updates (ground -> 0)
__device__ __forceinline__ void stage_w_pre(const FwdPre& p, int t, int stride, int kmax,
                                            const double* __restrict__ b, const double* upd, double* w) {
    const TriNode& nd = p.nd;
    if (nd.nI <= 0) return;
#pragma unroll
    for (int q = 0; q < SUB_KW; ++q) {
        if (q >= kmax) break;
        const int i = t + stride * q, ic = min(i, nd.nI - 1);
        const double v = b[nd.off + ic] - upd[p.mw[q].a >= 0 ? nd.u0 + p.mw[q].a : 0] -
                         upd[p.mw[q].b >= 0 ? nd.u1 + p.mw[q].b : 0];
        w[i < nd.nI ? i : SUB_MAXW] = v * (ic == nd.gi ? 0.0 : 1.0);
    }
}

struct BwdPre {
    TriNode nd;
    int64_t xi[SUB_KF];   // boundary indices of the lane's rows
};
__device__ __forceinline__ void bwd_load(const TriNode* __restrict__ sub_tn, const int64_t* __restrict__ bidx, int k,
                                         int lane, BwdPre& p) {
    p.nd = sub_tn[__builtin_amdgcn_readfirstlane(k)];
    const int nI = p.nd.nI, nF = nI + p.nd.nB;
#pragma unroll
    for (int q = 0; q < SUB_KF; ++q) {
        const int rc = max(0, min(lane + WAVE * q, nF - 1));
        p.xi[q] = bidx[p.nd.bidx + (rc >= nI ? rc - nI : 0)];
    }
}
// z = [y_t ; -x_B] from prefetched indices
__device__ __forceinline__ void stage_z_pre(const BwdPre& p, int lane, const double* __restrict__ y,
                                            const double* x, double* z) {
    const TriNode& nd = p.nd;
    const int nI = nd.nI, nF = nI + nd.nB;
    if (nF <= 0) return;
#pragma unroll
    for (int q = 0; q < SUB_KF; ++q) {
        const int r = lane + WAVE * q, rc = min(r, nF - 1);
        const double v = *(rc < nI ? y + nd.off + rc : x + p.xi[q]);
        z[r < nF ? r : SUB_MAXF] = rc < nI ? v : -v;
    }
}

// Forward: [y_t ; c_t] = P_t w_t, one panel row per thread of the node's
// waves (rows need no reduction).
template <typename T>
__global__ __launch_bounds__(SUB_BLOCK) void k_tri_fwd_sub(const TriNode* __restrict__ sub_tn,
                                                           const int32_t* __restrict__ sub_hoff, int hc,
                                                           const T* __restrict__ panel_cm,
                                                           const Ea* __restrict__ ea,
                                                           const double* __restrict__ b,
                                                           double* __restrict__ y,
                                                           double* upd, const uint8_t* __restrict__ skip) {
    __shared__ double wbuf[SUB_NW][SUB_MAXW + 1];
    const int lane = threadIdx.x % WAVE, wave = threadIdx.x / WAVE;
    const int32_t* hoff = sub_hoff + (size_t)blockIdx.x * (hc + 2);
    if (skip && skip[sub_tn[hoff[0]].tree]) return;   // a frozen slice of a batch
    FwdPre pre;
    SubSlot sl = fwd_slot(hoff, 0, wave, lane);
    if (sl.k >= 0) fwd_load(sub_tn, ea, sl.k, sl.t, sl.g * WAVE, pre);
    for (int h = 0; h <= hc; ++h) {
        const int k0 = hoff[h], k1 = hoff[h + 1], n = k1 - k0;
        const int stride = sl.g * WAVE;
        const int kmax = (SUB_MAXW + stride - 1) / stride;
        if (n > SUB_NW / 2) {
            double* w = wbuf[wave];
            for (int k = k0 + wave; k < k1; k += SUB_NW) {
                if (k != sl.k) fwd_load(sub_tn, ea, k, lane, WAVE, pre);
                const TriNode& nd = pre.nd;
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
                __builtin_amdgcn_wave_barrier();
                stage_w_pre(pre, lane, WAVE, SUB_KW, b, upd, w);
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
                const T* Pc = panel_cm + nd.panel;
                const int nF = nd.nI + nd.nB;
                for (int r = lane; r < nF; r += WAVE) {
                    const Ea m = r == lane ? pre.mr : ea[nd.ea + r];
                    const bool bnd = r >= nd.nI;
                    const double add = upd[bnd && m.a >= 0 ? nd.u0 + m.a : 0] + upd[bnd && m.b >= 0 ? nd.u1 + m.b : 0];
                    const double s = row_part<T>(Pc, nd.nI, nd.nB, r, 0, nd.nI, w);
                    store_row(nd, r, s + add, y, upd);
                }
            }
        } else if (sl.k >= 0) {
            const int grp = wave / sl.g;
            double* w = wbuf[grp * sl.g];
            stage_w_pre(pre, sl.t, stride, kmax, b, upd, w);
        }
        if (n > 0 && n <= SUB_NW / 2) __syncthreads();   // the group's w is staged
        if (n > 0 && n <= SUB_NW / 2 && sl.k >= 0) {
            const TriNode& nd = pre.nd;
            const double* w = wbuf[(wave / sl.g) * sl.g];
            const T* Pc = panel_cm + nd.panel;
            const int nF = nd.nI + nd.nB;
            for (int r = sl.t; r < nF; r += stride) {
                const Ea m = r == sl.t ? pre.mr : ea[nd.ea + r];
                const bool bnd = r >= nd.nI;
                const double add = upd[bnd && m.a >= 0 ? nd.u0 + m.a : 0] + upd[bnd && m.b >= 0 ? nd.u1 + m.b : 0];
                const double s = row_part<T>(Pc, nd.nI, nd.nB, r, 0, nd.nI, w);
                store_row(nd, r, s + add, y, upd);
            }
        }
        // records and maps of the next height, ahead of the barrier
        if (h < hc) {
            sl = fwd_slot(hoff, h + 1, wave, lane);
            if (sl.k >= 0) fwd_load(sub_tn, ea, sl.k, sl.t, sl.g * WAVE, pre);
        }
        __syncthreads();
    }
}

// Backward: x_t = P_t^T [y_t ; -x_B], z staged in LDS.  Lanes own columns
// (blocks of up to 64); a block of W < 64 columns splits the rows into
// 64 / W streams, summed across the wave.
template <typename T>
__global__ __launch_bounds__(SUB_BLOCK) void k_tri_bwd_sub(const TriNode* __restrict__ sub_tn,
                                                           const int32_t* __restrict__ sub_hoff, int hc,
                                                           const T* __restrict__ panel,
                                                           const int64_t* __restrict__ bidx,
                                                           const double* __restrict__ y,
                                                           double* x, int group_max,
                                                           const uint8_t* __restrict__ skip) {
    __shared__ double zbuf[SUB_NW][SUB_MAXF + 1];
    __shared__ double red[SUB_NW][WAVE];
    const int lane = threadIdx.x % WAVE, wave = threadIdx.x / WAVE;
    const int32_t* hoff = sub_hoff + (size_t)blockIdx.x * (hc + 2);
    if (skip && skip[sub_tn[hoff[0]].tree]) return;   // a frozen slice of a batch
    double* z = zbuf[wave];
    BwdPre pre;
    int kp = hoff[hc] + wave;
    if (kp < hoff[hc + 1]) bwd_load(sub_tn, bidx, kp, lane, pre);
    for (int h = hc; h >= 0; --h) {
        const int k0 = hoff[h], k1 = hoff[h + 1], n = k1 - k0;
        if (n > 0 && n <= group_max) {
            // g waves per node: row streams spread over the group, partial
            // column sums reduced across the wave, then across the group
            const int g = sub_group(n), grp = wave / g, wg = wave % g;
            const bool active = grp < n;
            const int lead = grp * g < SUB_NW ? grp * g : 0;
            double* zg = zbuf[lead];
            TriNode nd{};
            if (active) {
                nd = sub_tn[__builtin_amdgcn_readfirstlane(k0 + grp)];
                const int t = wg * WAVE + lane, nF = nd.nI + nd.nB;
                if (g == 2) stage_z<SUB_MAXF / (2 * WAVE)>(nd, t, 2 * WAVE, 0, nF, 0, bidx, y, x, zg, SUB_MAXF);
                else if (g == 4) stage_z<(SUB_MAXF + 4 * WAVE - 1) / (4 * WAVE)>(nd, t, 4 * WAVE, 0, nF, 0, bidx, y, x,
                                                                                  zg, SUB_MAXF);
                else stage_z<(SUB_MAXF + 8 * WAVE - 1) / (8 * WAVE)>(nd, t, g * WAVE, 0, nF, 0, bidx, y, x, zg,
                                                                      SUB_MAXF);
            }
            int ncb = 0;
            for (int k = k0; k < k1; ++k) ncb = max(ncb, (sub_tn[k].nI + WAVE - 1) / WAVE);
            __syncthreads();
            const int nI = nd.nI, nF = nd.nI + nd.nB;
            const T* P = panel + nd.panel;
            for (int cb = 0; cb < ncb * WAVE; cb += WAVE) {
                const bool on = active && cb < nI;
                const int ncols = on ? min(WAVE, nI - cb) : 1;
                const int W = pow2_ceil64(ncols);
                const int Sw = WAVE / W, S = g * Sw;
                const int col = lane % W, st = wg * Sw + lane / W;
                double acc = 0.0;
                if (on && col < ncols) acc = col_part<T>(P, nI, cb + col, cb + st, nF, S, zg, 0);
                for (int m = W; m < WAVE; m <<= 1) acc += __shfl_xor(acc, m, WAVE);
                if (lane < W) red[wave][lane] = acc;
                __syncthreads();
                if (on && wg == 0 && lane < ncols) {
                    double sum = 0.0;
                    for (int q = 0; q < g; ++q) sum += red[lead + q][lane];
                    x[nd.off + cb + lane] = sum;
                }
                __syncthreads();
            }
            if (h > 0) {
                kp = hoff[h - 1] + wave;
                if (kp < hoff[h]) bwd_load(sub_tn, bidx, kp, lane, pre);
            }
            __syncthreads();
            continue;
        }
        for (int k = k0 + wave; k < k1; k += SUB_NW) {
            if (k != kp) bwd_load(sub_tn, bidx, k, lane, pre);
            const TriNode& nd = pre.nd;
            const int nI = nd.nI, nF = nd.nI + nd.nB;
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
            __builtin_amdgcn_wave_barrier();
            stage_z_pre(pre, lane, y, x, z);
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
            const T* P = panel + nd.panel;
            for (int cb = 0; cb < nI; cb += WAVE) {
                const int ncols = min(WAVE, nI - cb);
                const int W = pow2_ceil64(ncols);
                const int S = WAVE / W;
                const int col = lane % W, st = lane / W;
                const int c = cb + col;
                double acc = 0.0;
                if (col < ncols) acc = col_part<T>(P, nI, c, cb + st, nF, S, z, 0);
                for (int m = W; m < WAVE; m <<= 1) acc += __shfl_xor(acc, m, WAVE);
                if (st == 0 && col < ncols) x[nd.off + c] = acc;
            }
        }
        // record and boundary indices of the next height, ahead of the barrier
        if (h > 0) {
            kp = hoff[h - 1] + wave;
            if (kp < hoff[h]) bwd_load(sub_tn, bidx, kp, lane, pre);
        }
        __syncthreads();
    }
}

// Level phase, forward: item = (64-row tile, column chunk) of one node.  The
// four waves split the chunk's columns.  A tile split over several chunks
// leaves its partial sums in scratch for the combine launch of the level.
template <typename T>
__global__ __launch_bounds__(BLOCK) void k_tri_fwd_lvl(const TriNode* __restrict__ nodes,
                                                       const TriItem* __restrict__ items,
                                                       const T* __restrict__ panel_cm,
                                                       const Ea* __restrict__ ea,
                                                       const double* __restrict__ b,
                                                       double* __restrict__ y,
                                                       double* upd, double* __restrict__ scratch, int spare,
                                                       const uint8_t* __restrict__ skip) {
    extern __shared__ double w[];   // the item's columns, then the spare slot
    __shared__ double red[BLOCK / WAVE][FWD_ROWS];
    const TriItem it = items[blockIdx.x];
    const TriNode nd = nodes[it.node];
    if (skip && skip[nd.tree]) return;
    const int64_t u0 = nd.u0, u1 = nd.u1;
    const int ncol = it.ce - it.cs;
    for (int i0 = it.cs; i0 < it.ce; i0 += 2 * BLOCK)
        stage_w<2>(nd, threadIdx.x, BLOCK, i0, it.ce, it.cs, ea, b, upd, u0, u1, w, spare);
    const int lane = threadIdx.x % WAVE, wave = threadIdx.x / WAVE;
    const int r = it.r0 + lane;
    const double add = wave == 0 && it.nparts == 1 && lane < it.nrows ? row_add(nd, r, ea, upd, u0, u1) : 0.0;
    __syncthreads();
    const int nw = BLOCK / WAVE;
    const int per = (ncol + nw - 1) / nw;
    const int c0 = it.cs + wave * per, c1 = min(it.ce, c0 + per);
    double s = 0.0;
    if (lane < it.nrows && c0 < c1)
        s = row_part<T>(panel_cm + nd.panel, nd.nI, nd.nB, r, c0, c1, w + (c0 - it.cs));
    red[wave][lane] = s;
    __syncthreads();
    if (wave != 0) return;
    double tot = 0.0;
    for (int k = 0; k < nw; ++k) tot += red[k][lane];
    if (it.nparts == 1) {
        if (lane < it.nrows) store_row(nd, r, tot + add, y, upd);
    } else {
        scratch[it.part + lane] = tot;
    }
}

// Combine launch of a forward level: one wave per split tile sums the parts
// in order (deterministic) and finishes its rows.
__global__ __launch_bounds__(BLOCK) void k_tri_fwd_comb(const TriNode* __restrict__ nodes,
                                                        const TriItem* __restrict__ comb, int ncomb,
                                                        const Ea* __restrict__ ea, double* __restrict__ y,
                                                        double* upd, const double* __restrict__ scratch,
                                                        const uint8_t* __restrict__ skip) {
    const int lane = threadIdx.x % WAVE, wave = threadIdx.x / WAVE;
    const int q = blockIdx.x * (BLOCK / WAVE) + wave;
    if (q >= ncomb) return;
    const TriItem it = comb[q];
    if (lane >= it.nrows) return;
    const TriNode nd = nodes[it.node];
    if (skip && skip[nd.tree]) return;
    const double add = row_add(nd, it.r0 + lane, ea, upd, nd.u0, nd.u1);
    double t = 0.0;
    for (int k = 0; k < it.nparts; ++k) t += scratch[it.part0 + (int64_t)k * FWD_ROWS + lane];
    store_row(nd, it.r0 + lane, t + add, y, upd);
}

// Level phase, backward: item = (column tile, row range) of one node; z for
// the row range is staged in LDS first.  A tile split over several row
// ranges leaves its partial sums in scratch for the combine launch.
template <typename T, int NT>
__global__ __launch_bounds__(NT) void k_tri_bwd_lvl(const TriNode* __restrict__ nodes,
                                                    const BwdItem* __restrict__ items,
                                                    const T* __restrict__ panel,
                                                    const int64_t* __restrict__ bidx,
                                                    const double* __restrict__ y,
                                                    double* x, double* __restrict__ scratch, int spare,
                                                    const uint8_t* __restrict__ skip) {
    extern __shared__ double z[];   // the item's rows, then the spare slot
    __shared__ double red[NT];
    const BwdItem it = items[blockIdx.x];
    const TriNode nd = nodes[it.node];
    if (skip && skip[nd.tree]) return;
    const int nI = nd.nI;
    for (int r0 = it.rs; r0 < it.re; r0 += 2 * NT)
        stage_z<2>(nd, threadIdx.x, NT, r0, it.re, it.rs, bidx, y, x, z, spare);
    __syncthreads();
    const int W = it.W;
    const int col = threadIdx.x % W, st = threadIdx.x / W;
    const int S = NT / W;
    const int c = it.c0 + col;
    const T* P = panel + nd.panel;
    double acc = 0.0;
    if (col < it.ncols) acc = col_part<T>(P, nI, c, max(it.rs, it.c0) + st, it.re, S, z, it.rs);
    red[threadIdx.x] = acc;
    __syncthreads();
    if (threadIdx.x >= W) return;
    double s = 0.0;
    for (int k = 0; k < S; ++k) s += red[k * W + threadIdx.x];
    if (it.nparts == 1) {
        if (threadIdx.x < it.ncols) x[nd.off + c] = s;
    } else {
        scratch[it.part + threadIdx.x] = s;
    }
}

// Combine launch of a backward level: one wave per split column tile.
__global__ __launch_bounds__(WAVE) void k_tri_bwd_comb(const TriNode* __restrict__ nodes,
                                                       const BwdItem* __restrict__ comb,
                                                       double* __restrict__ x, const double* __restrict__ scratch,
                                                       const uint8_t* __restrict__ skip) {
    const BwdItem it = comb[blockIdx.x];
    const int col = threadIdx.x;
    if (col >= it.ncols) return;
    const TriNode nd = nodes[it.node];
    if (skip && skip[nd.tree]) return;
    double t = 0.0;
    for (int k = 0; k < it.nparts; ++k) t += scratch[it.part0 + (int64_t)k * it.W + col];
    x[nd.off + it.c0 + col] = t;
}

// Dense top: w_top[k] = b[pos[k]] - sum of the bottom roots' updates at k.
__global__ void k_top_gather(int64_t n, const int64_t* __restrict__ pos, const int32_t* __restrict__ gptr,
                             const int64_t* __restrict__ gsrc, const double* __restrict__ b,
                             const double* __restrict__ upd, const uint8_t* __restrict__ zero,
                             double* __restrict__ w) {
    const int64_t k = blockIdx.x * (int64_t)BLOCK + threadIdx.x;
    if (k >= n) return;
    const int64_t g = pos[k];
    double v = b[g];
    for (int32_t q = gptr[k]; q < gptr[k + 1]; ++q) v -= upd[gsrc[q]];
    w[k] = zero[k] ? 0.0 : v;
}

// x[pos[i]] = sum_j inv[i][j] w[j]: one wave per row, w staged in LDS,
// eight independent loads in flight per lane.
constexpr int TOP_ROWS = BLOCK / WAVE;
template <typename T>
__global__ __launch_bounds__(BLOCK) void k_top_gemv(int64_t n, const T* __restrict__ inv,
                                                    const double* __restrict__ w,
                                                    const int64_t* __restrict__ pos, double* __restrict__ x) {
    extern __shared__ double ws[];
    for (int64_t j = threadIdx.x; j < n; j += BLOCK) ws[j] = w[j];
    __syncthreads();
    const int lane = threadIdx.x % WAVE, wave = threadIdx.x / WAVE;
    const int64_t row = blockIdx.x * (int64_t)TOP_ROWS + wave;
    if (row >= n) return;
    const T* a = inv + row * n;
    double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    int64_t j = lane;
    for (; j + 7 * WAVE < n; j += 8 * WAVE) {
#pragma unroll
        for (int k = 0; k < 8; ++k) acc[k] += (double)a[j + k * WAVE] * ws[j + k * WAVE];
    }
    for (int k = 0; j < n; j += WAVE, ++k) acc[k] += (double)a[j] * ws[j];
    double s = ((acc[0] + acc[1]) + (acc[2] + acc[3])) + ((acc[4] + acc[5]) + (acc[6] + acc[7]));
    for (int m = WAVE / 2; m > 0; m >>= 1) s += __shfl_xor(s, m, WAVE);
    if (lane == 0) x[pos[row]] = s;
}

// Hierarchical top, projections: one wave per column of every block,
// t[b.t + j] = V[:, j]^T w[m:e) (j < k) or U[:, j-k]^T w[a:m).
template <typename T>
__global__ __launch_bounds__(BLOCK) void k_hodlr_proj(const HodlrBlock* __restrict__ blocks,
                                                      const int32_t* __restrict__ cols, int ncols,
                                                      const T* __restrict__ val, const double* __restrict__ w,
                                                      double* __restrict__ t) {
    const int lane = threadIdx.x % WAVE, wave = threadIdx.x / WAVE;
    const int q = blockIdx.x * (BLOCK / WAVE) + wave;
    if (q >= ncols) return;
    const int code = cols[q];
    const HodlrBlock b = blocks[code >> 16];
    const int j = code & 0xffff;
    const bool first = j < b.k;
    const int len = first ? b.e - b.m : b.m - b.a;
    const T* col = val + (first ? b.v : b.u) + (int64_t)(first ? j : j - b.k) * len;
    const double* ws = w + (first ? b.m : b.a);
    double a[4] = {0, 0, 0, 0};
    int r = lane;
    for (; r + 3 * WAVE < len; r += 4 * WAVE) {
#pragma unroll
        for (int u = 0; u < 4; ++u) a[u] += (double)col[r + u * WAVE] * ws[r + u * WAVE];
    }
    for (; r < len; r += WAVE) a[0] += (double)col[r] * ws[r];
    double s = wave_sum((a[0] + a[1]) + (a[2] + a[3]));
    if (lane == 0) t[b.t + j] = s;
}

// Hierarchical top, rows of one leaf (<= 64), one lane per row: the terms
// (the dense diagonal block, then the leaf's ancestor blocks) are cut into
// chunks of 16 columns dealt round-robin to the 16 waves of the workgroup;
// x[pos[row]] = sum of the chunks (reduced in LDS, fixed order).
constexpr int HODLR_LEAF = 64;
constexpr int HODLR_BLOCK = 1024;
constexpr int HODLR_NW = HODLR_BLOCK / WAVE;
constexpr int HODLR_CHUNK = 16;
template <typename T>
__global__ __launch_bounds__(HODLR_BLOCK) void k_hodlr_apply(const HodlrLeaf* __restrict__ leaves,
                                                             const HodlrBlock* __restrict__ blocks,
                                                             const int32_t* __restrict__ anc,
                                                             const T* __restrict__ val,
                                                             const double* __restrict__ w,
                                                             const double* __restrict__ t,
                                                             const int64_t* __restrict__ pos,
                                                             double* __restrict__ x) {
    __shared__ double ws[HODLR_LEAF];
    __shared__ double part[HODLR_NW][HODLR_LEAF];
    const HodlrLeaf lf = leaves[blockIdx.x];
    const int len = lf.e - lf.a;
    const int lane = threadIdx.x % WAVE, wave = threadIdx.x / WAVE;
    if (threadIdx.x < len) ws[threadIdx.x] = w[lf.a + threadIdx.x];
    __syncthreads();
    double a[4] = {0, 0, 0, 0};
    if (lane < len) {
        int u = 0;
        for (int j0 = 0; j0 < len; j0 += HODLR_CHUNK, ++u) {
            if (u % HODLR_NW != wave) continue;
            const T* D = val + lf.d + lane;
            const int j1 = min(len, j0 + HODLR_CHUNK);
            int j = j0;
            for (; j + 3 < j1; j += 4) {
                a[0] += (double)D[(int64_t)j * len] * ws[j];
                a[1] += (double)D[(int64_t)(j + 1) * len] * ws[j + 1];
                a[2] += (double)D[(int64_t)(j + 2) * len] * ws[j + 2];
                a[3] += (double)D[(int64_t)(j + 3) * len] * ws[j + 3];
            }
            for (; j < j1; ++j) a[0] += (double)D[(int64_t)j * len] * ws[j];
        }
        for (int q = 0; q < lf.nanc; ++q) {
            const int code = anc[lf.anc + q];
            const HodlrBlock b = blocks[code >> 1];
            const bool upper = (code & 1) == 0;        // leaf rows in [a, m): U (V^T w[m:e))
            const int rows = upper ? b.m - b.a : b.e - b.m;
            const int r = lf.a + lane - (upper ? b.a : b.m);
            const T* M = val + (upper ? b.u : b.v) + r;
            const double* tt = t + b.t + (upper ? 0 : b.k);
            for (int c0 = 0; c0 < b.k; c0 += HODLR_CHUNK, ++u) {
                if (u % HODLR_NW != wave) continue;
                const int c1 = min(b.k, c0 + HODLR_CHUNK);
                int c = c0;
                for (; c + 3 < c1; c += 4) {
                    a[0] += (double)M[(int64_t)c * rows] * tt[c];
                    a[1] += (double)M[(int64_t)(c + 1) * rows] * tt[c + 1];
                    a[2] += (double)M[(int64_t)(c + 2) * rows] * tt[c + 2];
                    a[3] += (double)M[(int64_t)(c + 3) * rows] * tt[c + 3];
                }
                for (; c < c1; ++c) a[0] += (double)M[(int64_t)c * rows] * tt[c];
            }
        }
    }
    part[wave][lane] = (a[0] + a[1]) + (a[2] + a[3]);
    __syncthreads();
    if (wave == 0 && lane < len) {
        double s = 0.0;
        for (int k = 0; k < HODLR_NW; ++k) s += part[k][lane];
        x[pos[lf.a + lane]] = s;
    }
}

// ---------------------------------------------------------------------------
// launch wrappers
// ---------------------------------------------------------------------------
static inline unsigned grid_for(int64_t n, int64_t per_block = BLOCK, unsigned cap = 2048) {
    int64_t g = (n + per_block - 1) / per_block;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (unsigned)g;
}

void launch_add2(hipStream_t s, int64_t n, const double* a, const double* b, double* out) {
    if (n <= 0) return;
    k_add2<<<grid_for(n), BLOCK, 0, s>>>(n, a, b, out);
}
template <typename V>
void launch_dense_gemv(hipStream_t s, int64_t n, const double* A, const V* x, V* y) {
    if (n <= 0) return;
    const unsigned g = (unsigned)std::min<int64_t>((n + BLOCK / WAVE - 1) / (BLOCK / WAVE), 65535);
    k_dense_gemv<V><<<g, BLOCK, 0, s>>>(n, A, x, y);
}
template void launch_dense_gemv<double>(hipStream_t, int64_t, const double*, const double*, double*);
template void launch_dense_gemv<float>(hipStream_t, int64_t, const double*, const float*, float*);
void launch_axpy(hipStream_t s, int64_t n, double a, const double* x, double* y) {
    if (n <= 0) return;
    k_axpy<<<grid_for(n), BLOCK, 0, s>>>(n, a, x, y);
}
void launch_fill(hipStream_t s, int64_t n, double* x, double v) {
    if (n <= 0) return;
    k_fill<<<grid_for(n), BLOCK, 0, s>>>(n, x, v);
}
void launch_scatter_in(hipStream_t s, int64_t n, const int64_t* pos, const double* src, double* dst) {
    if (n <= 0) return;
    k_scatter_in<<<grid_for(n), BLOCK, 0, s>>>(n, pos, src, dst);
}
void launch_scatter_in_f(hipStream_t s, int64_t n, const int64_t* pos, const float* src, float* dst) {
    if (n <= 0) return;
    k_scatter_in_f<<<grid_for(n), BLOCK, 0, s>>>(n, pos, src, dst);
}
void launch_gather_f(hipStream_t s, int64_t n, const int64_t* pos, const float* src, float* dst) {
    if (n <= 0) return;
    k_gather_f<<<grid_for(n), BLOCK, 0, s>>>(n, pos, src, dst);
}
void launch_gather_out(hipStream_t s, int64_t n, const int64_t* pos, const double* src, double* dst,
                       const double* sc, int shift_slot, double shift_den) {
    if (n <= 0) return;
    k_gather_out<<<grid_for(n), BLOCK, 0, s>>>(n, pos, src, dst, sc, shift_slot, shift_den);
}
void launch_strang_in(hipStream_t s, int64_t nh, const double* v, double* h, const double* stim, double stim_on,
                      double tau, const IonicConst& c, double* vs) {
    if (nh <= 0) return;
    k_strang_in<<<grid_for(nh), BLOCK, 0, s>>>(nh, v, h, stim, stim_on, tau, c, vs);
}
void launch_strang_out(hipStream_t s, int64_t nh, const int64_t* pos, const double* x2, double* v, double* h,
                       const double* stim, double stim_on, double tau, const IonicConst& c, double* act, double v_act,
                       double t_n, double dt) {
    if (nh <= 0) return;
    k_strang_out<<<grid_for(nh), BLOCK, 0, s>>>(nh, pos, x2, v, h, stim, stim_on, tau, c, act, v_act, t_n, dt);
}
void launch_gather_v_act(hipStream_t s, int64_t n, const int64_t* pos, const double* src, double* dst, double* act,
                         double v_act, double t_n, double dt) {
    if (n <= 0) return;
    k_gather_v_act<<<grid_for(n), BLOCK, 0, s>>>(n, pos, src, dst, act, v_act, t_n, dt);
}
void launch_probe(hipStream_t s, int np, int nv, const int64_t* ids, const double* wts, const double* u,
                  double* out) {
    if (np <= 0) return;
    k_probe<<<(np + BLOCK - 1) / BLOCK, BLOCK, 0, s>>>(np, nv, ids, wts, u, out);
}
void launch_dot_reduce(hipStream_t s, int64_t n, const double* a, const double* b, Reduce rd, double* out) {
    k_dot_reduce<<<grid_for(n, BLOCK * 4, rd.max_blocks), BLOCK, 0, s>>>(n, a, b, rd.partials, rd.counter, out);
}
void launch_multidot(hipStream_t s, int64_t n, const GuessList& W, const double* y, Reduce rd, double* out) {
    k_multidot<<<grid_for(n, BLOCK * 4, rd.max_blocks), BLOCK, 0, s>>>(n, W, y, rd.partials, rd.counter, out);
}
void launch_guess_solve(hipStream_t s, const GuessList& W, const double* d, double* G, const double* b, double* c) {
    k_guess_solve<<<1, 64, 0, s>>>(W, d, G, b, c);
}
void launch_guess_combine(hipStream_t s, int64_t n, const GuessList& W, const double* c, double* x) {
    if (n > 0) k_guess_combine<<<grid_for(n), BLOCK, 0, s>>>(n, W, c, x);
}
void launch_shift(hipStream_t s, int64_t n, double* x, const double* sc, int slot, double den) {
    if (n <= 0) return;
    k_shift<<<grid_for(n), BLOCK, 0, s>>>(n, x, sc, slot, den);
}
void launch_ionic(hipStream_t s, int64_t nh, const double* v, double* h, const double* stim,
                  double stim_on, const double* mh, const int64_t* pos, double* y2, double* x2,
                  const double* sub, const IonicConst& c) {
    if (nh <= 0) return;
    k_ionic_rhs<<<grid_for(nh), BLOCK, 0, s>>>(nh, v, h, stim, stim_on, mh, pos, y2, x2, sub, c);
}

unsigned launch_spmv_lambda(hipStream_t s, const CsrDev& A, int group, int mode, const double* x,
                            const double* y, double* out, double* pp) {
    const unsigned g = grid_for(A.n * group, BLOCK * 2, PP_MAX);
#define BIDO_SPMV_CASE(G)                                                                               \
    if (group == G) {                                                                                   \
        if (mode == 0)                                                                                  \
            k_spmv_lambda<G, 0><<<g, BLOCK, 0, s>>>(A.n, A.ptr, A.col, A.val, x, y, out, pp);           \
        else                                                                                            \
            k_spmv_lambda<G, 1><<<g, BLOCK, 0, s>>>(A.n, A.ptr, A.col, A.val, x, y, out, pp);           \
        return g;                                                                                       \
    }
    BIDO_SPMV_CASE(4) BIDO_SPMV_CASE(8) BIDO_SPMV_CASE(16) BIDO_SPMV_CASE(32)
#undef BIDO_SPMV_CASE
    return 0;
}

unsigned launch_spmv_lam_blk(hipStream_t s, const LamBlk& A, int group, int mode, const double* x, const double* y,
                             double* out, double* pp) {
    (void)group;
    // one lane per two positions of the average row, two passes (measured
    // on the 128^3 slab, 15 positions per row: 8 lanes 5.6 ms per step, 16
    // lanes 6.0, 4 lanes with four passes 7.8)
    const int64_t avg = A.n > 0 ? (A.npos + A.n - 1) / A.n : 1;
    const int g4 = avg <= 8 ? 4 : avg <= 16 ? 8 : avg <= 32 ? 16 : 32;
    const unsigned g = grid_for(A.n * g4, BLOCK * 2, PP_MAX);
    const double2* v = reinterpret_cast<const double2*>(A.val);
#define BIDO_BLK_CASE(G)                                                                                    \
    if (g4 == G) {                                                                                          \
        if (A.c16 && mode == 0)                                                                             \
            k_spmv_lam_blk<G, 2, 0, uint16_t><<<g, BLOCK, 0, s>>>(A.n, A.ptr, A.c16, A.cb, v, A.gm, x, y, out, \
                                                                  pp);                                      \
        else if (A.c16)                                                                                     \
            k_spmv_lam_blk<G, 2, 1, uint16_t><<<g, BLOCK, 0, s>>>(A.n, A.ptr, A.c16, A.cb, v, A.gm, x, y, out, \
                                                                  pp);                                      \
        else if (mode == 0)                                                                                 \
            k_spmv_lam_blk<G, 2, 0, int32_t><<<g, BLOCK, 0, s>>>(A.n, A.ptr, A.col, nullptr, v, A.gm, x, y,    \
                                                                 out, pp);                                  \
        else                                                                                                \
            k_spmv_lam_blk<G, 2, 1, int32_t><<<g, BLOCK, 0, s>>>(A.n, A.ptr, A.col, nullptr, v, A.gm, x, y,    \
                                                                 out, pp);                                  \
        return g;                                                                                           \
    }
    BIDO_BLK_CASE(4) BIDO_BLK_CASE(8) BIDO_BLK_CASE(16) BIDO_BLK_CASE(32)
#undef BIDO_BLK_CASE
    return 0;
}

void launch_spmv_csr(hipStream_t s, const CsrDev& A, int group, const double* x, const double* b,
                     double* y) {
    if (A.n <= 0) return;
    const unsigned g = grid_for(A.n * group, BLOCK * 2, 4096);
    if (group == 4) k_spmv_csr<4><<<g, BLOCK, 0, s>>>(A.n, A.ptr, A.col, A.val, x, b, y);
    else if (group == 8) k_spmv_csr<8><<<g, BLOCK, 0, s>>>(A.n, A.ptr, A.col, A.val, x, b, y);
    else if (group == 16) k_spmv_csr<16><<<g, BLOCK, 0, s>>>(A.n, A.ptr, A.col, A.val, x, b, y);
    else k_spmv_csr<32><<<g, BLOCK, 0, s>>>(A.n, A.ptr, A.col, A.val, x, b, y);
}

void launch_cheb_init(hipStream_t s, int64_t n, const double* t, const double* dinv, double inv_theta, double* d,
                      double* z) {
    if (n <= 0) return;
    k_cheb_init<<<grid_for(n), BLOCK, 0, s>>>(n, t, dinv, inv_theta, d, z);
}
void launch_cheb_step(hipStream_t s, const CsrDev& K, int group, const double* dinv, const double* r_in, double* r,
                      const double* dp, double* dn, double* z, double c1, double c2, bool last) {
    if (K.n <= 0) return;
    const unsigned g = grid_for(K.n * group, BLOCK * 2, 4096);
#define BIDO_CHEB_CASE(G)                                                                                   \
    if (group == G) {                                                                                       \
        k_cheb_step<G><<<g, BLOCK, 0, s>>>(K.n, K.ptr, K.col, K.val, dinv, r_in, r, dp, dn, z, c1, c2,      \
                                           last ? 1 : 0);                                                   \
        return;                                                                                             \
    }
    BIDO_CHEB_CASE(4) BIDO_CHEB_CASE(8) BIDO_CHEB_CASE(16) BIDO_CHEB_CASE(32)
#undef BIDO_CHEB_CASE
}

unsigned launch_pcg_update(hipStream_t s, int64_t n, double* x, double* r, double* r_old, const double* p,
                           const double* q, double* pp, unsigned nb_pq, int rho_slot) {
    const unsigned g = grid_for(n, BLOCK * 4, PP_MAX);
    k_pcg_update<<<g, BLOCK, 0, s>>>(n, x, r, r_old, p, q, pp, (int)nb_pq, rho_slot);
    return g;
}
unsigned launch_combine_dot(hipStream_t s, int64_t n1, int64_t n, double* z, const double* a, const double* b,
                            const double* r, const double* r_old, double* pp) {
    const unsigned g = grid_for(n, BLOCK * 4, PP_MAX);
    k_combine_dot<<<g, BLOCK, 0, s>>>(n1, n, z, a, b, r, r_old, pp);
    return g;
}
void launch_p_update(hipStream_t s, int64_t n, const double* z, double* p, double* pp, unsigned nb_rz, int first,
                     int flexible, int rho_old_slot, int rho_new_slot) {
    k_p_update<<<grid_for(n), BLOCK, 0, s>>>(n, z, p, pp, (int)nb_rz, first, flexible, rho_old_slot, rho_new_slot);
}

template <typename T>
void launch_tri_top(hipStream_t s, const TriPlan& P, const T* inv, const double* b, const double* upd,
                    double* x) {
    const int64_t n = P.n_top;
    if (n <= 0) return;
    k_top_gather<<<(unsigned)((n + BLOCK - 1) / BLOCK), BLOCK, 0, s>>>(n, P.top_pos, P.top_gptr, P.top_gsrc, b,
                                                                        upd, P.top_zero, P.top_w);
    if (P.n_hleaves > 0) {
        if (P.n_hcols > 0)
            k_hodlr_proj<T><<<(unsigned)((P.n_hcols + BLOCK / WAVE - 1) / (BLOCK / WAVE)), BLOCK, 0, s>>>(
                P.hblocks, P.hcols, P.n_hcols, inv, P.top_w, P.ht);
        k_hodlr_apply<T><<<(unsigned)P.n_hleaves, HODLR_BLOCK, 0, s>>>(P.hleaves, P.hblocks, P.hanc, inv, P.top_w,
                                                                       P.ht, P.top_pos, x);
        return;
    }
    k_top_gemv<T><<<(unsigned)((n + TOP_ROWS - 1) / TOP_ROWS), BLOCK, n * sizeof(double), s>>>(
        n, inv, P.top_w, P.top_pos, x);
}

template <typename T>
void launch_tri_fwd_sub(hipStream_t s, const TriPlan& P, const TriNode* nodes, const T* panel_cm,
                        const Ea* ea, const double* b, double* y, double* upd) {
    if (P.n_sub == 0) return;
    k_tri_fwd_sub<T><<<P.n_sub, SUB_BLOCK, 0, s>>>(P.sub_tn, P.sub_hoff, P.hc, panel_cm, ea, b, y, upd, P.skip);
}
template <typename T>
void launch_tri_bwd_sub(hipStream_t s, const TriPlan& P, const TriNode* nodes, const T* panel,
                        const int64_t* bidx, const double* y, double* x) {
    if (P.n_sub == 0) return;
    const int group_max = std::max(0, std::min(SUB_NW / 2, P.bwd_group_max));
    k_tri_bwd_sub<T><<<P.n_sub, SUB_BLOCK, 0, s>>>(P.sub_tn, P.sub_hoff, P.hc, panel, bidx, y, x, group_max,
                                                   P.skip);
}
template <typename T>
void launch_tri_fwd_lvl(hipStream_t s, const TriTopLevel& L, const TriPlan& P, const TriNode* nodes,
                        const T* panel_cm, const Ea* ea, const double* b, double* y, double* upd) {
    if (L.n_fwd == 0) return;
    k_tri_fwd_lvl<T><<<L.n_fwd, BLOCK, L.lds_f + sizeof(double), s>>>(nodes, L.fwd, panel_cm, ea, b, y, upd,
                                                                      P.scratch, (int)(L.lds_f / sizeof(double)),
                                                                      P.skip);
    if (L.n_fcomb > 0)
        k_tri_fwd_comb<<<(L.n_fcomb + BLOCK / WAVE - 1) / (BLOCK / WAVE), BLOCK, 0, s>>>(nodes, L.fcomb, L.n_fcomb,
                                                                                       ea, y, upd, P.scratch, P.skip);
}
template <typename T>
void launch_tri_bwd_lvl(hipStream_t s, const TriTopLevel& L, const TriPlan& P, const TriNode* nodes,
                        const T* panel, const int64_t* bidx, const double* y, double* x) {
    if (L.n_bwd == 0) return;
    const size_t lds = L.lds_b + sizeof(double);
    const int spare = (int)(L.lds_b / sizeof(double));
    if (L.bwd_nt == 1024)
        k_tri_bwd_lvl<T, 1024><<<L.n_bwd, 1024, lds, s>>>(nodes, L.bwd, panel, bidx, y, x, P.scratch, spare, P.skip);
    else
        k_tri_bwd_lvl<T, BLOCK><<<L.n_bwd, BLOCK, lds, s>>>(nodes, L.bwd, panel, bidx, y, x, P.scratch, spare, P.skip);
    if (L.n_bcomb > 0) k_tri_bwd_comb<<<L.n_bcomb, WAVE, 0, s>>>(nodes, L.bcomb, x, P.scratch, P.skip);
}

#define BIDO_INST(T)                                                                                   \
    template void launch_tri_fwd_sub<T>(hipStream_t, const TriPlan&, const TriNode*, const T*,         \
                                        const Ea*, const double*, double*, double*);                   \
    template void launch_tri_bwd_sub<T>(hipStream_t, const TriPlan&, const TriNode*, const T*,         \
                                        const int64_t*, const double*, double*);                       \
    template void launch_tri_fwd_lvl<T>(hipStream_t, const TriTopLevel&, const TriPlan&, const TriNode*, \
                                        const T*, const Ea*, const double*, double*, double*);           \
    template void launch_tri_bwd_lvl<T>(hipStream_t, const TriTopLevel&, const TriPlan&, const TriNode*, \
                                        const T*, const int64_t*, const double*, double*);               \
    template void launch_tri_top<T>(hipStream_t, const TriPlan&, const T*, const double*, const double*, \
                                    double*);
BIDO_INST(double)
BIDO_INST(float)
#undef BIDO_INST

}  // namespace bido
