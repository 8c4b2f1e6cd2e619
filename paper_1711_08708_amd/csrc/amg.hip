// HIP kernels of the multigrid V-cycle (the alternative inner solves P_1,
// P_K of the block-LU preconditioner; host side in amg.cpp, driver in
// api.cpp).  Every product is a CSR row product by a group of G lanes with
// RU rows in flight (the row helper of the Lambda product), with the matrix
// values in FP64 or, in mixed precision, FP32 (FP64 accumulation); the
// level vectors are FP64 or FP32 (XV, BV, YV, VV, ZV: the input, added,
// output, level and result vector types of a kernel): the cycle is bound
// by the bytes of its level matrices and vectors.  A
// matrix whose rows each span fewer than 65536 columns (a banded order)
// holds its columns as 16-bit offsets from a per-row base (C = uint16_t,
// 2 instead of 4 bytes per entry); C = int32_t is the plain column.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "launch.h"
#include "rows.h"

namespace bido {

namespace {

constexpr int BLOCK = 256;
// rows per lane group in flight, and rounds of them per workgroup: many
// small workgroups (128^3 slab, mixed: RU 2 / ITER 1 gives 20.2 steps/s,
// 4 / 1 19.7, 4 / 2 18.2, 8 / 1 13.1, 4 / 4 16.0)
constexpr int RU = 2;
constexpr int ITER = 1;

template <int G>
__device__ __forceinline__ double group_sum(double v) {
#pragma unroll
    for (int o = G / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, G);
    return v;
}

// s[u] = sum_j A[row_u, j] x[j] for RU rows (FP64 accumulation); entries
// past a row's end reread entry 0 and are dropped by a select.  Column j of
// an entry is col[q] (C = int32_t) or cb[row] + col[q] (C = uint16_t).
template <int G, int K, typename T, typename C, typename XV>
__device__ __forceinline__ void rows_dot(const int64_t* __restrict__ ptr, const C* __restrict__ col,
                                         const int32_t* __restrict__ cb, const T* __restrict__ val,
                                         const XV* __restrict__ x, const int64_t (&row)[RU], const bool (&ok)[RU],
                                         int lane, double (&s)[RU]) {
    int64_t pb[RU], pe[RU];
    int32_t c0[RU];
#pragma unroll
    for (int u = 0; u < RU; ++u) {
        const int64_t rr = ok[u] ? row[u] : row[0];
        pb[u] = ptr[rr];
        pe[u] = ptr[rr + 1];
        if constexpr (sizeof(C) == 2) c0[u] = cb[rr];
        else c0[u] = 0;
        s[u] = 0.0;
    }
#pragma unroll
    for (int k = 0; k < K; ++k)
#pragma unroll
        for (int u = 0; u < RU; ++u) {
            const int64_t q = pb[u] + lane + k * G;
            const bool in = q < pe[u];
            const int64_t qc = in ? q : 0;
            const int32_t c = c0[u] + (int32_t)col[qc];
            const double v = (double)val[qc] * (double)x[c];
            s[u] += in ? v : 0.0;
        }
#pragma unroll
    for (int u = 0; u < RU; ++u)
        for (int64_t q = pb[u] + lane + K * G; q < pe[u]; q += G) {
            const int32_t c = c0[u] + (int32_t)col[q];
            s[u] += (double)val[q] * (double)x[c];
        }
#pragma unroll
    for (int u = 0; u < RU; ++u) s[u] = group_sum<G>(s[u]);
}

// y = b + sign * A x  (b may be null)
template <int G, int K, typename T, typename C, typename XV, typename BV, typename YV>
__global__ __launch_bounds__(BLOCK) void k_amg_spmv(int64_t n, const int64_t* __restrict__ ptr,
                                                    const C* __restrict__ col, const int32_t* __restrict__ cb,
                                                    const T* __restrict__ val,
                                                    const XV* __restrict__ x, const BV* __restrict__ b,
                                                    double sign, YV* __restrict__ y) {
    const int lane = threadIdx.x % G;
    constexpr int GPB = BLOCK / G;     // lane groups per workgroup
    const RowRange rr = block_rows(n);
    for (int64_t rb = rr.r0 + threadIdx.x / G; rb < rr.r1; rb += RU * GPB) {
        int64_t row[RU];
        bool ok[RU];
#pragma unroll
        for (int u = 0; u < RU; ++u) {
            row[u] = rb + u * GPB;
            ok[u] = row[u] < rr.r1;
        }
        double s[RU];
        rows_dot<G, K, T, C, XV>(ptr, col, cb, val, x, row, ok, lane, s);
        if (lane == 0) {
#pragma unroll
            for (int u = 0; u < RU; ++u)
                if (ok[u]) y[row[u]] = (YV)((b ? (double)b[row[u]] : 0.0) + sign * s[u]);
        }
    }
}

// One Chebyshev step from zero, the damped Jacobi sweep, plus an optional
// base: z = base + a0 D^-1 b.
template <typename BV, typename VV, typename ZV>
__global__ __launch_bounds__(BLOCK) void k_amg_jacobi(int64_t n, const BV* __restrict__ b,
                                                      const VV* __restrict__ dinv, double a0,
                                                      const VV* __restrict__ base, ZV* __restrict__ z) {
    for (int64_t i = blockIdx.x * (int64_t)BLOCK + threadIdx.x; i < n; i += (int64_t)gridDim.x * BLOCK)
        z[i] = (ZV)((base ? (double)base[i] : 0.0) + a0 * (double)dinv[i] * (double)b[i]);
}

// The first two Chebyshev smoothing steps from z = 0 in one pass:
// d0 = a0 D^-1 b, r1 = b - A d0 = b - a0 (A D^-1) b (the column-scaled copy
// As = A D^-1 of the level matrix, so one gather per entry),
// d1 = c1 d0 + c2 D^-1 r1, z = base + d0 + d1 (base may be null); r1, d0
// and d1 are kept when more steps follow (write_rd).
template <int G, int K, typename T, typename C, typename BV, typename VV, typename ZV>
__global__ __launch_bounds__(BLOCK) void k_amg_smooth2(int64_t n, const int64_t* __restrict__ ptr,
                                                       const C* __restrict__ col, const int32_t* __restrict__ cb,
                                                       const T* __restrict__ val, const VV* __restrict__ dinv,
                                                       const BV* __restrict__ b, double a0, double c1, double c2,
                                                       const VV* __restrict__ base,
                                                       ZV* __restrict__ z, VV* __restrict__ r1,
                                                       VV* __restrict__ d0o, VV* __restrict__ d1o,
                                                       int write_rd) {
    const int lane = threadIdx.x % G;
    constexpr int GPB = BLOCK / G;     // lane groups per workgroup
    const RowRange rr = block_rows(n);
    for (int64_t rb = rr.r0 + threadIdx.x / G; rb < rr.r1; rb += RU * GPB) {
        int64_t row[RU];
        bool ok[RU];
        double bv[RU], di[RU];
#pragma unroll
        for (int u = 0; u < RU; ++u) {
            row[u] = rb + u * GPB;
            ok[u] = row[u] < rr.r1;
            const int64_t i = ok[u] ? row[u] : rb;
            bv[u] = (double)b[i];
            di[u] = (double)dinv[i];
        }
        double s[RU];
        rows_dot<G, K, T, C, BV>(ptr, col, cb, val, b, row, ok, lane, s);        // (A D^-1 b)_i, val = As
        if (lane == 0) {
#pragma unroll
            for (int u = 0; u < RU; ++u) {
                if (!ok[u]) continue;
                const double d0 = a0 * di[u] * bv[u];
                const double r = bv[u] - a0 * s[u];
                const double d1 = c1 * d0 + c2 * di[u] * r;
                z[row[u]] = (ZV)((base ? (double)base[row[u]] : 0.0) + d0 + d1);
                if (write_rd) {
                    r1[row[u]] = (VV)r;
                    d0o[row[u]] = (VV)d0;
                    d1o[row[u]] = (VV)d1;
                }
            }
        }
    }
}

// One more Chebyshev step: r -= A dp, dn = c1 dp + c2 D^-1 r, z += dn.
template <int G, int K, typename T>
__global__ __launch_bounds__(BLOCK) void k_amg_cheb(int64_t n, const int64_t* __restrict__ ptr,
                                                    const int32_t* __restrict__ col, const T* __restrict__ val,
                                                    const double* __restrict__ dinv, double* r,
                                                    const double* __restrict__ dp, double* __restrict__ dn,
                                                    double* __restrict__ z, double c1, double c2) {
    const int lane = threadIdx.x % G;
    constexpr int GPB = BLOCK / G;     // lane groups per workgroup
    const RowRange rr = block_rows(n);
    for (int64_t rb = rr.r0 + threadIdx.x / G; rb < rr.r1; rb += RU * GPB) {
        int64_t row[RU];
        bool ok[RU];
        double rv[RU], dv[RU], di[RU], zv[RU];
#pragma unroll
        for (int u = 0; u < RU; ++u) {
            row[u] = rb + u * GPB;
            ok[u] = row[u] < rr.r1;
            const int64_t i = ok[u] ? row[u] : rb;
            rv[u] = r[i];
            dv[u] = dp[i];
            di[u] = dinv[i];
            zv[u] = z[i];
        }
        double s[RU];
        rows_dot<G, K, T, int32_t, double>(ptr, col, nullptr, val, dp, row, ok, lane, s);
        if (lane == 0) {
#pragma unroll
            for (int u = 0; u < RU; ++u) {
                if (!ok[u]) continue;
                const double rn = rv[u] - s[u];
                const double d = c1 * dv[u] + c2 * di[u] * rn;
                r[row[u]] = rn;
                dn[row[u]] = d;
                z[row[u]] = zv[u] + d;
            }
        }
    }
}

// workgroups of ITER rounds of RU rows per lane group
unsigned grid_rows(int64_t n, int G) {
    const int64_t rows = (int64_t)ITER * RU * (BLOCK / G);
    return (unsigned)std::max<int64_t>(1, (n + rows - 1) / rows);
}

// ---------------------------------------------------------------------------
// A new gamma on the device (a change of time step with a multigrid P_K):
// A_l += dg M_l, D^-1, the column-scaled copy, the Lanczos estimate of the
// smoother bound and the coarsest inverse.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(BLOCK) void k_amg_shift(int64_t nnz, double dg, const double* __restrict__ mass,
                                                     double* __restrict__ a64, float* __restrict__ a32) {
    for (int64_t p = blockIdx.x * (int64_t)BLOCK + threadIdx.x; p < nnz; p += (int64_t)gridDim.x * BLOCK) {
        const double v = a64[p] + dg * mass[p];
        a64[p] = v;
        if (a32) a32[p] = (float)v;
    }
}

// D^-1 of every row (the excluded row keeps 0), FP64 and FP32
__global__ __launch_bounds__(BLOCK) void k_amg_dinv(int64_t n, const int64_t* __restrict__ ptr,
                                                    const int32_t* __restrict__ col, const double* __restrict__ val,
                                                    int64_t excluded, double* __restrict__ dinv,
                                                    float* __restrict__ dinv32) {
    for (int64_t i = blockIdx.x * (int64_t)BLOCK + threadIdx.x; i < n; i += (int64_t)gridDim.x * BLOCK) {
        double d = 0.0;
        for (int64_t q = ptr[i]; q < ptr[i + 1]; ++q)
            if (col[q] == i) d += val[q];
        const double v = i == excluded ? 0.0 : 1.0 / d;
        dinv[i] = v;
        if (dinv32) dinv32[i] = (float)v;
    }
}

// A D^-1 (columns scaled), FP64 and FP32
__global__ __launch_bounds__(BLOCK) void k_amg_colscale(int64_t nnz, const int32_t* __restrict__ col,
                                                        const double* __restrict__ val,
                                                        const double* __restrict__ dinv, double* __restrict__ s64,
                                                        float* __restrict__ s32) {
    for (int64_t p = blockIdx.x * (int64_t)BLOCK + threadIdx.x; p < nnz; p += (int64_t)gridDim.x * BLOCK) {
        const double v = val[p] * dinv[col[p]];
        s64[p] = v;
        s32[p] = (float)v;
    }
}

// Lanczos on D^-1/2 A D^-1/2: t = D^-1/2 v; w = D^-1/2 y - beta vp; vp = v, v = w / b
__global__ __launch_bounds__(BLOCK) void k_lz_in(int64_t n, const double* __restrict__ dinv,
                                                 const double* __restrict__ v, double* __restrict__ t) {
    for (int64_t i = blockIdx.x * (int64_t)BLOCK + threadIdx.x; i < n; i += (int64_t)gridDim.x * BLOCK)
        t[i] = sqrt(dinv[i]) * v[i];
}
__global__ __launch_bounds__(BLOCK) void k_lz_w(int64_t n, const double* __restrict__ dinv,
                                                const double* __restrict__ y, double beta,
                                                const double* __restrict__ vp, double* __restrict__ w) {
    for (int64_t i = blockIdx.x * (int64_t)BLOCK + threadIdx.x; i < n; i += (int64_t)gridDim.x * BLOCK)
        w[i] = sqrt(dinv[i]) * y[i] - beta * vp[i];
}
__global__ __launch_bounds__(BLOCK) void k_lz_next(int64_t n, const double* __restrict__ w, double inv_b,
                                                   double* __restrict__ v, double* __restrict__ vp) {
    for (int64_t i = blockIdx.x * (int64_t)BLOCK + threadIdx.x; i < n; i += (int64_t)gridDim.x * BLOCK) {
        vp[i] = v[i];
        v[i] = w[i] * inv_b;
    }
}

// dense n x n copy of a CSR matrix (the output zeroed before); with an
// excluded row, its row and column become the unit vector
__global__ __launch_bounds__(BLOCK) void k_amg_densify(int64_t n, const int64_t* __restrict__ ptr,
                                                       const int32_t* __restrict__ col,
                                                       const double* __restrict__ val, int64_t excluded,
                                                       double* __restrict__ m) {
    for (int64_t i = blockIdx.x * (int64_t)BLOCK + threadIdx.x; i < n; i += (int64_t)gridDim.x * BLOCK) {
        if (i == excluded) {
            m[i * n + i] = 1.0;
            continue;
        }
        for (int64_t q = ptr[i]; q < ptr[i + 1]; ++q)
            if (col[q] != excluded) m[i * n + col[q]] = val[q];
    }
}
// Gauss-Jordan inversion in place, pivot k (SPD: no pivoting).  prep: f =
// column k (f[k] the pivot); row: row k / pivot with the identity's 1 at
// (k, k); update: every other row i minus f[i] times row k, its entry k
// starting from the identity's 0.
__global__ __launch_bounds__(BLOCK) void k_gj_prep(int64_t n, int64_t k, const double* __restrict__ m,
                                                   double* __restrict__ f) {
    for (int64_t i = blockIdx.x * (int64_t)BLOCK + threadIdx.x; i < n; i += (int64_t)gridDim.x * BLOCK)
        f[i] = m[i * n + k];
}
__global__ __launch_bounds__(BLOCK) void k_gj_row(int64_t n, int64_t k, double* __restrict__ m,
                                                  const double* __restrict__ f) {
    const double inv = 1.0 / f[k];
    for (int64_t j = blockIdx.x * (int64_t)BLOCK + threadIdx.x; j < n; j += (int64_t)gridDim.x * BLOCK)
        m[k * n + j] = (j == k ? 1.0 : m[k * n + j]) * inv;
}
__global__ __launch_bounds__(BLOCK) void k_gj_update(int64_t n, int64_t k, double* __restrict__ m,
                                                     const double* __restrict__ f) {
    const int64_t nn = n * n;
    for (int64_t e = blockIdx.x * (int64_t)BLOCK + threadIdx.x; e < nn; e += (int64_t)gridDim.x * BLOCK) {
        const int64_t i = e / n, j = e - i * n;
        if (i == k) continue;
        m[e] = (j == k ? 0.0 : m[e]) - f[i] * m[k * n + j];
    }
}
// the excluded row and column of the inverse are 0
__global__ __launch_bounds__(BLOCK) void k_amg_zero_rc(int64_t n, int64_t r, double* __restrict__ m) {
    for (int64_t j = blockIdx.x * (int64_t)BLOCK + threadIdx.x; j < n; j += (int64_t)gridDim.x * BLOCK) {
        m[r * n + j] = 0.0;
        m[j * n + r] = 0.0;
    }
}

__global__ __launch_bounds__(BLOCK) void k_amg_fill(int64_t n, double* __restrict__ m) {
    for (int64_t i = blockIdx.x * (int64_t)BLOCK + threadIdx.x; i < n; i += (int64_t)gridDim.x * BLOCK) m[i] = 0.0;
}

unsigned grid_elems(int64_t n) {
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + BLOCK - 1) / BLOCK, 8192));
}

}  // namespace

void launch_amg_shift(hipStream_t s, int64_t nnz, double dg, const double* mass, double* a64, float* a32) {
    if (nnz > 0) k_amg_shift<<<grid_elems(nnz), BLOCK, 0, s>>>(nnz, dg, mass, a64, a32);
}
void launch_amg_dinv(hipStream_t s, int64_t n, const int64_t* ptr, const int32_t* col, const double* val,
                     int64_t excluded, double* dinv, float* dinv32) {
    if (n > 0) k_amg_dinv<<<grid_elems(n), BLOCK, 0, s>>>(n, ptr, col, val, excluded, dinv, dinv32);
}
void launch_amg_colscale(hipStream_t s, int64_t nnz, const int32_t* col, const double* val, const double* dinv,
                         double* s64, float* s32) {
    if (nnz > 0) k_amg_colscale<<<grid_elems(nnz), BLOCK, 0, s>>>(nnz, col, val, dinv, s64, s32);
}
void launch_lz_in(hipStream_t s, int64_t n, const double* dinv, const double* v, double* t) {
    if (n > 0) k_lz_in<<<grid_elems(n), BLOCK, 0, s>>>(n, dinv, v, t);
}
void launch_lz_w(hipStream_t s, int64_t n, const double* dinv, const double* y, double beta, const double* vp,
                 double* w) {
    if (n > 0) k_lz_w<<<grid_elems(n), BLOCK, 0, s>>>(n, dinv, y, beta, vp, w);
}
void launch_lz_next(hipStream_t s, int64_t n, const double* w, double inv_b, double* v, double* vp) {
    if (n > 0) k_lz_next<<<grid_elems(n), BLOCK, 0, s>>>(n, w, inv_b, v, vp);
}
void launch_amg_dense_inverse(hipStream_t s, int64_t n, const int64_t* ptr, const int32_t* col, const double* val,
                              int64_t excluded, double* m, double* f) {
    if (n <= 0) return;
    k_amg_fill<<<grid_elems(n * n), BLOCK, 0, s>>>(n * n, m);
    k_amg_densify<<<grid_elems(n), BLOCK, 0, s>>>(n, ptr, col, val, excluded, m);
    for (int64_t k = 0; k < n; ++k) {
        k_gj_prep<<<grid_elems(n), BLOCK, 0, s>>>(n, k, m, f);
        k_gj_row<<<grid_elems(n), BLOCK, 0, s>>>(n, k, m, f);
        k_gj_update<<<grid_elems(n * n), BLOCK, 0, s>>>(n, k, m, f);
    }
    if (excluded >= 0) k_amg_zero_rc<<<grid_elems(n), BLOCK, 0, s>>>(n, excluded, m);
}

// lane groups of G lanes, K unrolled passes of G entries per row (the
// average row length over G, 2 to 4; longer rows finish in a loop)
#define BIDO_K_SWITCH(K, ...)                                   \
    switch (K) {                                                \
        case 2: { constexpr int KK = 2; __VA_ARGS__; } break;   \
        case 3: { constexpr int KK = 3; __VA_ARGS__; } break;   \
        default: { constexpr int KK = 4; __VA_ARGS__; } break;  \
    }
#define BIDO_G_SWITCH(A, ...)                                                       \
    {                                                                               \
        const int kk = unroll_for(A);                                               \
        switch (A.group) {                                                          \
            case 2: { constexpr int GG = 2; BIDO_K_SWITCH(kk, __VA_ARGS__) } break;   \
            case 4: { constexpr int GG = 4; BIDO_K_SWITCH(kk, __VA_ARGS__) } break;   \
            case 8: { constexpr int GG = 8; BIDO_K_SWITCH(kk, __VA_ARGS__) } break;   \
            case 16: { constexpr int GG = 16; BIDO_K_SWITCH(kk, __VA_ARGS__) } break; \
            case 32: { constexpr int GG = 32; BIDO_K_SWITCH(kk, __VA_ARGS__) } break; \
            default: { constexpr int GG = 64; BIDO_K_SWITCH(kk, __VA_ARGS__) } break; \
        }                                                                           \
    }

template <typename T>
int unroll_for(const AmgMat<T>& A) {
    const int64_t per = A.group * (int64_t)std::max<int64_t>(A.n, 1);
    const int64_t k = (A.nnz + per - 1) / per;
    return (int)std::min<int64_t>(4, std::max<int64_t>(2, k));
}

template <typename T, typename XV, typename BV, typename YV>
void launch_amg_spmv(hipStream_t s, const AmgMat<T>& A, const XV* x, const BV* b, double sign, YV* y) {
    if (A.n <= 0) return;
    if (A.c16)
        BIDO_G_SWITCH(A, k_amg_spmv<GG, KK, T, uint16_t, XV, BV, YV><<<grid_rows(A.n, GG), BLOCK, 0, s>>>(
                             A.n, A.ptr, A.c16, A.cb, A.val, x, b, sign, y))
    else
        BIDO_G_SWITCH(A, k_amg_spmv<GG, KK, T, int32_t, XV, BV, YV><<<grid_rows(A.n, GG), BLOCK, 0, s>>>(
                             A.n, A.ptr, A.col, nullptr, A.val, x, b, sign, y))
}

template <typename T, typename BV, typename VV, typename ZV>
void launch_amg_smooth2(hipStream_t s, const AmgMat<T>& A, const VV* dinv, const BV* b, double a0, double c1,
                        double c2, const VV* base, ZV* z, VV* r1, VV* d0, VV* d1, bool write_rd) {
    if (A.n <= 0) return;
    if (A.c16)
        BIDO_G_SWITCH(A, k_amg_smooth2<GG, KK, T, uint16_t, BV, VV, ZV><<<grid_rows(A.n, GG), BLOCK, 0, s>>>(
                             A.n, A.ptr, A.c16, A.cb, A.val, dinv, b, a0, c1, c2, base, z, r1, d0, d1,
                             write_rd ? 1 : 0))
    else
        BIDO_G_SWITCH(A, k_amg_smooth2<GG, KK, T, int32_t, BV, VV, ZV><<<grid_rows(A.n, GG), BLOCK, 0, s>>>(
                             A.n, A.ptr, A.col, nullptr, A.val, dinv, b, a0, c1, c2, base, z, r1, d0, d1,
                             write_rd ? 1 : 0))
}

template <typename BV, typename VV, typename ZV>
void launch_amg_jacobi(hipStream_t s, int64_t n, const BV* b, const VV* dinv, double a0, const VV* base, ZV* z) {
    if (n <= 0) return;
    const unsigned g = (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + BLOCK - 1) / BLOCK, 4096));
    k_amg_jacobi<BV, VV, ZV><<<g, BLOCK, 0, s>>>(n, b, dinv, a0, base, z);
}

template <typename T>
void launch_amg_cheb(hipStream_t s, const AmgMat<T>& A, const double* dinv, double* r, const double* dp, double* dn,
                     double* z, double c1, double c2) {
    if (A.n <= 0) return;
    BIDO_G_SWITCH(A, k_amg_cheb<GG, KK, T><<<grid_rows(A.n, GG), BLOCK, 0, s>>>(A.n, A.ptr, A.col, A.val, dinv, r,
                                                                                    dp, dn, z, c1, c2))
}

#undef BIDO_G_SWITCH
#undef BIDO_K_SWITCH

// the vector types in use: FP64 throughout (FP64 cycles, the coupling
// blocks), and in the mixed-precision cycle FP32 level vectors with the
// finest level's FP64 input and output
#define BIDO_SPMV(T, XV, BV, YV) \
    template void launch_amg_spmv<T, XV, BV, YV>(hipStream_t, const AmgMat<T>&, const XV*, const BV*, double, YV*);
#define BIDO_SM(T, BV, VV, ZV)                                                                                    \
    template void launch_amg_smooth2<T, BV, VV, ZV>(hipStream_t, const AmgMat<T>&, const VV*, const BV*, double,  \
                                                    double, double, const VV*, ZV*, VV*, VV*, VV*, bool);
#define BIDO_JAC(BV, VV, ZV) \
    template void launch_amg_jacobi<BV, VV, ZV>(hipStream_t, int64_t, const BV*, const VV*, double, const VV*, ZV*);
BIDO_SPMV(double, double, double, double)
BIDO_SPMV(float, double, double, double)
BIDO_SPMV(float, float, double, float)
BIDO_SPMV(float, float, float, float)
BIDO_SM(double, double, double, double)
BIDO_SM(float, double, double, double)
BIDO_SM(float, double, float, float)
BIDO_SM(float, float, float, double)
BIDO_SM(float, float, float, float)
BIDO_JAC(double, double, double)
BIDO_JAC(double, float, float)
BIDO_JAC(float, float, double)
BIDO_JAC(float, float, float)
template void launch_amg_cheb<double>(hipStream_t, const AmgMat<double>&, const double*, double*, const double*,
                                      double*, double*, double, double);
template void launch_amg_cheb<float>(hipStream_t, const AmgMat<float>&, const double*, double*, const double*,
                                     double*, double*, double, double);
#undef BIDO_SPMV
#undef BIDO_SM
#undef BIDO_JAC

}  // namespace bido
