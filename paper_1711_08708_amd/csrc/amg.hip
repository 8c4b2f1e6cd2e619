// HIP kernels of the multigrid V-cycle (the alternative inner solves P_1,
// P_K of the block-LU preconditioner; host side in amg.cpp, driver in
// api.cpp).  Every product is a CSR row product by a group of G lanes with
// RU rows in flight (the row helper of the Lambda product), with the matrix
// values in FP64 or, in mixed precision, FP32 (FP64 accumulation, FP64
// vectors): the cycle is bound by the bytes of its level matrices.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "launch.h"
#include "rows.h"

namespace bido {

namespace {

constexpr int BLOCK = 256;
constexpr int RU = 4;
constexpr int ITER = 2;       // row rounds of RU rows per lane group and workgroup

template <int G>
__device__ __forceinline__ double group_sum(double v) {
#pragma unroll
    for (int o = G / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, G);
    return v;
}

// s[u] = sum_j A[row_u, j] * f(j) for RU rows, f(j) = x[j] (or x[j] * w[j]
// when w is given: the scaled input of a fused smoother step); entries
// past a row's end reread entry 0 and are dropped by a select.
template <int G, int K, typename T>
__device__ __forceinline__ void rows_dot(const int64_t* __restrict__ ptr, const int32_t* __restrict__ col,
                                         const T* __restrict__ val, const double* __restrict__ x,
                                         const double* __restrict__ w, const int64_t (&row)[RU],
                                         const bool (&ok)[RU], int lane, double (&s)[RU]) {
    int64_t pb[RU], pe[RU];
#pragma unroll
    for (int u = 0; u < RU; ++u) {
        const int64_t rr = ok[u] ? row[u] : row[0];
        pb[u] = ptr[rr];
        pe[u] = ptr[rr + 1];
        s[u] = 0.0;
    }
#pragma unroll
    for (int k = 0; k < K; ++k)
#pragma unroll
        for (int u = 0; u < RU; ++u) {
            const int64_t q = pb[u] + lane + k * G;
            const bool in = q < pe[u];
            const int64_t qc = in ? q : 0;
            const int32_t c = col[qc];
            double xv = x[c];
            if (w) xv *= w[c];
            const double v = (double)val[qc] * xv;
            s[u] += in ? v : 0.0;
        }
#pragma unroll
    for (int u = 0; u < RU; ++u)
        for (int64_t q = pb[u] + lane + K * G; q < pe[u]; q += G) {
            const int32_t c = col[q];
            double xv = x[c];
            if (w) xv *= w[c];
            s[u] += (double)val[q] * xv;
        }
#pragma unroll
    for (int u = 0; u < RU; ++u) s[u] = group_sum<G>(s[u]);
}

// y = b + sign * A x  (b may be null)
template <int G, int K, typename T>
__global__ __launch_bounds__(BLOCK) void k_amg_spmv(int64_t n, const int64_t* __restrict__ ptr,
                                                    const int32_t* __restrict__ col, const T* __restrict__ val,
                                                    const double* __restrict__ x, const double* __restrict__ b,
                                                    double sign, double* __restrict__ y) {
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
        rows_dot<G, K, T>(ptr, col, val, x, nullptr, row, ok, lane, s);
        if (lane == 0) {
#pragma unroll
            for (int u = 0; u < RU; ++u)
                if (ok[u]) y[row[u]] = (b ? b[row[u]] : 0.0) + sign * s[u];
        }
    }
}

// One Chebyshev step from zero, the damped Jacobi sweep, plus an optional
// base: z = base + a0 D^-1 b.
__global__ __launch_bounds__(BLOCK) void k_amg_jacobi(int64_t n, const double* __restrict__ b,
                                                      const double* __restrict__ dinv, double a0,
                                                      const double* __restrict__ base, double* __restrict__ z) {
    for (int64_t i = blockIdx.x * (int64_t)BLOCK + threadIdx.x; i < n; i += (int64_t)gridDim.x * BLOCK)
        z[i] = (base ? base[i] : 0.0) + a0 * dinv[i] * b[i];
}

// The first two Chebyshev smoothing steps from z = 0 in one pass:
// d0 = a0 D^-1 b, r1 = b - A d0 = b - a0 (A D^-1) b (the column-scaled copy
// As = A D^-1 of the level matrix, so one gather per entry),
// d1 = c1 d0 + c2 D^-1 r1, z = base + d0 + d1 (base may be null); r1, d0
// and d1 are kept when more steps follow (write_rd).
template <int G, int K, typename T>
__global__ __launch_bounds__(BLOCK) void k_amg_smooth2(int64_t n, const int64_t* __restrict__ ptr,
                                                       const int32_t* __restrict__ col,
                                                       const T* __restrict__ val, const double* __restrict__ dinv,
                                                       const double* __restrict__ b, double a0, double c1, double c2,
                                                       const double* __restrict__ base,
                                                       double* __restrict__ z, double* __restrict__ r1,
                                                       double* __restrict__ d0o, double* __restrict__ d1o,
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
            bv[u] = b[i];
            di[u] = dinv[i];
        }
        double s[RU];
        rows_dot<G, K, T>(ptr, col, val, b, nullptr, row, ok, lane, s);   // (A D^-1 b)_i with val = As
        if (lane == 0) {
#pragma unroll
            for (int u = 0; u < RU; ++u) {
                if (!ok[u]) continue;
                const double d0 = a0 * di[u] * bv[u];
                const double r = bv[u] - a0 * s[u];
                const double d1 = c1 * d0 + c2 * di[u] * r;
                z[row[u]] = (base ? base[row[u]] : 0.0) + d0 + d1;
                if (write_rd) {
                    r1[row[u]] = r;
                    d0o[row[u]] = d0;
                    d1o[row[u]] = d1;
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
        rows_dot<G, K, T>(ptr, col, val, dp, nullptr, row, ok, lane, s);
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

}  // namespace

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

template <typename T>
void launch_amg_spmv(hipStream_t s, const AmgMat<T>& A, const double* x, const double* b, double sign, double* y) {
    if (A.n <= 0) return;
    BIDO_G_SWITCH(A, k_amg_spmv<GG, KK, T><<<grid_rows(A.n, GG), BLOCK, 0, s>>>(A.n, A.ptr, A.col, A.val, x, b,
                                                                                    sign, y))
}

template <typename T>
void launch_amg_smooth2(hipStream_t s, const AmgMat<T>& A, const double* dinv, const double* b, double a0, double c1,
                        double c2, const double* base, double* z, double* r1, double* d0, double* d1,
                        bool write_rd) {
    if (A.n <= 0) return;
    BIDO_G_SWITCH(A, k_amg_smooth2<GG, KK, T><<<grid_rows(A.n, GG), BLOCK, 0, s>>>(
                         A.n, A.ptr, A.col, A.val, dinv, b, a0, c1, c2, base, z, r1, d0, d1, write_rd ? 1 : 0))
}

void launch_amg_jacobi(hipStream_t s, int64_t n, const double* b, const double* dinv, double a0, const double* base,
                       double* z) {
    if (n <= 0) return;
    const unsigned g = (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + BLOCK - 1) / BLOCK, 4096));
    k_amg_jacobi<<<g, BLOCK, 0, s>>>(n, b, dinv, a0, base, z);
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

#define BIDO_INST(T)                                                                                              \
    template void launch_amg_spmv<T>(hipStream_t, const AmgMat<T>&, const double*, const double*, double, double*); \
    template void launch_amg_smooth2<T>(hipStream_t, const AmgMat<T>&, const double*, const double*, double,       \
                                        double, double, const double*, double*, double*, double*, double*, bool);  \
    template void launch_amg_cheb<T>(hipStream_t, const AmgMat<T>&, const double*, double*, const double*,         \
                                     double*, double*, double, double);
BIDO_INST(double)
BIDO_INST(float)
#undef BIDO_INST

}  // namespace bido
