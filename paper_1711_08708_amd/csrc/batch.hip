// PCG vector kernels of a batch of independent slices held in one union
// vector (slice s at [base[s], base[s] + n2_s), u rows first): each block
// works on a row range of one slice, and every scalar of the recurrences
// (p.q, r.z, alpha, beta) is a per-slice sum of that slice's block partials,
// formed in the same order by every block that needs it.  The blocks of a
// slice whose stopping test is met (done[s]) leave its vectors alone.
#include <hip/hip_runtime.h>

#include "kernels.h"
#include "launch.h"
#include "rows.h"

namespace bido {
namespace {

constexpr int BB = 256;         // threads per block
constexpr int BW = 64;          // wave

__device__ __forceinline__ double wsum(double v) {
#pragma unroll
    for (int o = BW / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, BW);
    return v;
}
__device__ __forceinline__ double bsum(double v, double* sh) {
    v = wsum(v);
    __syncthreads();
    if (threadIdx.x % BW == 0) sh[threadIdx.x / BW] = v;
    __syncthreads();
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < BB / BW; ++k) s += sh[k];
    return s;
}
// sum of the partials of slice s (blocks [b0, b1)), same order in every block
__device__ __forceinline__ double slice_sum(const double* __restrict__ part, int b0, int b1, double* sh) {
    double s = 0.0;
    for (int b = b0 + threadIdx.x; b < b1; b += BB) s += part[b];
    return bsum(s, sh);
}


// mode 0: q = A p, partials p.q;  mode 1: r = y - A x, partials |r|^2, |y|^2
template <int G, int MODE>
__global__ __launch_bounds__(BB) void k_seg_spmv(SegTable T, const int64_t* __restrict__ ptr,
                                                 const int32_t* __restrict__ col, const double* __restrict__ val,
                                                 const double* __restrict__ x, const double* __restrict__ y,
                                                 double* __restrict__ out, double* __restrict__ part0,
                                                 double* __restrict__ part1, const uint8_t* __restrict__ done) {
    __shared__ double sh[BB / BW];
    const SegBlock bk = T.blk[blockIdx.x];
    if (done && done[bk.slice]) return;
    constexpr int RU = SPMV_RU, NG = BB / G;
    const int64_t r0 = bk.r0, r1 = bk.r1;
    const int lane = threadIdx.x % G;
    const int grp = threadIdx.x / G;
    double acc0 = 0.0, acc1 = 0.0;
    for (int64_t rb = r0 + grp; rb < r1; rb += RU * NG) {
        int64_t row[RU];
        bool ok[RU];
        double own[RU];   // x[row] (p.q) or y[row] (residual), loaded with the rows
#pragma unroll
        for (int u = 0; u < RU; ++u) {
            row[u] = rb + u * NG;
            ok[u] = row[u] < r1;
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
    acc0 = bsum(acc0, sh);
    if (MODE == 1) acc1 = bsum(acc1, sh);
    if (threadIdx.x == 0) {
        part0[blockIdx.x] = acc0;
        if (MODE == 1) part1[blockIdx.x] = acc1;
    }
}

// y = b - A x (b may be null: y = A x) on the rows of the table
template <int G>
__global__ __launch_bounds__(BB) void k_seg_csr(SegTable T, const int64_t* __restrict__ ptr,
                                                const int32_t* __restrict__ col, const double* __restrict__ val,
                                                const double* __restrict__ x, const double* __restrict__ b,
                                                double* __restrict__ y, const uint8_t* __restrict__ done) {
    const SegBlock bk = T.blk[blockIdx.x];
    if (done && done[bk.slice]) return;
    constexpr int RU = SPMV_RU, NG = BB / G;
    const int lane = threadIdx.x % G;
    for (int64_t rb = bk.r0 + threadIdx.x / G; rb < bk.r1; rb += RU * NG) {
        int64_t row[RU];
        bool ok[RU];
        double bv[RU];
#pragma unroll
        for (int u = 0; u < RU; ++u) {
            row[u] = rb + u * NG;
            ok[u] = row[u] < bk.r1;
            bv[u] = b ? b[ok[u] ? row[u] : rb] : 0.0;
        }
        double s[RU];
        csr_rows<G, RU>(ptr, col, val, x, row, ok, lane, s);
        if (lane == 0) {
#pragma unroll
            for (int u = 0; u < RU; ++u)
                if (ok[u]) y[row[u]] = b ? bv[u] - s[u] : s[u];
        }
    }
}

// P_K by Chebyshev-accelerated Jacobi on K_m, per slice (its coefficients at
// index slice): d = z = inv_theta[s] D^-1 t on the rows of the table
__global__ __launch_bounds__(BB) void k_seg_cheb_init(SegTable T, const double* __restrict__ t,
                                                      const double* __restrict__ dinv,
                                                      const double* __restrict__ inv_theta, double* __restrict__ d,
                                                      double* __restrict__ z, const uint8_t* __restrict__ done) {
    const SegBlock bk = T.blk[blockIdx.x];
    if (done[bk.slice]) return;
    const double it = inv_theta[bk.slice];
    for (int64_t i = bk.r0 + threadIdx.x; i < bk.r1; i += BB) {
        const double v = it * dinv[i] * t[i];
        d[i] = v;
        z[i] = v;
    }
}

// r = r_in - K dp ; dn = c1[s] dp + c2[s] D^-1 r ; z += dn (r_in may be r;
// the last step writes z only)
template <int G>
__global__ __launch_bounds__(BB) void k_seg_cheb_step(SegTable T, const int64_t* __restrict__ ptr,
                                                      const int32_t* __restrict__ col,
                                                      const double* __restrict__ val,
                                                      const double* __restrict__ dinv, const double* r_in, double* r,
                                                      const double* __restrict__ dp, double* __restrict__ dn,
                                                      double* __restrict__ z, const double* __restrict__ c1,
                                                      const double* __restrict__ c2, int last,
                                                      const uint8_t* __restrict__ done) {
    const SegBlock bk = T.blk[blockIdx.x];
    if (done[bk.slice]) return;
    const double a1 = c1[bk.slice], a2 = c2[bk.slice];
    constexpr int RU = SPMV_RU, NG = BB / G;
    const int lane = threadIdx.x % G;
    for (int64_t rb = bk.r0 + threadIdx.x / G; rb < bk.r1; rb += RU * NG) {
        int64_t row[RU];
        bool ok[RU];
        double rv[RU], dv[RU], di[RU], zv[RU];
#pragma unroll
        for (int u = 0; u < RU; ++u) {
            row[u] = rb + u * NG;
            ok[u] = row[u] < bk.r1;
            const int64_t i = ok[u] ? row[u] : rb;
            rv[u] = r_in[i];
            dv[u] = dp[i];
            di[u] = dinv[i];
            zv[u] = z[i];
        }
        double sum[RU];
        csr_rows<G, RU>(ptr, col, val, dp, row, ok, lane, sum);
        if (lane == 0) {
#pragma unroll
            for (int u = 0; u < RU; ++u) {
                if (!ok[u]) continue;
                const double rn = rv[u] - sum[u];
                const double d = a1 * dv[u] + a2 * di[u] * rn;
                z[row[u]] = zv[u] + d;
                if (!last) {
                    r[row[u]] = rn;
                    dn[row[u]] = d;
                }
            }
        }
    }
}

// alpha_s = rho_s / (p.q)_s (0 for a frozen slice); x += alpha p; r -= alpha q
__global__ __launch_bounds__(BB) void k_seg_pcg_update(SegTable T, double* __restrict__ x, double* __restrict__ r,
                                                       double* __restrict__ r_old, const double* __restrict__ p,
                                                       const double* __restrict__ q,
                                                       const double* __restrict__ part_pq,
                                                       double* __restrict__ part_rr, const double* __restrict__ rho,
                                                       const uint8_t* __restrict__ done, double* __restrict__ pq_out) {
    __shared__ double sh[BB / BW];
    const SegBlock bk = T.blk[blockIdx.x];
    const int s = bk.slice;
    if (done[s]) return;                 // frozen: x, r and its partials stay as they are
    const SegSlice sl = T.sl[s];
    const double pq = slice_sum(part_pq, sl.b0, sl.b1, sh);
    const double alpha = rho[s] / pq;
    if ((int)blockIdx.x == sl.b0 && threadIdx.x == 0) pq_out[s] = pq;
    double acc = 0.0;
    for (int64_t i = bk.r0 + threadIdx.x; i < bk.r1; i += BB) {
        x[i] += alpha * p[i];
        if (r_old) r_old[i] = r[i];
        const double ri = r[i] - alpha * q[i];
        r[i] = ri;
        acc += ri * ri;
    }
    acc = bsum(acc, sh);
    if (threadIdx.x == 0) part_rr[blockIdx.x] = acc;
}

// z = a - b on the u rows of each slice (v rows already hold Z_2);
// partials r.z and r_old.z
__global__ __launch_bounds__(BB) void k_seg_combine(SegTable T, double* __restrict__ z, const double* __restrict__ a,
                                                    const double* __restrict__ bb, const double* __restrict__ r,
                                                    const double* __restrict__ r_old, double* __restrict__ part_rz,
                                                    double* __restrict__ part_zro, const uint8_t* __restrict__ done) {
    __shared__ double sh[BB / BW];
    const SegBlock bk = T.blk[blockIdx.x];
    if (done[bk.slice]) return;
    const SegSlice sl = T.sl[bk.slice];
    const int64_t uend = sl.base + sl.nu;
    double acc = 0.0, acc2 = 0.0;
    for (int64_t i = bk.r0 + threadIdx.x; i < bk.r1; i += BB) {
        double zi;
        if (i < uend) {
            zi = a[i] - bb[i];
            z[i] = zi;
        } else {
            zi = z[i];
        }
        acc += r[i] * zi;
        if (r_old) acc2 += r_old[i] * zi;
    }
    acc = bsum(acc, sh);
    if (r_old) acc2 = bsum(acc2, sh);
    if (threadIdx.x == 0) {
        part_rz[blockIdx.x] = acc;
        if (r_old) part_zro[blockIdx.x] = acc2;
    }
}

// beta_s = (r.z - r_old.z)_s / rho_old_s (0 first or frozen); p = z + beta p;
// block b0[s] stores rho_new_s = (r.z)_s
__global__ __launch_bounds__(BB) void k_seg_p_update(SegTable T, const double* __restrict__ z, double* __restrict__ p,
                                                     const double* __restrict__ part_rz,
                                                     const double* __restrict__ part_zro, int first, int flexible,
                                                     const double* __restrict__ rho_old, double* __restrict__ rho_new,
                                                     const uint8_t* __restrict__ done) {
    __shared__ double sh[BB / BW];
    const SegBlock bk = T.blk[blockIdx.x];
    const int s = bk.slice;
    if (done[s]) return;
    const SegSlice sl = T.sl[s];
    const double rz = slice_sum(part_rz, sl.b0, sl.b1, sh);
    double beta = 0.0;
    if (!first) {
        const double zro = flexible ? slice_sum(part_zro, sl.b0, sl.b1, sh) : 0.0;
        beta = (rz - zro) / rho_old[s];
    }
    if ((int)blockIdx.x == sl.b0 && threadIdx.x == 0) rho_new[s] = rz;
    // the first direction is z itself: p may hold stale bits (0 * NaN = NaN)
    for (int64_t i = bk.r0 + threadIdx.x; i < bk.r1; i += BB) p[i] = first ? z[i] : z[i] + beta * p[i];
}

// The stopping test of every slice after a PCG iteration, on the device (one
// thread per slice): a slice still active counts the iteration, forms
// |r| / |Y| from its |r|^2 partials (summed in block order, as the host did)
// and stops at the tolerance, at a breakdown (p.Ap or r.z not positive, or a
// non-finite residual) or at its iteration cap.  The next iteration's
// kernels read the flags, so the host need not look between iterations.
__global__ void k_seg_stop(int S, SegTable T, const double* __restrict__ part_rr, const double* __restrict__ sc,
                           int rho_slot, const double* __restrict__ yy, const double* __restrict__ tol,
                           const int* __restrict__ max_it, uint8_t* __restrict__ done, int* __restrict__ iters,
                           int* __restrict__ status, double* __restrict__ rel) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= S || done[s]) return;
    double rr = 0.0;
    for (int b = T.sl[s].b0; b < T.sl[s].b1; ++b) rr += part_rr[b];
    const int it = iters[s] + 1;
    iters[s] = it;
    const double q = sqrt(rr / yy[s]);
    const double pq = sc[2 * (int64_t)S + s], rz = sc[(int64_t)rho_slot * S + s];
    rel[s] = q;
    if (!(pq > 0.0) || !(rz > 0.0) || !isfinite(q)) {
        done[s] = 1;
        status[s] = 1;            // breakdown
    } else if (q <= tol[s]) {
        done[s] = 1;
        status[s] = 0;            // converged
    } else if (it >= max_it[s]) {
        done[s] = 1;
        status[s] = 2;            // iteration cap
    }
}

}  // namespace

void launch_seg_spmv(hipStream_t s, const SegTable& T, const CsrDev& A, int group, int mode, const double* x,
                     const double* y, double* out, double* part0, double* part1, const uint8_t* done) {
    if (T.nblocks <= 0) return;
#define BIDO_SEG_CASE(G)                                                                                     \
    if (group == G) {                                                                                        \
        if (mode == 0)                                                                                       \
            k_seg_spmv<G, 0><<<T.nblocks, BB, 0, s>>>(T, A.ptr, A.col, A.val, x, y, out, part0, part1, done); \
        else                                                                                                 \
            k_seg_spmv<G, 1><<<T.nblocks, BB, 0, s>>>(T, A.ptr, A.col, A.val, x, y, out, part0, part1, done); \
        return;                                                                                              \
    }
    BIDO_SEG_CASE(4) BIDO_SEG_CASE(8) BIDO_SEG_CASE(16)
#undef BIDO_SEG_CASE
    if (mode == 0) k_seg_spmv<32, 0><<<T.nblocks, BB, 0, s>>>(T, A.ptr, A.col, A.val, x, y, out, part0, part1, done);
    else k_seg_spmv<32, 1><<<T.nblocks, BB, 0, s>>>(T, A.ptr, A.col, A.val, x, y, out, part0, part1, done);
}
void launch_seg_csr(hipStream_t s, const SegTable& T, const CsrDev& A, int group, const double* x, const double* b,
                    double* y, const uint8_t* done) {
    if (T.nblocks <= 0) return;
    if (group == 4) k_seg_csr<4><<<T.nblocks, BB, 0, s>>>(T, A.ptr, A.col, A.val, x, b, y, done);
    else if (group == 8) k_seg_csr<8><<<T.nblocks, BB, 0, s>>>(T, A.ptr, A.col, A.val, x, b, y, done);
    else if (group == 16) k_seg_csr<16><<<T.nblocks, BB, 0, s>>>(T, A.ptr, A.col, A.val, x, b, y, done);
    else k_seg_csr<32><<<T.nblocks, BB, 0, s>>>(T, A.ptr, A.col, A.val, x, b, y, done);
}
void launch_seg_cheb_init(hipStream_t s, const SegTable& T, const double* t, const double* dinv,
                          const double* inv_theta, double* d, double* z, const uint8_t* done) {
    if (T.nblocks <= 0) return;
    k_seg_cheb_init<<<T.nblocks, BB, 0, s>>>(T, t, dinv, inv_theta, d, z, done);
}
void launch_seg_cheb_step(hipStream_t s, const SegTable& T, const CsrDev& K, int group, const double* dinv,
                          const double* r_in, double* r, const double* dp, double* dn, double* z, const double* c1,
                          const double* c2, bool last, const uint8_t* done) {
    if (T.nblocks <= 0) return;
#define BIDO_SEG_CHEB_CASE(G)                                                                             \
    if (group == G) {                                                                                     \
        k_seg_cheb_step<G><<<T.nblocks, BB, 0, s>>>(T, K.ptr, K.col, K.val, dinv, r_in, r, dp, dn, z, c1, \
                                                    c2, last ? 1 : 0, done);                              \
        return;                                                                                           \
    }
    BIDO_SEG_CHEB_CASE(4) BIDO_SEG_CHEB_CASE(8) BIDO_SEG_CHEB_CASE(16) BIDO_SEG_CHEB_CASE(32)
#undef BIDO_SEG_CHEB_CASE
}
void launch_seg_pcg_update(hipStream_t s, const SegTable& T, double* x, double* r, double* r_old, const double* p,
                           const double* q, const double* part_pq, double* part_rr, const double* rho,
                           const uint8_t* done, double* pq_out) {
    if (T.nblocks <= 0) return;
    k_seg_pcg_update<<<T.nblocks, BB, 0, s>>>(T, x, r, r_old, p, q, part_pq, part_rr, rho, done, pq_out);
}
void launch_seg_combine(hipStream_t s, const SegTable& T, double* z, const double* a, const double* b,
                        const double* r, const double* r_old, double* part_rz, double* part_zro,
                        const uint8_t* done) {
    if (T.nblocks <= 0) return;
    k_seg_combine<<<T.nblocks, BB, 0, s>>>(T, z, a, b, r, r_old, part_rz, part_zro, done);
}
void launch_seg_p_update(hipStream_t s, const SegTable& T, const double* z, double* p, const double* part_rz,
                         const double* part_zro, int first, int flexible, const double* rho_old, double* rho_new,
                         const uint8_t* done) {
    if (T.nblocks <= 0) return;
    k_seg_p_update<<<T.nblocks, BB, 0, s>>>(T, z, p, part_rz, part_zro, first, flexible, rho_old, rho_new, done);
}

void launch_seg_stop(hipStream_t s, int S, const SegTable& T, const double* part_rr, const double* sc, int rho_slot,
                     const double* yy, const double* tol, const int* max_it, uint8_t* done, int* iters, int* status,
                     double* rel) {
    if (S <= 0) return;
    k_seg_stop<<<(S + BB - 1) / BB, BB, 0, s>>>(S, T, part_rr, sc, rho_slot, yy, tol, max_it, done, iters, status,
                                                rel);
}

}  // namespace bido
