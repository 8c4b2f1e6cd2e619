// CSR row products shared by the SpMV kernels (kernels.hip, batch.hip): a
// group of G lanes computes RU rows at once.  The first two G-wide passes
// over each row load unconditionally (an entry past the row's end rereads
// entry 0 of the arrays and is dropped by a select), so the row pointers,
// the column/value pairs and the gathered x of all RU rows are each one
// memory latency, not one per row.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace bido {

constexpr int SPMV_RU = 4;   // rows per group in flight
constexpr unsigned XCDS = 8; // the dispatcher deals workgroups round robin over 8 XCDs

// The rows [r0, r1) of this workgroup.  Each workgroup takes a contiguous
// range, and the workgroups of one XCD take consecutive ranges (logical index
// = the XCD's first index + its count of earlier workgroups), so an XCD sweeps
// one contiguous part of the rows: the vector entries its rows gather stay in
// its own L2 instead of being fetched by every XCD.
struct RowRange {
    int64_t r0, r1;
};
__device__ __forceinline__ RowRange block_rows(int64_t n) {
    const unsigned nb = gridDim.x, b = blockIdx.x;
    const unsigned x = b % XCDS, q = nb / XCDS, rem = nb % XCDS;
    const unsigned lb = x * q + (x < rem ? x : rem) + b / XCDS;
    const int64_t rpb = (n + nb - 1) / nb;
    const int64_t r0 = (int64_t)lb * rpb < n ? (int64_t)lb * rpb : n;
    return {r0, r0 + rpb < n ? r0 + rpb : n};
}

template <int G>
__device__ __forceinline__ double lane_group_sum(double v) {
#pragma unroll
    for (int o = G / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, G);
    return v;
}

// s[u] = (A x)[row[u]] for the rows with ok[u] (ok[0] must hold; the other
// s[u] are not meaningful); every lane of the group gets the sums
template <int G, int RU>
__device__ __forceinline__ void csr_rows(const int64_t* __restrict__ ptr, const int32_t* __restrict__ col,
                                         const double* __restrict__ val, const double* x, const int64_t (&row)[RU],
                                         const bool (&ok)[RU], int lane, double (&s)[RU]) {
    int64_t pb[RU], pe[RU];
    // a row past the range repeats row[0] (its sums are not used), so the
    // pointer loads need no select that could sink them into a branch
#pragma unroll
    for (int u = 0; u < RU; ++u) {
        const int64_t rr = ok[u] ? row[u] : row[0];
        pb[u] = ptr[rr];
        pe[u] = ptr[rr + 1];
    }
#pragma unroll
    for (int u = 0; u < RU; ++u) s[u] = 0.0;
#pragma unroll
    for (int k = 0; k < 2; ++k)
#pragma unroll
        for (int u = 0; u < RU; ++u) {
            const int64_t q = pb[u] + lane + k * G;
            const bool in = q < pe[u];
            const int64_t qc = in ? q : 0;
            const double v = val[qc] * x[col[qc]];
            s[u] += in ? v : 0.0;
        }
#pragma unroll
    for (int u = 0; u < RU; ++u)
        for (int64_t q = pb[u] + lane + 2 * G; q < pe[u]; q += G) s[u] += val[q] * x[col[q]];
#pragma unroll
    for (int u = 0; u < RU; ++u) s[u] = lane_group_sum<G>(s[u]);
}

}  // namespace bido
