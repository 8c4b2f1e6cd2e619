// Device data layouts shared by the HIP kernels and the host code.
#pragma once
#include <cstdint>

namespace bido {

// One tree node of a hierarchical Cholesky factor, as seen by the kernels.
// The panel P_t = [L_tt^-1 ; L_Bt L_tt^-1] ((nI+nB) x nI, lower-triangular
// top block) is stored twice, at the same offset of two arrays:
//   row-major:    row r holds r+1 entries (r < nI) or nI entries (r >= nI)
//   column-major: column c holds rows c .. nI+nB-1
// The forward sweep (one thread per row) reads the column-major copy, the
// backward sweep (one thread per column) the row-major one, so both read
// consecutive addresses across the lanes of a wave.
struct TriNode {
    int64_t off;     // first own index in the vector
    int64_t panel;   // offset of P_t in the panel array (elements)
    int64_t bidx;    // offset of B(t) in the boundary index array
    int64_t upd;     // offset of the update vector c_t in the workspace
    int64_t ea;      // offset of the extend-add map (nI + nB entries)
    int64_t u0, u1;  // update offsets of the two children (0 when absent)
    int32_t nI, nB;
    int32_t child[2];
    int32_t gi;      // own index of a grounded vertex (its entry is fixed to 0), or -1
    int32_t tree;    // slice of a merged forest the node belongs to (0 otherwise)
};

// Extend-add map entry: position in each child's update vector (-1: none).
struct Ea {
    int32_t a, b;
};

// Forward work item of one level above the subtree cut: rows
// [r0, r0+nrows) (nrows <= 64) of the panel of `node`, columns [cs, ce).
// Items that split a row tile's columns write 64 partial sums each to
// scratch; the combine launch after the level sums the parts in order and
// stores the rows.
struct TriItem {
    int32_t node;
    int32_t r0, nrows;
    int32_t cs, ce;
    int32_t nparts;      // items of this row tile
    int32_t tile;        // index of the tile (plan bookkeeping)
    int32_t pad;
    int64_t part;        // scratch offset of this item's partial sums
    int64_t part0;       // scratch offset of the tile's first part
};

// Backward work item of one level above the subtree cut: columns
// [c0, c0+ncols) of the panel of `node`, rows [rs, re).  Items that share a
// column tile write W partial sums each to scratch; the combine launch after
// the level sums the parts in order (deterministic) and writes x.
struct BwdItem {
    int32_t node;
    int32_t c0, ncols, W;
    int32_t rs, re;
    int32_t nparts;      // items of this column tile
    int32_t tile;        // index of the tile (plan bookkeeping)
    int64_t part;        // scratch offset of this item's partial sums
    int64_t part0;       // scratch offset of the tile's first part
};

// Hierarchical (off-diagonal low-rank) form of a symmetric matrix in a
// bisection order: block b couples rows [a, m) with columns [m, e) as
// U V^T (U: (m-a) x k, V: (e-m) x k, both column-major at offsets u, v of the
// value array); its transpose couples [m, e) with [a, m).  t is the offset
// of the block's projections V^T w[m:e) and U^T w[a:m) (k each).
struct HodlrBlock {
    int32_t a, m, e, k;
    int64_t u, v;
    int32_t t, pad;
};
// Leaf rows [a, e): dense diagonal block (column-major at offset d) and the
// list anc[anc .. anc+nanc) of its ancestor blocks, each coded 2*block +
// (1 if the leaf lies in the block's second half).
struct HodlrLeaf {
    int32_t a, e, nanc, anc;
    int64_t d;
};

// Scalars of the PCG recurrences, resident on the device.
enum ScalarSlot {
    S_RHO = 0,      // r^T z of the current search direction
    S_RHO_NEW,      // r^T z after the latest preconditioner apply
    S_ZR_OLD,       // z^T r_old (flexible CG; adjacent to S_RHO_NEW)
    S_PQ,           // p^T Lambda p
    S_RR,           // |r|^2
    S_YY,           // |Y|^2 (adjacent to S_RR)
    S_MU,           // (M U, 1)
    S_Y1SUM,        // sum of Y_1 (range check)
    S_TN2,          // |t|^2 of the learned correction's input
    S_ALPHA,        // step length of the latest PCG update
    S_EL_RR,        // |b - S_1 x|^2 of the elliptic solve of a Strang step
    S_EL_BB,        // |b|^2 of that solve
    S_LZ,           // a dot product of the multigrid smoother-bound estimate
    S_COUNT = 32
};

// Per-block partial sums of the PCG reductions, stored right after the
// scalar slots in the same device buffer: region k holds at most PP_MAX
// block partials.  The kernel that needs a total sums the partials itself
// (every block in the same order), so no reduction needs a device-scope
// fence; the host sums the regions it reads.
enum PartialRegion { PP_RR = 0, PP_YY, PP_RZ, PP_ZRO, PP_PQ, PP_COUNT };
constexpr int PP_MAX = 1024;
constexpr int64_t pp_offset(int region) { return S_COUNT + (int64_t)region * PP_MAX; }

}  // namespace bido
