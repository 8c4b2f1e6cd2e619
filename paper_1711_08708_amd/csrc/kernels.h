// Device data layouts shared by the HIP kernels and the driver.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace bido {

// One tree node of a hierarchical Cholesky factor, as seen by the kernels.
// The panel P_t = [L_tt^-1 ; L_Bt L_tt^-1] is stored row-major with the
// L_tt^-1 rows packed (row r holds r+1 entries) followed by nB full rows of
// nI entries.
struct TriNode {
    int64_t off;     // first own index in the vector
    int64_t panel;   // offset of P_t in the panel array (elements)
    int64_t bidx;    // offset of B(t) in the boundary index array
    int64_t upd;     // offset of the update vector c_t in the workspace
    int64_t ea;      // offset of the extend-add map (nI + nB entries)
    int32_t nI, nB;
    int32_t child[2];
};

// A unit of work of one level: rows [start, start+count) of a panel in the
// forward sweep, or columns [start, start+count) in the backward sweep.
struct TriItem {
    int32_t node;
    int32_t start;
    int32_t count;
    int32_t group;   // lanes per row (forward) / per column tile width (backward)
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
    S_COUNT = 32
};

}  // namespace bido
