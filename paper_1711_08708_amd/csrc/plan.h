// Device layout and execution plan of one factor's triangular sweeps, built
// on the host (pure C++), plus a sequential CPU emulation of the sweep
// kernels that runs the same plan with the same index arithmetic.
#pragma once
#include <string>
#include <vector>

#include "host.h"
#include "kernels.h"

namespace bido {

struct FactorPlan {
    int64_t n = 0, ground = -1;
    int height = 0;
    std::vector<TriNode> nodes;
    std::vector<double> panel;          // FP64 panels, row-major packed (see TriNode)
    std::vector<double> panel_cm;       // the same panels, column-major packed
    std::vector<int64_t> bidx;          // boundary indices of every node
    std::vector<Ea> ea;                 // extend-add maps
    int64_t upd_size = 0;               // update workspace entries
    int max_nI = 0;
    // subtree phase
    int hc = -1, n_sub = 0, sub_maxw = 0;
    std::vector<int32_t> sub_nodes, sub_hoff;
    // level phases (heights hc+1 .. height)
    std::vector<TriItem> fwd_items;
    std::vector<BwdItem> bwd_items;
    struct Span { size_t f0, nf, b0, nb, lds_f, lds_b; };
    std::vector<Span> spans;
    int64_t scratch_size = 0;           // partial sums of split tiles
    int n_tiles = 0;                    // completion counters (forward + backward)
    // algorithmic bytes per height (panel at 8 or 4 bytes per entry)
    std::vector<double> fwd_bytes64, bwd_bytes64, fwd_bytes32, bwd_bytes32;
    double sub_fwd_bytes64 = 0, sub_bwd_bytes64 = 0, sub_fwd_bytes32 = 0, sub_bwd_bytes32 = 0;
    int64_t meta_bytes = 0;
};

// Limits and tile sizes the kernels rely on.
constexpr int PLAN_SUB_MAXW = 256;     // own size of a node in the subtree phase
constexpr int PLAN_SUB_MAXF = 384;     // panel rows of a node in the subtree phase
constexpr int PLAN_LDS_MAXW = 1 << 20; // (no own-size limit in the level phases)
constexpr int PLAN_FWD_ROWS = 64;      // forward row tile (one row per lane)
constexpr int PLAN_FWD_COLS = 128;     // forward column chunk per work item (4 waves)
constexpr int PLAN_BWD_MAXR = 512;     // backward rows per work item (LDS staging)

bool build_plan(const Factor& f, FactorPlan& p, std::string& err);

// CPU emulation of the sweep kernels over the plan: x = (L L^T)^-1 b.
void emulate_plan(const FactorPlan& p, const double* b, double* x);

}  // namespace bido
