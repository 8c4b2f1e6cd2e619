// Device layout and execution plan of one factor's triangular sweeps, built
// on the host (pure C++), plus a sequential CPU emulation of the sweep
// kernels that runs the same plan with the same index arithmetic.
#pragma once
#include <string>
#include <vector>

#include "host.h"
#include "kernels.h"

namespace bido {

// Work-item shapes, the subtree cuts and the top cut of a plan.  Zero or
// negative values take the built-in defaults (the cost model for the top
// cut).  These are the only plan knobs; the library reads no environment.
struct PlanOptions {
    int fwd_cols = 0;   // columns per forward level item (0: PLAN_FWD_COLS)
    int bwd_rows = 0;   // rows per backward level item (0: the level rule below)
    int top_h = -1;     // first height of the top (raised to fit the top-size bound)
    int sub_h = -1;     // highest subtree cut of any tree (< 0: the size rule alone)
    int sub_want = 0;   // subtrees wanted per tree (0: 256)
    int sub_total = 0;  // > 0: subtrees wanted over the whole forest, shared by the trees
                        // in proportion to their vertices (each tree's cut then stays
                        // below its recorded top cut); 0: sub_want per tree
    int bwd_wide = -1;  // backward level items of 1024 threads over whole column tiles
                        // (1), of 256 threads over row ranges (0); < 0: 1
    int level_items = -1; // wide backward items wanted per level of tall tiles (< 0:
                          // PLAN_BWD_LEVEL_ITEMS; 0 keeps every tile whole)
    int bwd_group_max = 0; // backward subtree heights with at most this many nodes
                           // use wave groups (0: 2 in 2D, 4 in 3D)
};

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
    int hc = -1, n_sub = 0, sub_maxw = 0;  // hc: the highest subtree cut of any tree
    std::vector<int32_t> sub_nodes, sub_hoff;
    std::vector<TriNode> sub_tn;        // node records in sub_nodes order
    // level phases: span k covers height lvl0 + k (heights above each tree's
    // subtree cut, below its top)
    int lvl0 = 0;
    std::vector<TriItem> fwd_items;
    std::vector<BwdItem> bwd_items;
    // split tiles (more than one item) are summed by a combine launch after
    // their level: one entry (the tile's first item) per split tile
    std::vector<TriItem> fwd_comb;
    std::vector<BwdItem> bwd_comb;
    struct Span { size_t f0, nf, b0, nb, lds_f, lds_b, cf0, ncf, cb0, ncb; };
    bool bwd_wide = false;              // backward level items of 1024 threads
    std::vector<Span> spans;
    int64_t scratch_size = 0;           // partial sums of split tiles
    int n_tiles = 0;                    // tiles (forward + backward)
    // dense top: the nodes of height >= top_h are replaced by x_top = S_top^-1 w_top,
    // S_top the Schur complement of their vertices (top_h = height + 1: none)
    int top_h = 0;
    int64_t n_top = 0;
    std::vector<int64_t> top_pos;       // top index -> vertex (tree order)
    std::vector<uint8_t> top_zero;      // 1 at the grounded top entries
    std::vector<int32_t> top_gptr;      // top index -> [gptr, gptr+1) in top_gsrc
    std::vector<int64_t> top_gsrc;      // update-workspace entries of the bottom roots
    std::vector<double> top_inv;        // S_top^-1, n_top x n_top row-major (exact mode)
    bool top_hodlr = false;             // S_top^-1 in hierarchical low-rank form instead
    Hodlr hodlr;                        // (top indices then in bisection order)
    std::vector<int32_t> hodlr_cols;    // projection columns: block << 16 | column
    double top_seconds = 0.0;           // host time spent on S_top^-1
    // algorithmic bytes per height (panel at 8 or 4 bytes per entry)
    std::vector<double> fwd_bytes64, bwd_bytes64, fwd_bytes32, bwd_bytes32;
    double sub_fwd_bytes64 = 0, sub_bwd_bytes64 = 0, sub_fwd_bytes32 = 0, sub_bwd_bytes32 = 0;
    int64_t meta_bytes = 0;
    PlanOptions used;                   // the options the plan was built with
};

// Limits and tile sizes the kernels rely on.
constexpr int PLAN_SUB_MAXW = 256;     // own size of a node in the subtree phase
constexpr int PLAN_SUB_MAXF = 384;     // panel rows of a node in the subtree phase
constexpr int PLAN_LDS_MAXW = 1 << 20; // (no own-size limit in the level phases)
constexpr int PLAN_FWD_ROWS = 64;      // forward row tile (one row per lane)
constexpr int PLAN_FWD_COLS = 128;     // forward column chunk per work item (4 waves)
constexpr int PLAN_BWD_MAXR = 512;     // backward rows per 256-thread work item (LDS staging)
constexpr int PLAN_BWD_WIDE = 1024;    // threads of a wide backward work item
constexpr int PLAN_BWD_LEVEL_ITEMS = 512; // wide backward items wanted per level (2 per CU)
constexpr int PLAN_LDS_DOUBLES = 4096; // bound of the LDS staging per level item
constexpr int PLAN_TOP_MAX = 6144;     // max n_top (w_top staged in LDS, FP64)
constexpr int PLAN_HODLR_LEAF = 64;    // leaf size of the hierarchical top

// n_threads: host threads for S_top^-1 (<= 0: OpenMP default).
bool build_plan(const Factor& f, FactorPlan& p, std::string& err, int n_threads = 0,
                const PlanOptions* opt = nullptr);

// CPU emulation of the sweep kernels over the plan: x = (L L^T)^-1 b.
void emulate_plan(const FactorPlan& p, const double* b, double* x);

}  // namespace bido
