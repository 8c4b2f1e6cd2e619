// Device context, the PCG loop and the C ABI (include/bido.h).
//
// Step 2 of the resolution algorithm (Sec. 3.2) is solved by conjugate
// gradient on Lambda X = Y, preconditioned by the block-LU preconditioner
// of Def. 2: with P_1 ~ S_1 (grounded, hierarchical Cholesky) and
// P_K ~ K_m = gamma M_H + S_m (Sec. 5.2), X = P_Lambda^-1 R is
//     Z1 = P_1^-1 R1,  Z2 = P_K^-1 (R2 - S_i Pi Z1),
//     X1 = Z1 - P_1^-1 Pi^T S_i Z2,  X2 = Z2.
// Scalars, dot products and vector updates stay in FP64; in mixed mode only
// the factors are read in FP32 and the outer iteration is flexible CG.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <random>
#include <string>
#include <type_traits>
#include <vector>

#include "../../include/bido.h"
#include "gnn.h"
#include "launch.h"
#include "plan.h"
#include "setup.h"

using namespace bido;

namespace {

thread_local std::string g_err;

bido_status fail(bido_status code, const std::string& msg) {
    g_err = msg;
    return code;
}

#define HIP_OK(expr)                                                                  \
    do {                                                                              \
        hipError_t e_ = (expr);                                                       \
        if (e_ != hipSuccess)                                                         \
            return fail(BIDO_ERR_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

template <typename T>
hipError_t upload(T** dst, const T* src, size_t n) {
    *dst = nullptr;
    if (n == 0) return hipSuccess;
    hipError_t e = hipMalloc((void**)dst, n * sizeof(T));
    if (e != hipSuccess) return e;
    return hipMemcpy(*dst, src, n * sizeof(T), hipMemcpyHostToDevice);
}

int pow2_at_least(int n, int cap) {
    int g = 1;
    while (g < n && g < cap) g <<= 1;
    return g;
}

// Kernel classes of the optional per-launch profiler.
enum KClass { K_SPMV_LAMBDA = 0, K_PCG_UPDATE, K_COMBINE_DOT, K_P_UPDATE, K_TRI_FWD_SUB,
              K_TRI_FWD_LVL, K_TRI_BWD_SUB, K_TRI_BWD_LVL, K_TRI_TOP, K_SPMV_CSR, K_IONIC, K_GNN, K_MISC,
              K_CHEB, K_AMG_SMOOTH, K_AMG_SPMV, K_AMG_TRANSFER, K_AMG_COARSE, K_NCLASS };
const char* const kclass_name[K_NCLASS] = {"spmv_lambda", "pcg_update", "combine_dot", "p_update",
                                           "tri_fwd_sub", "tri_fwd_lvl", "tri_bwd_sub", "tri_bwd_lvl",
                                           "tri_top", "spmv_csr", "ionic_rhs", "gnn_infer", "misc",
                                           "pk_chebyshev", "amg_smooth_l0", "amg_resid_l0", "amg_transfer_l0",
                                           "amg_coarser"};

// Per-launch HIP-event timing with the algorithmic bytes of each launch.
struct Profiler {
    bool on = false;
    struct Rec { int cls; hipEvent_t a, b; double bytes; };
    std::vector<hipEvent_t> pool;
    size_t used = 0;
    std::vector<Rec> recs;
    hipEvent_t get() {
        if (used == pool.size()) {
            hipEvent_t e;
            hipEventCreate(&e);
            pool.push_back(e);
        }
        return pool[used++];
    }
    ~Profiler() { for (auto e : pool) hipEventDestroy(e); }
};

// Device copy of one hierarchical Cholesky factor.
struct FactorDev {
    int64_t n = 0, ground = -1;
    int height = 0;
    int lvl0 = 0;                   // height of the first level phase
    TriNode* nodes = nullptr;
    double* panel64 = nullptr;      // row-major copy (backward sweep)
    float* panel32 = nullptr;
    double* panel64_cm = nullptr;   // column-major copy (forward sweep)
    float* panel32_cm = nullptr;
    Ea* ea = nullptr;
    int64_t* bidx = nullptr;
    double* upd = nullptr;
    double* ytmp = nullptr;
    TriItem* items = nullptr;
    BwdItem* bitems = nullptr;
    TriItem* fcomb = nullptr;
    BwdItem* bcomb = nullptr;
    double* top_inv64 = nullptr;    // dense top S_top^-1 (n_top x n_top)
    float* top_inv32 = nullptr;
    double top_bytes64 = 0, top_bytes32 = 0;
    int top_h = 0;
    double top_seconds = 0;
    PlanOptions opts;               // the options of the current plan
    TriPlan plan;
    std::vector<TriTopLevel> top;                   // heights hc+1 .. height
    std::vector<double> fwd_bytes64, bwd_bytes64;   // algorithmic bytes per height (FP64 panel)
    std::vector<double> fwd_bytes32, bwd_bytes32;   // same with the FP32 panel
    double sub_fwd_bytes64 = 0, sub_bwd_bytes64 = 0, sub_fwd_bytes32 = 0, sub_bwd_bytes32 = 0;
    int64_t panel_entries = 0;
    int64_t dense_entries = 0;
    int64_t meta_bytes = 0;
    int64_t upd_size = 0;
    int64_t scratch_size = 0;       // split-tile partial sums (doubles)
    int64_t ht_size = 0;            // projections of the hierarchical top (doubles)
    int64_t top_lowrank = 0;        // blocks of rank > 0 stored in the hierarchical top
    int max_nI = 0;

    void release() {
        hipFree(nodes); hipFree(panel64); hipFree(panel32); hipFree(panel64_cm); hipFree(panel32_cm);
        hipFree(ea); hipFree(bidx);
        hipFree(upd); hipFree(ytmp); hipFree(items); hipFree(bitems);
        hipFree(plan.sub_nodes); hipFree(plan.sub_tn); hipFree(plan.sub_hoff); hipFree(plan.scratch);
        hipFree(fcomb); hipFree(bcomb); fcomb = nullptr; bcomb = nullptr;
        hipFree(top_inv64); hipFree(top_inv32); top_inv64 = nullptr; top_inv32 = nullptr;
        hipFree((void*)plan.hblocks); hipFree((void*)plan.hleaves); hipFree((void*)plan.hanc);
        hipFree((void*)plan.hcols); hipFree(plan.ht);
        hipFree((void*)plan.top_pos); hipFree((void*)plan.top_gptr); hipFree((void*)plan.top_gsrc);
        hipFree((void*)plan.top_zero);
        hipFree(plan.top_w);
        nodes = nullptr; panel64 = nullptr; panel32 = nullptr; panel64_cm = nullptr; panel32_cm = nullptr;
        ea = nullptr; bidx = nullptr;
        upd = nullptr; ytmp = nullptr; items = nullptr; bitems = nullptr;
        plan = TriPlan();
    }
};

struct CsrHostView {
    static bido_status up(const Csr& a, CsrDev& d) {
        d.n = a.n;
        d.nnz = a.nnz();
        HIP_OK(upload(&d.ptr, a.ptr.data(), a.ptr.size()));
        HIP_OK(upload(&d.col, a.col.data(), a.col.size()));
        HIP_OK(upload(&d.val, a.val.data(), a.val.size()));
        return BIDO_OK;
    }
    static void release(CsrDev& d) {
        hipFree(d.ptr); hipFree(d.col); hipFree(d.val); hipFree(d.c16); hipFree(d.cb);
        d = CsrDev();
    }
    // the compact columns of d (c16, cb) when every row of a spans fewer
    // than 65536 columns; otherwise none (the products read col)
    static bido_status compact(const Csr& a, CsrDev& d) {
        if (a.nnz() == 0 || a.n <= 0) return BIDO_OK;
        std::vector<int32_t> base(a.n, 0);
        for (int64_t i = 0; i < a.n; ++i) {
            if (a.ptr[i] == a.ptr[i + 1]) continue;
            int32_t lo = a.col[a.ptr[i]], hi = lo;
            for (int64_t q = a.ptr[i]; q < a.ptr[i + 1]; ++q) {
                lo = std::min(lo, a.col[q]);
                hi = std::max(hi, a.col[q]);
            }
            if ((int64_t)hi - lo > 65535) return BIDO_OK;
            base[i] = lo;
        }
        std::vector<uint16_t> c16(a.nnz());
        for (int64_t i = 0; i < a.n; ++i)
            for (int64_t q = a.ptr[i]; q < a.ptr[i + 1]; ++q) c16[q] = (uint16_t)(a.col[q] - base[i]);
        HIP_OK(upload(&d.c16, c16.data(), c16.size()));
        HIP_OK(upload(&d.cb, base.data(), base.size()));
        return BIDO_OK;
    }
};

bido_status build_factor_dev(const Factor& f, bool want32, FactorDev& fd, int n_threads = 0,
                             const PlanOptions* opt = nullptr) {
    FactorPlan p;
    std::string err;
    if (!build_plan(f, p, err, n_threads, opt)) return fail(BIDO_ERR_ARG, err);
    fd.opts = p.used;
    fd.n = p.n;
    fd.ground = p.ground;
    fd.height = p.height;
    fd.max_nI = p.max_nI;
    fd.upd_size = p.upd_size;
    fd.scratch_size = p.scratch_size;
    fd.panel_entries = (int64_t)p.panel.size();
    fd.dense_entries = f.dense_entries();
    HIP_OK(upload(&fd.nodes, p.nodes.data(), p.nodes.size()));
    HIP_OK(upload(&fd.panel64, p.panel.data(), p.panel.size()));
    HIP_OK(upload(&fd.panel64_cm, p.panel_cm.data(), p.panel_cm.size()));
    if (want32) {
        std::vector<float> p32(p.panel.begin(), p.panel.end());
        HIP_OK(upload(&fd.panel32, p32.data(), p32.size()));
        std::vector<float> c32(p.panel_cm.begin(), p.panel_cm.end());
        HIP_OK(upload(&fd.panel32_cm, c32.data(), c32.size()));
    }
    HIP_OK(upload(&fd.ea, p.ea.data(), p.ea.size()));
    HIP_OK(upload(&fd.bidx, p.bidx.data(), p.bidx.size()));
    HIP_OK(upload(&fd.items, p.fwd_items.data(), p.fwd_items.size()));
    HIP_OK(upload(&fd.bitems, p.bwd_items.data(), p.bwd_items.size()));
    fd.plan.hc = p.hc;
    // backward subtree heights of at most this many nodes use wave groups:
    // the thin upper nodes of 2D subtrees gain nothing from them beyond 2,
    // the fat 3D ones do up to 4 (slab64 tri_bwd_sub 133 -> 102 us)
    fd.plan.bwd_group_max = p.used.bwd_group_max > 0 ? p.used.bwd_group_max : (f.dim == 3 ? 4 : 2);
    fd.lvl0 = p.lvl0;
    fd.plan.n_sub = p.n_sub;
    fd.plan.sub_maxw = p.sub_maxw;
    HIP_OK(upload(&fd.plan.sub_nodes, p.sub_nodes.data(), p.sub_nodes.size()));
    HIP_OK(upload(&fd.plan.sub_tn, p.sub_tn.data(), p.sub_tn.size()));
    HIP_OK(upload(&fd.plan.sub_hoff, p.sub_hoff.data(), p.sub_hoff.size()));
    HIP_OK(hipMalloc((void**)&fd.plan.scratch, std::max<int64_t>(p.scratch_size, 1) * sizeof(double)));
    HIP_OK(upload(&fd.fcomb, p.fwd_comb.data(), p.fwd_comb.size()));   // empty: no combine launch
    HIP_OK(upload(&fd.bcomb, p.bwd_comb.data(), p.bwd_comb.size()));
    HIP_OK(hipMalloc((void**)&fd.upd, std::max<int64_t>(p.upd_size, 1) * sizeof(double)));
    HIP_OK(hipMemset(fd.upd, 0, sizeof(double)));                    // the 0.0 entry
    HIP_OK(hipMalloc((void**)&fd.ytmp, std::max<int64_t>(p.n, 1) * sizeof(double)));
    fd.top_h = p.top_h;
    fd.top_seconds = p.top_seconds;
    fd.plan.n_top = p.n_top;
    if (p.n_top > 0) {
        int64_t* pos = nullptr; int32_t* gptr = nullptr; int64_t* gsrc = nullptr; uint8_t* zero = nullptr;
        HIP_OK(upload(&pos, p.top_pos.data(), p.top_pos.size()));
        HIP_OK(upload(&zero, p.top_zero.data(), p.top_zero.size()));
        fd.plan.top_zero = zero;
        HIP_OK(upload(&gptr, p.top_gptr.data(), p.top_gptr.size()));
        HIP_OK(upload(&gsrc, p.top_gsrc.data(), p.top_gsrc.size()));
        fd.plan.top_pos = pos; fd.plan.top_gptr = gptr; fd.plan.top_gsrc = gsrc;
        HIP_OK(hipMalloc((void**)&fd.plan.top_w, p.n_top * sizeof(double)));
        const std::vector<double>& vals = p.top_hodlr ? p.hodlr.val : p.top_inv;
        HIP_OK(upload(&fd.top_inv64, vals.data(), vals.size()));
        if (want32) {
            std::vector<float> i32(vals.begin(), vals.end());
            HIP_OK(upload(&fd.top_inv32, i32.data(), i32.size()));
        }
        double vec = 8.0 * (3.0 * p.n_top) + 16.0 * (double)p.top_gsrc.size();
        if (p.top_hodlr) {
            const Hodlr& hd = p.hodlr;
            HodlrBlock* hb = nullptr; HodlrLeaf* hl = nullptr; int32_t* ha = nullptr; int32_t* hc = nullptr;
            HIP_OK(upload(&hb, hd.blocks.data(), hd.blocks.size()));
            HIP_OK(upload(&hl, hd.leaves.data(), hd.leaves.size()));
            HIP_OK(upload(&ha, hd.anc.data(), hd.anc.size()));
            HIP_OK(upload(&hc, p.hodlr_cols.data(), p.hodlr_cols.size()));
            fd.plan.hblocks = hb; fd.plan.hleaves = hl; fd.plan.hanc = ha; fd.plan.hcols = hc;
            fd.plan.n_hblocks = (int)hd.blocks.size();
            fd.plan.n_hleaves = (int)hd.leaves.size();
            fd.plan.n_hcols = (int)p.hodlr_cols.size();
            HIP_OK(hipMalloc((void**)&fd.plan.ht, hd.t_size * sizeof(double)));
            fd.ht_size = hd.t_size;
            fd.top_lowrank = 0;
            for (const auto& b : hd.blocks) fd.top_lowrank += b.k > 0;
            vec += 8.0 * 2.0 * (double)hd.t_size;
        }
        fd.top_bytes64 = 8.0 * (double)vals.size() + vec;
        fd.top_bytes32 = 4.0 * (double)vals.size() + vec;
    }
    fd.top.clear();
    for (const auto& sp : p.spans) {
        TriTopLevel L;
        L.fwd = fd.items + sp.f0;
        L.n_fwd = (int)sp.nf;
        L.bwd = fd.bitems + sp.b0;
        L.n_bwd = (int)sp.nb;
        L.lds_f = sp.lds_f;
        L.lds_b = sp.lds_b;
        L.fcomb = fd.fcomb + sp.cf0;
        L.n_fcomb = (int)sp.ncf;
        L.bcomb = fd.bcomb + sp.cb0;
        L.n_bcomb = (int)sp.ncb;
        L.bwd_nt = p.bwd_wide ? PLAN_BWD_WIDE : 256;
        fd.top.push_back(L);
    }
    fd.fwd_bytes64 = p.fwd_bytes64;
    fd.bwd_bytes64 = p.bwd_bytes64;
    fd.fwd_bytes32 = p.fwd_bytes32;
    fd.bwd_bytes32 = p.bwd_bytes32;
    fd.sub_fwd_bytes64 = p.sub_fwd_bytes64;
    fd.sub_bwd_bytes64 = p.sub_bwd_bytes64;
    fd.sub_fwd_bytes32 = p.sub_fwd_bytes32;
    fd.sub_bwd_bytes32 = p.sub_bwd_bytes32;
    fd.meta_bytes = p.meta_bytes;
    return BIDO_OK;
}

// Work vectors of a factor's sweeps start as NaN (all-ones bits), so that a
// read before a write shows up in every result; entry 0 of the update
// workspace is the 0.0 the sweeps read for a missing child update.
// Device copy of a multigrid hierarchy (Amg): per level the matrix A, the
// prolongation P and R = P^T (FP64 values, and FP32 copies of the values for
// mixed precision), D^-1, the Chebyshev coefficients of the smoother and the
// work vectors of one V-cycle.
struct AmgDev {
    struct Lev {
        int64_t n = 0;
        CsrDev A, P, R;
        float *A32 = nullptr, *P32 = nullptr, *R32 = nullptr;
        double* As64 = nullptr;            // A D^-1 (columns scaled), for the fused smoother
        float* As32 = nullptr;
        int gA = 4, gP = 4, gR = 4;        // lanes per row of the three products
        int steps = 2;                     // Chebyshev steps per smoothing on this level
        double lo = 0.0, hi = 0.0;         // the smoother's interval of D^-1 A
        double* mass = nullptr;            // Galerkin mass part on A's pattern (K_m), or null
        double* dinv = nullptr;
        ChebCoef cf;
        double *b = nullptr, *out = nullptr;   // input and output of this level (levels >= 1)
        double *x = nullptr, *r = nullptr, *d0 = nullptr, *d1 = nullptr, *xp = nullptr;
        // FP32 copies of D^-1 and of the level vectors (the mixed-precision cycle)
        float *dinv32 = nullptr, *b32 = nullptr, *out32 = nullptr, *x32 = nullptr, *r32 = nullptr,
              *xp32 = nullptr;
        int64_t nnz_A = 0, nnz_P = 0, nnz_R = 0;
        template <typename T>
        AmgMat<T> mat(const CsrDev& m, const float* v32, int g) const {
            AmgMat<T> o;
            o.n = m.n;
            o.nnz = m.nnz;
            o.ptr = m.ptr;
            o.col = m.col;
            if constexpr (sizeof(T) == 4) o.val = v32;
            else o.val = m.val;
            o.group = g;
            o.c16 = m.c16;
            o.cb = m.cb;
            return o;
        }
    };
    std::vector<Lev> lv;
    double* cinv = nullptr;
    int64_t nc = 0;
    // the gamma the level matrices hold, and what a refresh needs
    double gamma = 0.0;
    int64_t excluded = -1;
    int lanczos_steps = 20;
    double smooth_ratio = 10.0;
    bool refreshable() const { return !lv.empty() && lv[0].mass; }
    // the mixed-precision cycle keeps FP32 level vectors when no level
    // smooths with more than two Chebyshev steps
    bool fp32_vectors() const {
        for (const Lev& L : lv)
            if (L.steps > 2) return false;
        return true;
    }
    double op_complexity = 1.0, setup_seconds = 0.0;
    bool on() const { return !lv.empty(); }
    // algorithmic bytes of one V-cycle with value bytes w (8 or 4)
    // (level vectors of vb bytes: FP32 in the mixed-precision cycle; the
    // finest level's input and output counted at that width too)
    double bytes(int w) const {
        const double vb = (w == 4 && fp32_vectors()) ? 4.0 : 8.0;
        double b = 8.0 * (double)nc * nc + 2.0 * vb * nc;
        for (size_t l = 0; l + 1 < lv.size(); ++l) {
            const Lev& L = lv[l];
            auto mb = [&](const CsrDev& m, int64_t nnz, int64_t rows) {
                return (m.col_bytes() + w) * nnz + m.row_bytes() * rows + 8.0;
            };
            const double A = mb(L.A, L.nnz_A, L.n), vec = vb * L.n;
            const double A32 = (4.0 + w) * L.nnz_A + 8.0 * (L.n + 1);
            const double nc_l = vb * lv[l + 1].n;
            // two smoothings (one step: b and D^-1 read, z written; the fused first two
            // steps read A D^-1, b and D^-1 and write z, plus r1, d0 and d1 when more
            // steps follow; each further step A + 7 vectors; the post-smoothing also
            // reads the base it adds), two residuals, restriction, prolongation
            const int steps = L.steps;
            const double sm = steps < 2    ? 3.0 * vec
                              : steps == 2 ? A + 3.0 * vec
                                           : A + 6.0 * vec + (steps - 2) * (A32 + 7.0 * vec);
            b += 2.0 * sm + vec + 2.0 * (A + 3.0 * vec) + mb(L.R, L.nnz_R, lv[l + 1].n) + vec + nc_l +
                 mb(L.P, L.nnz_P, L.n) + nc_l + 2.0 * vec;
        }
        return b;
    }
    void release() {
        for (auto& L : lv) {
            for (CsrDev* m : {&L.A, &L.P, &L.R}) {
                hipFree(m->ptr); hipFree(m->col); hipFree(m->val); hipFree(m->c16); hipFree(m->cb);
            }
            for (float* v : {L.A32, L.P32, L.R32, L.As32, L.dinv32, L.b32, L.out32, L.x32, L.r32, L.xp32}) hipFree(v);
            for (double* v : {L.dinv, L.b, L.out, L.x, L.r, L.d0, L.d1, L.xp, L.As64, L.mass}) hipFree(v);
        }
        lv.clear();
        hipFree(cinv);
        cinv = nullptr;
        nc = 0;
    }
};

// lanes per row of a multigrid product: one lane per two to four entries
// of the average row (2 to 64 lanes; the kernels unroll the passes the row
// needs).  Measured on the 128^3 slab against one lane per one or two
// entries (fine-level products 10-15 % faster) and per four to eight
// entries (restriction and coarser levels 5-20 % slower, the finest
// level's A with 2 lanes 20 % slower; the prolongations, ~6 entries per
// row, 6 % faster with 2).
int group_for(const Csr& a) {
    const double avg = a.n > 0 ? (double)a.nnz() / (double)a.n : 0.0;
    return avg <= 8 ? 2 : avg <= 16 ? 4 : avg <= 32 ? 8 : avg <= 64 ? 16 : avg <= 128 ? 32 : 64;
}

// compact: 16-bit column offsets for the matrices whose rows allow them
bido_status upload_amg(const Amg& M, AmgDev& d, bool compact) {
    d.release();
    d.op_complexity = M.op_complexity;
    d.setup_seconds = M.setup_seconds;
    d.gamma = M.gamma;
    d.excluded = M.excluded;
    d.lanczos_steps = M.lanczos_steps;
    d.smooth_ratio = M.smooth_ratio;
    const size_t L = M.levels.size();
    const bool refresh = M.mass.size() == L;   // K_m: a new gamma moves the levels on the device
    d.lv.resize(L);
    for (size_t l = 0; l < L; ++l) {
        const AmgLevel& h = M.levels[l];
        AmgDev::Lev& v = d.lv[l];
        v.n = h.A.n;
        const bool last = l + 1 == L;
        const int64_t n = std::max<int64_t>(v.n, 1);
        if (l > 0) {
            HIP_OK(hipMalloc((void**)&v.b, n * sizeof(double)));
            HIP_OK(hipMalloc((void**)&v.out, n * sizeof(double)));
            HIP_OK(hipMalloc((void**)&v.b32, n * sizeof(float)));
            HIP_OK(hipMalloc((void**)&v.out32, n * sizeof(float)));
        }
        bido_status e;
        if (last) {
            if (refresh) {           // the coarsest matrix, its mass part and the inverse's scratch
                if ((e = CsrHostView::up(h.A, v.A))) return e;
                v.nnz_A = h.A.nnz();
                HIP_OK(upload(&v.mass, M.mass[l].data(), std::max<size_t>(M.mass[l].size(), 1)));
                HIP_OK(hipMalloc((void**)&v.x, n * sizeof(double)));
            }
            break;
        }
        if ((e = CsrHostView::up(h.A, v.A))) return e;
        if ((e = CsrHostView::up(h.P, v.P))) return e;
        if ((e = CsrHostView::up(h.R, v.R))) return e;
        for (auto [hm, dm] : {std::pair<const Csr*, CsrDev*>{&h.A, &v.A}, {&h.P, &v.P}, {&h.R, &v.R}})
            if (compact && (e = CsrHostView::compact(*hm, *dm))) return e;
        auto up32 = [&](const Csr& m, float** dst) -> hipError_t {
            std::vector<float> f(m.val.begin(), m.val.end());
            if (f.empty()) f.push_back(0.0f);
            return upload(dst, f.data(), f.size());
        };
        HIP_OK(up32(h.A, &v.A32));
        HIP_OK(up32(h.P, &v.P32));
        HIP_OK(up32(h.R, &v.R32));
        {
            Csr as = h.A;
            for (int64_t i = 0; i < as.n; ++i)
                for (int64_t p = as.ptr[i]; p < as.ptr[i + 1]; ++p) as.val[p] *= h.dinv[as.col[p]];
            HIP_OK(upload(&v.As64, as.val.data(), std::max<size_t>(as.val.size(), 1)));
            HIP_OK(up32(as, &v.As32));
        }
        v.gA = group_for(h.A);
        v.gP = group_for(h.P);
        v.gR = group_for(h.R);
        v.nnz_A = h.A.nnz();
        v.nnz_P = h.P.nnz();
        v.nnz_R = h.R.nnz();
        HIP_OK(upload(&v.dinv, h.dinv.data(), h.dinv.size()));
        {
            std::vector<float> d32(h.dinv.begin(), h.dinv.end());
            HIP_OK(upload(&v.dinv32, d32.data(), d32.size()));
        }
        v.steps = h.steps;
        v.lo = h.lo;
        v.hi = h.hi;
        v.cf = chebyshev_coefficients(h.lo, h.hi, std::max(2, h.steps));
        if (refresh) HIP_OK(upload(&v.mass, M.mass[l].data(), std::max<size_t>(M.mass[l].size(), 1)));
        for (double** b : {&v.x, &v.r, &v.d0, &v.d1, &v.xp}) HIP_OK(hipMalloc((void**)b, n * sizeof(double)));
        for (float** b : {&v.x32, &v.r32, &v.xp32}) HIP_OK(hipMalloc((void**)b, n * sizeof(float)));
    }
    d.nc = M.levels.back().A.n;
    HIP_OK(upload(&d.cinv, M.coarse_inv.data(), M.coarse_inv.size()));
    return BIDO_OK;
}

hipError_t poison_workspace(const FactorDev& f) {
    hipError_t e = hipMemset(f.ytmp, 0xFF, std::max<int64_t>(f.n, 1) * sizeof(double));
    if (e == hipSuccess) e = hipMemset(f.upd, 0xFF, std::max<int64_t>(f.upd_size, 1) * sizeof(double));
    if (e == hipSuccess) e = hipMemset(f.upd, 0, sizeof(double));
    return e;
}

// Device state of the learned correction (see gnn.h).
struct GnnState {
    float* stat = nullptr;                 // N_H x 16 features, internal v order
    GnnGraph A, At;                        // neighbour weights and their transpose
    GnnGraph Wk;                           // K_m / mean diag: norm of the training loss
    float *theta = nullptr, *m = nullptr, *v = nullptr, *grad = nullptr;
    float* theta_best = nullptr;           // the kept weights of a stencil training
    uint16_t* wbf = nullptr;               // BF16 working weights
    GnnAct act;
    float* partials = nullptr;
    double* dloss = nullptr;
    float *ft = nullptr, *fy = nullptr;    // check-entry buffers (internal order)
    double* tz = nullptr;
    // training samples: t/|t| and target/|t| (FP32), |t|^2 (FP64)
    int max_samples = 0, n_samples = 0;
    float *s_t = nullptr, *s_y = nullptr;
    double* s_tn2 = nullptr;
    double* pend = nullptr;                // V_k + Z2_k of the running solve
    int max_pending = 64, n_pending = 0;
    bool collecting = false;
    int adam_step = 0;
    float out_scale = 1.0f;                // output unit: RMS of the training targets
    // learned Schur-complement stencil (K_m + C)
    StencilPattern P;
    StencilKm K;
    double dbar = 1.0;                     // mean diagonal of K_m
    float *cval = nullptr, *G = nullptr, *r = nullptr;
    float *s_z = nullptr, *s_b = nullptr;  // samples z*/rms and (t - K_m z*)/(dbar rms)
    double *s_zz = nullptr;
    double *pend_t = nullptr, *pend_v = nullptr;
    bool stencil_ready = false;
    bool wk_like_k = false;                // Wk stores K_m's pattern in K_m's order
    // pairs from consecutive steps instead of PCG iterates (an inexact P_1):
    // K (V^{n+1} - V^n) = Y_2^n - Y_2^{n-1}, exact whatever the inner solves
    bool increments = false, inc_ok = false;
    double *inc_v = nullptr, *inc_y = nullptr;
    void release() {
        for (void* b : {(void*)stat, (void*)A.ptr, (void*)A.col, (void*)A.val, (void*)At.ptr, (void*)At.col,
                        (void*)At.val, (void*)Wk.ptr, (void*)Wk.col, (void*)Wk.val, (void*)act.res,
                        (void*)act.zero, (void*)theta, (void*)theta_best, (void*)m, (void*)v, (void*)grad,
                        (void*)wbf,
                        (void*)act.f, (void*)act.m0, (void*)act.h1, (void*)act.m1, (void*)act.h2,
                        (void*)act.o, (void*)act.dout, (void*)act.dz2, (void*)act.g2, (void*)act.dz1,
                        (void*)partials, (void*)dloss, (void*)ft, (void*)fy, (void*)tz, (void*)s_t,
                        (void*)s_y, (void*)s_tn2, (void*)pend, (void*)inc_v, (void*)inc_y, (void*)P.ptr,
                        (void*)P.col, (void*)P.row, (void*)P.tpos, (void*)K.ptr, (void*)K.col, (void*)K.val,
                        (void*)cval, (void*)G, (void*)r, (void*)s_z, (void*)s_b, (void*)s_zz, (void*)pend_t,
                        (void*)pend_v})
            hipFree(b);
        *this = GnnState();
    }
};

}  // namespace

void release_lam_blk(LamBlk& b) {
    hipFree(b.ptr); hipFree(b.col); hipFree(b.val); hipFree(b.gm); hipFree(b.c16); hipFree(b.cb);
    b = LamBlk();
}

bido_status upload_lam_blk(const HostSetup& hs, LamBlk& b, bool compact) {
    release_lam_blk(b);
    const LamBlocked& h = hs.lamb;
    if (h.n == 0) return BIDO_OK;
    HIP_OK(upload(&b.ptr, h.ptr.data(), h.ptr.size()));
    HIP_OK(upload(&b.col, h.col.data(), h.col.size()));
    HIP_OK(upload(&b.val, h.val.data(), h.val.size()));
    HIP_OK(upload(&b.gm, h.gm.data(), h.gm.size()));
    b.npos = (int64_t)h.col.size();
    b.n = h.n;
    if (compact) {              // 16-bit offsets when every row's positions allow them
        Csr pat;
        pat.n = h.n;
        pat.ptr = h.ptr;
        pat.col = h.col;
        CsrDev d;
        if (bido_status e = CsrHostView::compact(pat, d)) return e;
        b.c16 = d.c16;
        b.cb = d.cb;
    }
    return BIDO_OK;
}

struct bido_ctx {
    hipStream_t stream = nullptr;
    int device = 0;
    HostSetup hs;
    bido_params params{};
    int64_t N = 0, NH = 0, n2 = 0;
    int spmv_group = 8;
    int precision = BIDO_PREC_FP64;
    CsrDev lam, avu, auv;
    FactorDev p1, pk;
    double *x = nullptr, *r = nullptr, *z = nullptr, *p = nullptr, *q = nullptr, *Y = nullptr;
    double *tA = nullptr, *tB = nullptr, *tC = nullptr, *tD = nullptr, *r_old = nullptr;
    double* sc = nullptr;        // scalar slots, then the PCG partial regions
    double* sc_host = nullptr;   // pinned
    unsigned nb_rz = 0;          // partials of r.z written by the latest apply
    bool batched = false;        // owned by a bido_batch (runs on its stream)
    bido_batch* batch = nullptr; // that batch
    // HIP graphs of one PCG iteration's launch sequence (preconditioner apply,
    // direction update, SpMV, PCG update, scalar copy): [0] the first
    // iteration, [1] and [2] the later ones by the slot of r.z they read
    hipStream_t work = nullptr;  // capturable stream for bido_run
    hipEvent_t ev_in = nullptr, ev_out = nullptr;
    int graph_mode = -1;         // 1 on, 0 off, -1 only inside a batch
    hipGraphExec_t gx[3] = {nullptr, nullptr, nullptr};
    unsigned gx_nb[3] = {0, 0, 0}, gx_nbrz[3] = {0, 0, 0};
    const void* gx_key[4] = {nullptr, nullptr, nullptr, nullptr};
    void drop_graphs() {
        for (auto& g : gx)
            if (g) { hipGraphExecDestroy(g); g = nullptr; }
    }
    Reduce rd;
    int64_t *u_pos = nullptr, *v_pos = nullptr;
    double *m_int = nullptr, *mh_loc = nullptr, *stim_loc = nullptr;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    std::vector<int64_t> heart_ids;
    Profiler prof;
    GnnState gnn;
    FactorDev pk_learned;             // factor of K_m + C (learned stencil)
    std::unique_ptr<Factor> pk_learned_host;   // its host factor (a fused batch merges it)
    AmgDev amg1, amgk;                // multigrid P_1 / P_K (inner_p1 / inner_pk = AMG)
    LamBlk lamb;                      // blocked Lambda (heart = whole mesh, one order)
    int64_t* lam_vdiag = nullptr;     // positions of the v-v diagonal in Lambda's values
    float *avu32 = nullptr, *auv32 = nullptr;   // FP32 values of S_i Pi, Pi^T S_i (mixed precision)
    AmgDev amgk_learned;              // multigrid of K_m + C (learned stencil with a multigrid P_K)
    int precond = BIDO_PRECOND_PLAIN;
    int fallbacks = 0;
    // P_K ~ K_m: the factor `pk`, or Chebyshev-accelerated Jacobi on K_m
    int pk_kind = BIDO_PK_CHOLESKY;
    int cheb_steps = 0;
    double cheb_lo = 0.0, cheb_hi = 0.0;
    bool cheb_auto = false;           // interval estimated by the library
    ChebCoef cheb;
    CsrDev km;                        // K_m, internal v order (uploaded on first use)
    double *km_dinv = nullptr, *ch_r = nullptr, *ch_d[2] = {nullptr, nullptr};
    double* vs = nullptr;             // Strang splitting: V* after the first reaction half-step
    // recording of the steps (bido_record): activation times, probe rows
    int64_t step_n = 0;               // index of the step in progress
    // projected initial guess: a ring of params.guess_states states (the
    // ones the last steps started from) and their Lambda images, gw[g_head]
    // the state of step g_n and g_len consecutive ones; their Gram matrix
    // (by slot), dot and coefficient scratch, and the reduction of the dots
    double* gw[GUESS_MAX] = {};
    double* gaw[GUESS_MAX] = {};
    double *gG = nullptr, *gd = nullptr, *gb = nullptr, *gc = nullptr;
    Reduce grd;
    int g_head = 0, g_len = 0;
    int64_t g_n = -2;
    struct Recording {
        bool on = false;
        double v_act = 0.0;
        bool act_on = false;
        double* act = nullptr;        // N_H, heart-local order; < 0: not reached
        int np = 0, nv = 0;
        int64_t* ids = nullptr;       // np x nv vertex ids (caller's numbering)
        double* wts = nullptr;        // np x nv barycentric weights
        double* rows = nullptr;       // max_steps x np
        int64_t max_steps = 0, n_rows = 0;
        void release() {
            hipFree(act);
            hipFree(ids);
            hipFree(wts);
            hipFree(rows);
            *this = Recording();
        }
    } rec;

    ~bido_ctx() {
        if (stream) hipStreamSynchronize(stream);
        p1.release();
        pk.release();
        pk_learned.release();
        amg1.release();
        amgk.release();
        amgk_learned.release();
        gnn.release();
        rec.release();
        CsrHostView::release(lam);
        release_lam_blk(lamb);
        hipFree(lam_vdiag);
        hipFree(avu32);
        hipFree(auv32);
        CsrHostView::release(avu);
        CsrHostView::release(auv);
        CsrHostView::release(km);
        for (double* b : gw) hipFree(b);
        for (double* b : gaw) hipFree(b);
        hipFree(gG);
        hipFree(gd);
        hipFree(grd.partials);
        hipFree(grd.counter);
        for (double* b : {x, r, z, p, q, Y, tA, tB, tC, tD, r_old, sc, m_int, mh_loc, stim_loc, km_dinv, ch_r,
                          ch_d[0], ch_d[1], vs})
            hipFree(b);
        hipFree(rd.partials);
        hipFree(rd.counter);
        hipFree(u_pos);
        hipFree(v_pos);
        if (sc_host) hipHostFree(sc_host);
        if (ev0) hipEventDestroy(ev0);
        if (ev1) hipEventDestroy(ev1);
        drop_graphs();
        if (ev_in) hipEventDestroy(ev_in);
        if (ev_out) hipEventDestroy(ev_out);
        if (work) hipStreamDestroy(work);
    }
};

namespace {

// Launch `stmt`, bracketed by profiler events when profiling is on.
#define PROF(c, cls, bytes, stmt)                                                \
    do {                                                                         \
        if ((c)->prof.on) {                                                      \
            hipEvent_t a_ = (c)->prof.get(), b_ = (c)->prof.get();               \
            hipEventRecord(a_, (c)->stream);                                     \
            stmt;                                                                \
            hipEventRecord(b_, (c)->stream);                                     \
            (c)->prof.recs.push_back({(cls), a_, b_, (double)(bytes)});          \
        } else {                                                                 \
            stmt;                                                                \
        }                                                                        \
    } while (0)

// Aggregate a profiler's records by kernel class into out[0..cap) (after
// the stream has drained) and clear them.
bido_status profile_aggregate(Profiler& P, bido_kprof* out, int cap, int* n) {
    bido_kprof agg[K_NCLASS];
    std::memset(agg, 0, sizeof(agg));
    for (int k = 0; k < K_NCLASS; ++k) std::strncpy(agg[k].name, kclass_name[k], sizeof(agg[k].name) - 1);
    for (const auto& r : P.recs) {
        float ms = 0.f;
        HIP_OK(hipEventElapsedTime(&ms, r.a, r.b));
        agg[r.cls].launches += 1;
        agg[r.cls].ms += ms;
        agg[r.cls].bytes += r.bytes;
    }
    int m = 0;
    for (int k = 0; k < K_NCLASS; ++k)
        if (agg[k].launches > 0) {
            if (out && m < cap) out[m] = agg[k];
            ++m;
        }
    *n = m;
    P.recs.clear();
    P.used = 0;
    return BIDO_OK;
}

double csr_bytes(const CsrDev& a, int64_t ncols_read) {
    return 12.0 * a.nnz + 8.0 * (a.n + 1) + 8.0 * ncols_read + 8.0 * a.n;
}
// blocked Lambda product: positions (4 + 16 bytes), row pointers, gm, x (u
// and v), the output (u and v), and y in mode 1
double blk_bytes(const LamBlk& b, int mode) {
    const double colb = b.c16 ? 2.0 : 4.0, rowb = b.c16 ? 12.0 : 8.0;
    return (16.0 + colb) * b.npos + rowb * b.n + 8.0 + 8.0 * b.n + 32.0 * b.n + (mode == 1 ? 16.0 * b.n : 0.0);
}

template <typename T> const T* top_inv(const FactorDev& f);
template <> const double* top_inv<double>(const FactorDev& f) { return f.top_inv64; }
template <> const float* top_inv<float>(const FactorDev& f) { return f.top_inv32; }

// C: a context or a fused batch (stream, profiler, precision)
template <typename T, typename C>
void tri_solve(C* c, const FactorDev& f, const T* panel, const T* panel_cm, const double* in, double* out) {
    hipStream_t s = c->stream;
    const bool f32 = sizeof(T) == 4;
    PROF(c, K_TRI_FWD_SUB, f32 ? f.sub_fwd_bytes32 : f.sub_fwd_bytes64,
         launch_tri_fwd_sub<T>(s, f.plan, f.nodes, panel_cm, f.ea, in, f.ytmp, f.upd));
    for (size_t k = 0; k < f.top.size(); ++k) {
        const int h = f.lvl0 + (int)k;
        PROF(c, K_TRI_FWD_LVL, f32 ? f.fwd_bytes32[h] : f.fwd_bytes64[h],
             launch_tri_fwd_lvl<T>(s, f.top[k], f.plan, f.nodes, panel_cm, f.ea, in, f.ytmp, f.upd));
    }
    PROF(c, K_TRI_TOP, f32 ? f.top_bytes32 : f.top_bytes64,
         launch_tri_top<T>(s, f.plan, top_inv<T>(f), in, f.upd, out));
    for (size_t k = f.top.size(); k-- > 0;) {
        const int h = f.lvl0 + (int)k;
        PROF(c, K_TRI_BWD_LVL, f32 ? f.bwd_bytes32[h] : f.bwd_bytes64[h],
             launch_tri_bwd_lvl<T>(s, f.top[k], f.plan, f.nodes, panel, f.bidx, f.ytmp, out));
    }
    PROF(c, K_TRI_BWD_SUB, f32 ? f.sub_bwd_bytes32 : f.sub_bwd_bytes64,
         launch_tri_bwd_sub<T>(s, f.plan, f.nodes, panel, f.bidx, f.ytmp, out));
}

template <typename C>
void inner_solve(C* c, const FactorDev& f, const double* in, double* out) {
    if (c->precision == BIDO_PREC_MIXED && f.panel32)
        tri_solve<float>(c, f, f.panel32, f.panel32_cm, in, out);
    else
        tri_solve<double>(c, f, f.panel64, f.panel64_cm, in, out);
}

// The level vectors of a cycle in type V: FP64 ones, or the FP32 copies
// of the mixed-precision cycle.
template <typename V>
struct LevVecs {
    V *b, *out, *x, *r, *xp, *d0, *d1;
    const V* dinv;
};
inline LevVecs<double> lev_vecs(const AmgDev::Lev& L, double*) { return {L.b, L.out, L.x, L.r, L.xp, L.d0, L.d1, L.dinv}; }
inline LevVecs<float> lev_vecs(const AmgDev::Lev& L, float*) {
    return {L.b32, L.out32, L.x32, L.r32, L.xp32, nullptr, nullptr, L.dinv32};
}

// z = S b for level L of a multigrid hierarchy: the Chebyshev steps of the
// smoother from z = 0 (the recurrence of the Chebyshev P_K on the level's
// interval of D^-1 A; the first two steps in one fused pass).  V: the level
// vectors; BT, ZT: the input and output (FP64 on the finest level).  More
// than two steps run on FP64 level vectors only.
template <typename T, typename V, typename BT, typename ZT, typename C>
void amg_smooth(C* c, const AmgDev& M, const AmgDev::Lev& L, const BT* b, ZT* z, int cls,
                const V* base = nullptr) {
    hipStream_t s = c->stream;
    const int64_t n = L.n;
    const LevVecs<V> lv = lev_vecs(L, (V*)nullptr);
    const AmgMat<T> A = L.mat<T>(L.A, L.A32, L.gA);
    AmgMat<T> As = A;                      // the column-scaled copy A D^-1
    if constexpr (sizeof(T) == 4) As.val = L.As32;
    else As.val = L.As64;
    const double Ab = (L.A.col_bytes() + sizeof(T)) * L.nnz_A + L.A.row_bytes() * n + 8.0;
    const double Ab32 = (4.0 + sizeof(T)) * L.nnz_A + 8.0 * (n + 1);   // the further steps read col
    // b and D^-1 read, z written, and the base added
    const double vb = (sizeof(BT) + sizeof(V) + sizeof(ZT)) * (double)n + (base ? sizeof(V) * (double)n : 0.0);
    if (L.steps < 2) {
        PROF(c, cls, vb, (launch_amg_jacobi<BT, V, ZT>(s, n, b, lv.dinv, L.cf.inv_theta, base, z)));
        return;
    }
    const bool more = L.steps > 2;
    PROF(c, cls, Ab + vb + (more ? 3.0 * sizeof(V) * n : 0.0),
         (launch_amg_smooth2<T, BT, V, ZT>(s, As, lv.dinv, b, L.cf.inv_theta, L.cf.c1[0], L.cf.c2[0], base, z,
                                           lv.r, lv.d0, lv.d1, more)));
    if constexpr (std::is_same<V, double>::value && std::is_same<ZT, double>::value) {
        double* d[2] = {L.d0, L.d1};
        for (int k = 2; k < L.steps; ++k)
            PROF(c, cls, Ab32 + 56.0 * n,
                 launch_amg_cheb<T>(s, A, L.dinv, L.r, d[(k - 1) & 1], d[k & 1], z, L.cf.c1[k - 1], L.cf.c2[k - 1]));
    }
}

// out = B b: the symmetric V-cycle from level l (pre-smoothing, residual,
// restriction, the coarser cycle, prolongation, residual, post-smoothing;
// the coarsest level by its dense inverse).  V: the level vectors; BT, OT:
// the cycle's input and output (FP64 on the finest level, V below).
template <typename T, typename V, typename BT, typename OT, typename C>
void amg_vcycle_t(C* c, const AmgDev& M, size_t l, const BT* b, OT* out) {
    hipStream_t s = c->stream;
    const AmgDev::Lev& L = M.lv[l];
    if (l + 1 == M.lv.size()) {
        if constexpr (std::is_same<BT, OT>::value)
            PROF(c, K_AMG_COARSE, 8.0 * (double)M.nc * M.nc + 2.0 * sizeof(BT) * M.nc,
                 launch_dense_gemv<BT>(s, M.nc, M.cinv, b, out));
        return;
    }
    const AmgDev::Lev& Lc = M.lv[l + 1];
    const LevVecs<V> lv = lev_vecs(L, (V*)nullptr), lc = lev_vecs(Lc, (V*)nullptr);
    const double vec = (double)sizeof(V) * L.n, bvec = (double)sizeof(BT) * L.n, w = sizeof(T);
    const double cvec = (double)sizeof(V) * Lc.n;
    const AmgMat<T> A = L.mat<T>(L.A, L.A32, L.gA);
    const AmgMat<T> P = L.mat<T>(L.P, L.P32, L.gP);
    const AmgMat<T> R = L.mat<T>(L.R, L.R32, L.gR);
    // values and columns per entry, row pointers (and column bases) per row
    const double Ab = (w + L.A.col_bytes()) * L.nnz_A + L.A.row_bytes() * L.n,
                 Pb = (w + L.P.col_bytes()) * L.nnz_P + L.P.row_bytes() * L.n,
                 Rb = (w + L.R.col_bytes()) * L.nnz_R + L.R.row_bytes() * Lc.n;
    // profiler classes: the finest level by kernel (its smoother is one
    // kernel on one matrix), the coarser levels together
    const bool fine = l == 0;
    const int c_sm = fine ? K_AMG_SMOOTH : K_AMG_COARSE, c_re = fine ? K_AMG_SPMV : K_AMG_COARSE,
              c_tr = fine ? K_AMG_TRANSFER : K_AMG_COARSE;
    amg_smooth<T, V, BT, V>(c, M, L, b, lv.x, c_sm);
    PROF(c, c_re, Ab + 2 * vec + bvec, (launch_amg_spmv<T, V, BT, V>(s, A, lv.x, b, -1.0, lv.r)));  // r = b - A x
    PROF(c, c_tr, Rb + vec + cvec, (launch_amg_spmv<T, V, V, V>(s, R, lv.r, (const V*)nullptr, 1.0, lc.b)));
    amg_vcycle_t<T, V, V, V>(c, M, l + 1, (const V*)lc.b, lc.out);
    PROF(c, c_tr, Pb + cvec + 2 * vec, (launch_amg_spmv<T, V, V, V>(s, P, lc.out, lv.x, 1.0, lv.xp)));  // xp = x + P e
    PROF(c, c_re, Ab + 2 * vec + bvec, (launch_amg_spmv<T, V, BT, V>(s, A, lv.xp, b, -1.0, lv.r)));  // r = b - A xp
    amg_smooth<T, V, V, OT>(c, M, L, (const V*)lv.r, out, c_sm, (const V*)lv.xp);                // out = xp + S r
}

// The cycle with FP32 level values and vectors in mixed precision (FP64
// level vectors when a level smooths with more than two steps), FP64
// otherwise; the input and output stay FP64.
template <typename C>
void amg_vcycle(C* c, const AmgDev& M, size_t l, const double* b, double* out, bool fp64 = false) {
    if (c->precision == BIDO_PREC_MIXED && !fp64) {
        if (M.fp32_vectors()) amg_vcycle_t<float, float, double, double>(c, M, l, b, out);
        else amg_vcycle_t<float, double, double, double>(c, M, l, b, out);
    } else {
        amg_vcycle_t<double, double, double, double>(c, M, l, b, out);
    }
}

// Z1 = P_1^-1 r1: the factor's sweeps, or the multigrid V-cycle.
template <typename C>
void p1_solve(C* c, const double* in, double* out) {
    if (c->amg1.on()) amg_vcycle(c, c->amg1, 0, in, out);
    else inner_solve(c, c->p1, in, out);
}

// Z2 = P_K^-1 t: the factor of K_m, the multigrid V-cycle, or `cheb_steps`
// steps of the Chebyshev acceleration of the Jacobi iteration on K_m
// (always FP64; z_0 = 0).
void pk_solve(bido_ctx* c, const double* in, double* out, double* ch_r, double* ch_d0, double* ch_d1);
void pk_solve(bido_ctx* c, const double* in, double* out) {
    pk_solve(c, in, out, c->ch_r, c->ch_d[0], c->ch_d[1]);
}
void pk_solve(bido_ctx* c, const double* in, double* out, double* ch_r, double* ch_d0, double* ch_d1) {
    if (c->pk_kind == BIDO_PK_AMG) {
        amg_vcycle(c, c->amgk, 0, in, out);
        return;
    }
    if (c->pk_kind != BIDO_PK_CHEBYSHEV) {
        inner_solve(c, c->pk, in, out);
        return;
    }
    double* ch_d[2] = {ch_d0, ch_d1};
    hipStream_t s = c->stream;
    const int64_t n = c->NH;
    const double step_bytes = 12.0 * c->km.nnz + 8.0 * (n + 1) + 8.0 * 8 * n;
    PROF(c, K_CHEB, 32.0 * n, launch_cheb_init(s, n, in, c->km_dinv, c->cheb.inv_theta, ch_d[0], out));
    for (int k = 1; k < c->cheb_steps; ++k) {
        const bool last = k + 1 == c->cheb_steps;
        PROF(c, K_CHEB, last ? step_bytes - 16.0 * n : step_bytes,
             launch_cheb_step(s, c->km, c->spmv_group, c->km_dinv, k == 1 ? in : ch_r, ch_r,
                              ch_d[(k - 1) & 1], ch_d[k & 1], out, c->cheb.c1[k - 1], c->cheb.c2[k - 1],
                              last));
    }
}

// Opt-in check (environment BIDO_DEBUG=1): report the first non-finite
// intermediate vector of a preconditioner apply on stderr.
bool debug_on() {
    static int on = -1;
    if (on < 0) {
        const char* e = std::getenv("BIDO_DEBUG");
        on = (e && e[0] == '1') ? 1 : 0;
    }
    return on == 1;
}
void debug_check(bido_ctx* c, const char* name, const double* v, int64_t n) {
    if (!debug_on()) return;
    std::vector<double> h(n);
    hipStreamSynchronize(c->stream);
    hipMemcpy(h.data(), v, n * sizeof(double), hipMemcpyDeviceToHost);
    int64_t bad = 0, first = -1;
    double mx = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        if (!std::isfinite(h[i])) { if (first < 0) first = i; ++bad; }
        else mx = std::max(mx, std::fabs(h[i]));
    }
    std::fprintf(stderr, "[bido debug] %-6s n=%lld nonfinite=%lld first=%lld max|.|=%.3e\n", name,
                 (long long)n, (long long)bad, (long long)first, mx);
}

// y = b + sign * B x for a coupling block B (S_i Pi or Pi^T S_i) on the
// multigrid products' kernels (row groups sized to the average row): FP32
// values in mixed precision, where the block only feeds the preconditioner
void coupling_product(bido_ctx* c, const CsrDev& B, const float* v32, const double* x, const double* b,
                      double sign, double* y) {
    const int64_t avg = B.n > 0 ? (B.nnz + B.n - 1) / B.n : 1;
    const int g = avg <= 16 ? 4 : avg <= 32 ? 8 : avg <= 64 ? 16 : 32;
    const bool f32 = c->precision == BIDO_PREC_MIXED;
    const double bytes = (B.col_bytes() + (f32 ? 4.0 : 8.0)) * B.nnz + B.row_bytes() * B.n + 8.0 +
                         8.0 * B.n * (b ? 2 : 1) + 8.0 * (B.nnz > 0 ? B.n : 0);
    if (f32) {
        AmgMat<float> m{B.n, B.nnz, B.ptr, B.col, v32, g, B.c16, B.cb};
        PROF(c, K_SPMV_CSR, bytes, launch_amg_spmv<float>(c->stream, m, x, b, sign, y));
    } else {
        AmgMat<double> m{B.n, B.nnz, B.ptr, B.col, B.val, g, B.c16, B.cb};
        PROF(c, K_SPMV_CSR, bytes, launch_amg_spmv<double>(c->stream, m, x, b, sign, y));
    }
}

// z = P_Lambda^-1 r  and  rho_new = r.z  (plus z.r_old for flexible CG).
// learned: add the network's correction to Z2 (Schur-complement block);
// collecting: record (t, V_k + Z2_k) for training targets.
void precond_apply(bido_ctx* c, const double* r, double* z, const double* r_old, bool learned,
                   bool stencil = false) {
    hipStream_t s = c->stream;
    const int64_t N = c->N, NH = c->NH;
    GnnState& g = c->gnn;
    debug_check(c, "r", r, c->n2);
    p1_solve(c, r, c->tA);                                           // Z1 = P1^-1 R1
    debug_check(c, "Z1", c->tA, N);
    coupling_product(c, c->avu, c->avu32, c->tA, r + N, -1.0, c->tB);     // R2 - S_i Pi Z1
    debug_check(c, "t", c->tB, c->NH);
    if (stencil && c->amgk_learned.on()) amg_vcycle(c, c->amgk_learned, 0, c->tB, z + N);
    else if (stencil) inner_solve(c, c->pk_learned, c->tB, z + N);   // Z2 = PK^-1 (...)
    else pk_solve(c, c->tB, z + N);
    debug_check(c, "Z2", z + N, c->NH);
    if (g.collecting && !g.increments && g.n_samples + g.n_pending < g.max_samples &&
        g.n_pending < g.max_pending) {
        const int k = g.n_samples + g.n_pending;
        launch_dot_reduce(s, NH, c->tB, c->tB, c->rd, g.s_tn2 + k);
        launch_gnn_store_sample(s, NH, c->tB, g.s_tn2 + k, g.s_t + (int64_t)k * NH);
        launch_gnn_pending(s, NH, c->x + N, z + N, g.pend + (int64_t)g.n_pending * NH);
        hipMemcpyAsync(g.pend_t + (int64_t)g.n_pending * NH, c->tB, NH * sizeof(double),
                       hipMemcpyDeviceToDevice, s);
        hipMemcpyAsync(g.pend_v + (int64_t)g.n_pending * NH, c->x + N, NH * sizeof(double),
                       hipMemcpyDeviceToDevice, s);
        ++g.n_pending;
    }
    if (learned) {
        PROF(c, K_MISC, 16.0 * NH, launch_dot_reduce(s, NH, c->tB, c->tB, c->rd, c->sc + S_TN2));
        PROF(c, K_GNN, 200.0 * NH,
             launch_gnn_forward(s, NH, c->tB, c->sc + S_TN2, g.stat, g.A, g.wbf, g.act, 0, z + N,
                                g.out_scale));
    }
    coupling_product(c, c->auv, c->auv32, z + N, nullptr, 1.0, c->tC);     // Pi^T S_i Z2
    debug_check(c, "PiSZ2", c->tC, N);
    p1_solve(c, c->tC, c->tD);                                       // P1^-1 Pi^T S_i Z2
    debug_check(c, "W", c->tD, N);
    PROF(c, K_COMBINE_DOT, 8.0 * (3 * N + c->NH + c->n2 * (r_old ? 2 : 1)),
         c->nb_rz = launch_combine_dot(s, N, c->n2, z, c->tA, c->tD, r, r_old, c->sc));
}

// Copy the scalar slots and the partial regions below `regions` to the host.
bido_status read_scalars(bido_ctx* c, int regions = 0) {
    HIP_OK(hipMemcpyAsync(c->sc_host, c->sc, pp_offset(regions) * sizeof(double), hipMemcpyDeviceToHost,
                          c->stream));
    HIP_OK(hipStreamSynchronize(c->stream));
    return BIDO_OK;
}
double host_partials(const bido_ctx* c, int region, unsigned nb) {
    double s = 0.0;
    for (unsigned b = 0; b < nb; ++b) s += c->sc_host[pp_offset(region) + b];
    return s;
}

// PCG on the internal vectors: x (initial guess in, solution out), Y, run as
// a sequence of phases so that a batch of contexts can advance in lockstep.
// Each phase ends with an asynchronous copy of the scalar slots and the
// partials the host needs; pcg_advance runs once that copy has landed.
// With a nonlinear or inexact preconditioner (learned correction, mixed
// precision) the direction update is the flexible (Polak-Ribiere) one.  A
// learned additive apply that is not a descent direction (r.z <= 0) is redone
// without the correction and counted as a fallback.
struct PcgRun {
    double tol = 0.0, yy = 0.0, rel = 0.0;
    int it = 0;                 // completed updates x += alpha p
    int rho = S_RHO;            // slot of r.z of the current direction
    int fallbacks = 0;
    unsigned nb = 0;            // partials written by the latest reduction
    bool learned = false, stencil = false, flexible = false;
    bool started = false, done = false, conv = false;
    double* r_old = nullptr;
    bido_status status = BIDO_OK;
    std::string err;
};

void copy_scalars_async(bido_ctx* c, int regions) {
    hipMemcpyAsync(c->sc_host, c->sc, pp_offset(regions) * sizeof(double), hipMemcpyDeviceToHost, c->stream);
}

bido_status pcg_apply(bido_ctx* c, PcgRun& ps, const double* ro) {
    precond_apply(c, c->r, c->z, ro, ps.learned, ps.stencil);
    if (!ps.learned) return BIDO_OK;
    bido_status e = read_scalars(c, PP_RZ + 1);
    if (e) return e;
    const double rz = host_partials(c, PP_RZ, c->nb_rz);
    if (!(rz > 0.0) || !std::isfinite(rz)) {
        ++ps.fallbacks;
        precond_apply(c, c->r, c->z, ro, false, false);
    }
    return BIDO_OK;
}

// q = Lambda p, x += alpha p, r -= alpha q; copy |r|^2 partials and p.q
void pcg_tail(bido_ctx* c, PcgRun& ps) {
    hipStream_t s = c->stream;
    const int64_t n = c->n2;
    unsigned nb = 0;
    if (c->lamb.on())
        PROF(c, K_SPMV_LAMBDA, blk_bytes(c->lamb, 0),
             nb = launch_spmv_lam_blk(s, c->lamb, c->spmv_group, 0, c->p, nullptr, c->q, c->sc));
    else
        PROF(c, K_SPMV_LAMBDA, csr_bytes(c->lam, n),
             nb = launch_spmv_lambda(s, c->lam, c->spmv_group, 0, c->p, nullptr, c->q, c->sc));
    PROF(c, K_PCG_UPDATE, (ps.r_old ? 56.0 : 48.0) * n,
         ps.nb = launch_pcg_update(s, n, c->x, c->r, ps.r_old, c->p, c->q, c->sc, nb, ps.rho));
    copy_scalars_async(c, PP_RR + 1);
}

// r0 = Y - Lambda x0; copy |r|^2 and |Y|^2 partials
void pcg_start(bido_ctx* c, PcgRun& ps, double tol) {
    ps = PcgRun();
    ps.tol = tol;
    ps.learned = c->precond == BIDO_PRECOND_LEARNED_ADDITIVE && !c->gnn.collecting;
    ps.stencil = c->precond == BIDO_PRECOND_LEARNED && !c->gnn.collecting && c->gnn.stencil_ready;
    ps.flexible = c->precision == BIDO_PREC_MIXED || ps.learned || ps.stencil;
    ps.r_old = ps.flexible ? c->r_old : nullptr;
    const int64_t n = c->n2;
    if (c->lamb.on())
        PROF(c, K_SPMV_LAMBDA, blk_bytes(c->lamb, 1),
             ps.nb = launch_spmv_lam_blk(c->stream, c->lamb, c->spmv_group, 1, c->x, c->Y, c->r, c->sc));
    else
        PROF(c, K_SPMV_LAMBDA, csr_bytes(c->lam, n) + 8.0 * n,
             ps.nb = launch_spmv_lambda(c->stream, c->lam, c->spmv_group, 1, c->x, c->Y, c->r, c->sc));
    copy_scalars_async(c, PP_YY + 1);
}

// The launch sequences between two host checks: the first iteration (apply
// to r0, p = z, update) and a later one (apply, direction update, update).
void seq_first(bido_ctx* c, PcgRun& ps) {
    const int64_t n = c->n2;
    pcg_apply(c, ps, nullptr);
    PROF(c, K_P_UPDATE, 24.0 * n, launch_p_update(c->stream, n, c->z, c->p, c->sc, c->nb_rz, 1, 0, ps.rho, ps.rho));
    ps.it = 1;
    pcg_tail(c, ps);
}
void seq_iter(bido_ctx* c, PcgRun& ps) {
    const int64_t n = c->n2;
    pcg_apply(c, ps, ps.r_old);
    // r.z alternates between two slots, so that the direction update never
    // overwrites the value its other blocks read
    const int next = ps.rho == S_RHO ? S_RHO_NEW : S_RHO;
    PROF(c, K_P_UPDATE, 24.0 * n,
         launch_p_update(c->stream, n, c->z, c->p, c->sc, c->nb_rz, 0, ps.flexible ? 1 : 0, ps.rho, next));
    ps.rho = next;
    ++ps.it;
    pcg_tail(c, ps);
}

// Replay (capturing it first if needed) the graph of a sequence.  Returns
// false when the sequence has to run eagerly: graphs off, profiling, sample
// collection or the additive learned mode (host checks inside the apply),
// or a stream that cannot be captured.
bool seq_graph(bido_ctx* c, PcgRun& ps, int variant) {
    const bool on = c->graph_mode > 0 || (c->graph_mode < 0 && c->batched);
    if (!on || c->prof.on || c->gnn.collecting || ps.learned || !c->stream || debug_on()) return false;
    const void* key[4] = {(const void*)(intptr_t)(c->precision + 1), (const void*)(intptr_t)(ps.stencil ? 2 : 1),
                          c->amgk_learned.on() ? (const void*)c->amgk_learned.cinv : (const void*)c->pk_learned.nodes,
                          ps.r_old};
    if (!std::equal(key, key + 4, c->gx_key)) {
        c->drop_graphs();
        std::copy(key, key + 4, c->gx_key);
    }
    if (!c->gx[variant]) {
        PcgRun tmp = ps;
        if (hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal) != hipSuccess) {
            (void)hipGetLastError();
            c->graph_mode = 0;
            return false;
        }
        if (variant == 0) seq_first(c, tmp); else seq_iter(c, tmp);
        hipGraph_t g = nullptr;
        hipError_t e1 = hipStreamEndCapture(c->stream, &g);
        hipGraphExec_t x = nullptr;
        hipError_t e2 = e1 == hipSuccess ? hipGraphInstantiate(&x, g, nullptr, nullptr, 0) : e1;
        if (g) hipGraphDestroy(g);
        if (e2 != hipSuccess) {
            (void)hipGetLastError();
            c->graph_mode = 0;
            return false;
        }
        c->gx[variant] = x;
        c->gx_nb[variant] = tmp.nb;
        c->gx_nbrz[variant] = c->nb_rz;
    }
    if (hipGraphLaunch(c->gx[variant], c->stream) != hipSuccess) {
        (void)hipGetLastError();
        c->drop_graphs();
        c->graph_mode = 0;
        return false;
    }
    ps.nb = c->gx_nb[variant];
    c->nb_rz = c->gx_nbrz[variant];
    if (variant == 0) {
        ps.it = 1;
    } else {
        ps.rho = ps.rho == S_RHO ? S_RHO_NEW : S_RHO;
        ++ps.it;
    }
    return true;
}

// Decide on the scalars of the latest phase and launch the next one.
void pcg_advance(bido_ctx* c, PcgRun& ps) {
    const int64_t n = c->n2;
    auto finish = [&](bool conv, bido_status st, const std::string& msg) {
        ps.done = true;
        ps.conv = conv;
        ps.status = st;
        ps.err = msg;
    };
    if (!ps.started) {
        ps.started = true;
        ps.yy = host_partials(c, PP_YY, ps.nb);
        ps.rel = ps.yy > 0 ? std::sqrt(host_partials(c, PP_RR, ps.nb) / ps.yy) : 0.0;
        if (ps.yy == 0.0) {
            launch_fill(c->stream, n, c->x, 0.0);
            return finish(true, BIDO_OK, "");
        }
        if (ps.rel <= ps.tol) return finish(true, BIDO_OK, "");
        if (!seq_graph(c, ps, 0)) seq_first(c, ps);
        return;
    }
    const double pq = c->sc_host[S_PQ], rz = c->sc_host[ps.rho];
    ps.rel = std::sqrt(host_partials(c, PP_RR, ps.nb) / ps.yy);
    if (!(pq > 0.0) || !(rz > 0.0) || !std::isfinite(ps.rel))
        return finish(false, BIDO_ERR_NOT_SPD,
                      "CG breakdown (p.Ap = " + std::to_string(pq) + ", r.z = " + std::to_string(rz) + ")");
    if (ps.rel <= ps.tol) return finish(true, BIDO_OK, "");
    if (ps.it >= c->params.max_iter)
        return finish(false, BIDO_ERR_NOT_CONVERGED, "tolerance not reached within max_iter");
    if (!seq_graph(c, ps, ps.rho == S_RHO ? 1 : 2)) seq_iter(c, ps);
}

bido_status pcg_result(bido_ctx* c, const PcgRun& ps, bido_stats* st) {
    c->fallbacks += ps.fallbacks;
    if (st) {
        st->iterations = ps.it;
        st->rel_residual = ps.rel;
        st->converged = ps.conv ? 1 : 0;
        st->fallbacks = ps.fallbacks;
    }
    return ps.status ? fail(ps.status, ps.err) : BIDO_OK;
}

bido_status pcg(bido_ctx* c, double tol, bido_stats* st) {
    PcgRun ps;
    pcg_start(c, ps, tol);
    while (!ps.done) {
        HIP_OK(hipStreamSynchronize(c->stream));
        pcg_advance(c, ps);
    }
    return pcg_result(c, ps, st);
}

// After a converged solve while collecting: targets (V* - V_k - Z2_k) / |t_k|.
void finish_collection(bido_ctx* c, bool converged) {
    GnnState& g = c->gnn;
    if (!g.collecting) return;
    if (g.increments) {
        // one stencil pair per step from the converged solutions of this step
        // and the previous one: z = V^{n+1} - V^n, t = Y_2^n - Y_2^{n-1}
        const int64_t NH = c->NH;
        if (!converged) {
            g.inc_ok = false;
            return;
        }
        if (g.inc_ok && g.n_samples < g.max_samples) {
            const int slot = g.n_samples;
            launch_gnn_sub(c->stream, NH, c->x + c->N, g.inc_v, g.tz);
            launch_gnn_sub(c->stream, NH, c->Y + c->N, g.inc_y, g.pend_t);
            launch_dot_reduce(c->stream, NH, g.tz, g.tz, c->rd, g.s_zz + slot);
            launch_stencil_sample(c->stream, NH, g.K, g.tz, g.s_zz + slot, g.pend_t, g.dbar,
                                  g.s_z + (int64_t)slot * NH, g.s_b + (int64_t)slot * NH);
            ++g.n_samples;
        }
        hipMemcpyAsync(g.inc_v, c->x + c->N, NH * sizeof(double), hipMemcpyDeviceToDevice, c->stream);
        hipMemcpyAsync(g.inc_y, c->Y + c->N, NH * sizeof(double), hipMemcpyDeviceToDevice, c->stream);
        g.inc_ok = true;
        return;
    }
    if (converged)
        for (int k = 0; k < g.n_pending; ++k) {
            const int slot = g.n_samples + k;
            const int64_t NH = c->NH;
            launch_gnn_finish_targets(c->stream, NH, c->x + c->N, g.pend + (int64_t)k * NH,
                                      g.s_tn2 + slot, g.s_y + (int64_t)slot * NH);
            // stencil pair: z* = V* - V_k, b = t_k - K_m z*
            launch_gnn_sub(c->stream, NH, c->x + c->N, g.pend_v + (int64_t)k * NH, g.tz);
            launch_dot_reduce(c->stream, NH, g.tz, g.tz, c->rd, g.s_zz + slot);
            launch_stencil_sample(c->stream, NH, g.K, g.tz, g.s_zz + slot, g.pend_t + (int64_t)k * NH,
                                  g.dbar, g.s_z + (int64_t)slot * NH, g.s_b + (int64_t)slot * NH);
        }
    if (converged) g.n_samples += g.n_pending;
    g.n_pending = 0;
}

IonicConst ionic_consts(const bido_ctx* c) {
    IonicConst k;
    k.gamma = c->hs.gamma;
    k.chi = c->params.chi;
    k.cm = c->params.cm;
    k.dt = c->params.dt;
    k.dv = 100.0;
    k.inv_dv = 1.0 / 100.0;
    k.inv_tau_in = 1.0 / 0.3;
    k.inv_tau_out = 1.0 / 6.0;
    k.inv_tau_open = 1.0 / 120.0;
    k.inv_tau_close = 1.0 / 150.0;
    k.v_gate = 0.13;
    k.scale = c->params.scheme == BIDO_SCHEME_EULER ? 1.0 : 2.0;
    k.reaction = c->params.scheme == BIDO_SCHEME_STRANG ? 0.0 : 1.0;
    return k;
}

// The elliptic solve of a Strang step, S_1 tA = tC (tC = Pi^T S_i V*, zero
// sum), to the context's tolerance: P_1 is exact only with exact factors
// (a hierarchical top at eps_h > 0 leaves an O(eps_h) error), so the one
// P_1 apply in tA is refined, tA += P_1^-1 (tC - S_1 tA), until
// |tC - S_1 tA| <= tol/10 |tC| (S_1 tA is the u-row product of Lambda with
// (tA, 0)).  FP64 throughout; one residual check (a host wait) per round.
void elliptic_refine(bido_ctx* c) {
    hipStream_t s = c->stream;
    const int64_t N = c->N;
    CsrDev urows = c->lam;                   // the u rows of Lambda: [S_1, Pi^T S_i]
    urows.n = N;
    urows.nnz = c->hs.lam.ptr[N];
    const double want = 0.1 * c->params.tol;
    PROF(c, K_MISC, 16.0 * N, launch_dot_reduce(s, N, c->tC, c->tC, c->rd, c->sc + S_EL_BB));
    PROF(c, K_MISC, 8.0 * c->n2, launch_fill(s, c->n2, c->q, 0.0));
    for (int round = 0; round < 60; ++round) {
        if (hipMemcpyAsync(c->q, c->tA, N * sizeof(double), hipMemcpyDeviceToDevice, s) != hipSuccess) return;
        PROF(c, K_SPMV_CSR, csr_bytes(urows, c->n2),
             launch_spmv_csr(s, urows, c->spmv_group, c->q, c->tC, c->tD));            // tC - S_1 tA
        PROF(c, K_MISC, 16.0 * N, launch_dot_reduce(s, N, c->tD, c->tD, c->rd, c->sc + S_EL_RR));
        if (hipMemcpyAsync(c->sc_host + S_EL_RR, c->sc + S_EL_RR, 2 * sizeof(double), hipMemcpyDeviceToHost,
                           s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            return;                              // reported by the caller's error check
        const double rr = c->sc_host[S_EL_RR], bb = c->sc_host[S_EL_BB];
        if (!(rr > want * want * bb)) break;     // converged (or b = 0)
        if (c->amg1.on()) amg_vcycle(c, c->amg1, 0, c->tD, c->r, true);
        else tri_solve<double>(c, c->p1, c->p1.panel64, c->p1.panel64_cm, c->tD, c->r);
        PROF(c, K_MISC, 24.0 * N, launch_axpy(s, N, 1.0, c->r, c->tA));
    }
}

// The initial guess of step n from the states the previous steps of this
// context started from (consecutive steps n - 1, n - 2, ... at the same
// dt): X^n (the state passed in) joins the ring with its Lambda image and
// its Gram row, and X0 = W c with (W^T Lambda W) c = W^T Y over the ring,
// the Lambda-orthogonal projection of the solution onto the span of the
// states (Fischer's projection for a sequence of right-hand sides), which
// holds X^n: the guess is never farther from the solution in the Lambda
// norm than X^n.  Launches only; no host wait.
void project_guess(bido_ctx* c, int64_t n) {
    hipStream_t s = c->stream;
    const int K = c->params.guess_states;
    const int64_t n2 = c->n2;
    if (c->g_n != n - 1) c->g_len = 0;
    const int slot = (c->g_head + K - 1) % K;       // the oldest (or a free) slot becomes the newest
    c->g_head = slot;
    c->g_len = std::min(c->g_len + 1, K);
    c->g_n = n;
    if (hipMemcpyAsync(c->gw[slot], c->x, n2 * sizeof(double), hipMemcpyDeviceToDevice, s) != hipSuccess) {
        c->g_len = 0;                               // X0 = X^n; the next step starts a new span
        c->g_n = -2;
        return;
    }
    if (c->lamb.on())
        PROF(c, K_SPMV_LAMBDA, blk_bytes(c->lamb, 0),
             launch_spmv_lam_blk(s, c->lamb, c->spmv_group, 0, c->x, nullptr, c->gaw[slot], c->sc));
    else
        PROF(c, K_SPMV_LAMBDA, csr_bytes(c->lam, n2),
             launch_spmv_lambda(s, c->lam, c->spmv_group, 0, c->x, nullptr, c->gaw[slot], c->sc));
    GuessList W;
    W.m = c->g_len;
    for (int k = 0; k < W.m; ++k) {
        W.slot[k] = (slot + k) % K;
        W.v[k] = c->gw[W.slot[k]];
    }
    const double vb = 8.0 * n2 * (W.m + 1);
    PROF(c, K_MISC, vb, launch_multidot(s, n2, W, c->gaw[slot], c->grd, c->gd));     // the new Gram row
    PROF(c, K_MISC, vb, launch_multidot(s, n2, W, c->Y, c->grd, c->gb));             // W^T Y
    PROF(c, K_MISC, 0.0, launch_guess_solve(s, W, c->gd, c->gG, c->gb, c->gc));
    PROF(c, K_MISC, vb, launch_guess_combine(s, n2, W, c->gc, c->x));
}

// Steps 1 and 3 on the device: X0 = (U^n, V^n) and the right-hand side Y.
void step_prepare(bido_ctx* c, double* v, double* w, double* u, int64_t n) {
    hipStream_t s = c->stream;
    const int64_t N = c->N, NH = c->NH;
    c->step_n = n;
    const double on = (n >= c->hs.stim_n0 && n < c->hs.stim_n1) ? 1.0 : 0.0;
    const double* sub = nullptr;
    const double* vin = v;
    CsrDev rows = c->lam;                    // the v rows of Lambda
    rows.n = NH;
    rows.ptr = c->lam.ptr + N;
    rows.nnz = c->hs.lam.ptr[c->n2] - c->hs.lam.ptr[N];
    if (c->params.scheme == BIDO_SCHEME_STRANG) {
        // Strang splitting: a reaction half-step first (V* into vs, h* into
        // w), then the Crank-Nicolson diffusion step without the ionic term
        // from (U*, V*), U* the elliptic potential of V*
        // (S_1 U* = -Pi^T S_i V*; one P_1 apply): with tA = S_1^+ Pi^T S_i V*
        // (up to a constant, which S_i Pi ignores) and X = (0, V*),
        // S_i (V* + Pi U*) + 2 gamma M_H V* = (Lambda X)_v - S_i Pi tA
        PROF(c, K_IONIC, 32.0 * NH,
             launch_strang_in(s, NH, v, w, c->stim_loc, on, 0.5 * c->params.dt, ionic_consts(c), c->vs));
        vin = c->vs;
        PROF(c, K_MISC, 24.0 * NH, launch_scatter_in(s, NH, c->v_pos, vin, c->x + N));
        PROF(c, K_SPMV_CSR, csr_bytes(c->auv, NH),
             launch_spmv_csr(s, c->auv, c->spmv_group, c->x + N, nullptr, c->tC));   // Pi^T S_i V*
        if (c->amg1.on()) amg_vcycle(c, c->amg1, 0, c->tC, c->tA, true);             // FP64 in both precisions
        else tri_solve<double>(c, c->p1, c->p1.panel64, c->p1.panel64_cm, c->tC, c->tA);
        elliptic_refine(c);
        PROF(c, K_MISC, 8.0 * N, launch_fill(s, N, c->x, 0.0));
        PROF(c, K_SPMV_CSR, csr_bytes(rows, c->n2),
             launch_spmv_csr(s, rows, c->spmv_group, c->x, nullptr, c->tB));          // (Lambda (0, V*))_v
        PROF(c, K_SPMV_CSR, csr_bytes(c->avu, N) + 8.0 * NH,
             launch_spmv_csr(s, c->avu, c->spmv_group, c->tA, c->tB, c->tD));
        sub = c->tD;
        PROF(c, K_MISC, 24.0 * N, launch_scatter_in(s, N, c->u_pos, u, c->x));      // initial guess U^n
    } else {
        PROF(c, K_MISC, 24.0 * N, launch_scatter_in(s, N, c->u_pos, u, c->x));      // X0 = (U^n, V^n)
        if (c->params.scheme == BIDO_SCHEME_CN) {
            // Crank-Nicolson: S_i (V^n + Pi U^n) = (Lambda X^n)_v - 2 gamma M_H V^n,
            // so Y_2 = 2 M_H (2 gamma V^n - chi (I_ion - I_st)) - (Lambda X^n)_v
            // with 2 gamma the coefficient of M_H in Lambda
            PROF(c, K_MISC, 24.0 * NH, launch_scatter_in(s, NH, c->v_pos, v, c->x + N));
            PROF(c, K_SPMV_CSR, csr_bytes(rows, c->n2),
                 launch_spmv_csr(s, rows, c->spmv_group, c->x, nullptr, c->tB));
            sub = c->tB;
        }
    }
    PROF(c, K_IONIC, 64.0 * NH,
         launch_ionic(s, NH, vin, w, c->stim_loc, on, c->mh_loc, c->v_pos, c->Y + N, c->x + N, sub,
                      ionic_consts(c)));                               // Steps 1 and 3
    PROF(c, K_MISC, 8.0 * N, launch_fill(s, N, c->Y, 0.0));           // Y1 = 0
    if (c->params.guess_states) project_guess(c, n);
}

// Steps 1 and 3 and the start of Step 2 (no wait).
void step_begin(bido_ctx* c, double* v, double* w, double* u, int64_t n, PcgRun& ps) {
    step_prepare(c, v, w, u, n);
    pcg_start(c, ps, c->params.tol);                                   // Step 2
}

// After Step 2: normalisation (M U, 1) = 0 and the write-back of U, V.
void step_write(bido_ctx* c, double* v, double* w, double* u) {
    hipStream_t s = c->stream;
    const int64_t N = c->N, NH = c->NH;
    PROF(c, K_MISC, 16.0 * N, launch_dot_reduce(s, N, c->m_int, c->x, c->rd, c->sc + S_MU));  // (M U, 1)
    PROF(c, K_MISC, 24.0 * N, launch_gather_out(s, N, c->u_pos, c->x, u, c->sc, S_MU, c->hs.msum));
    auto& rec = c->rec;
    if (c->params.scheme == BIDO_SCHEME_STRANG) {
        // Strang splitting: the second reaction half-step from (V**, h*)
        const int64_t n = c->step_n;
        const double on = (n >= c->hs.stim_n0 && n < c->hs.stim_n1) ? 1.0 : 0.0;
        const bool act = rec.on && rec.act_on;
        PROF(c, K_IONIC, 48.0 * NH,
             launch_strang_out(s, NH, c->v_pos, c->x + N, v, w, c->stim_loc, on, 0.5 * c->params.dt, ionic_consts(c),
                               act ? rec.act : nullptr, rec.v_act, (double)n * c->params.dt, c->params.dt));
    } else if (rec.on && rec.act_on) {
        PROF(c, K_MISC, 48.0 * NH,
             launch_gather_v_act(s, NH, c->v_pos, c->x + N, v, rec.act, rec.v_act, (double)c->step_n * c->params.dt,
                                 c->params.dt));
    } else {
        PROF(c, K_MISC, 24.0 * NH, launch_gather_out(s, NH, c->v_pos, c->x + N, v, c->sc, -1, 1.0));
    }
    if (rec.on && rec.np > 0 && rec.n_rows < rec.max_steps) {
        PROF(c, K_MISC, 24.0 * rec.np * rec.nv,
             launch_probe(s, rec.np, rec.nv, rec.ids, rec.wts, u, rec.rows + rec.n_rows * rec.np));
        ++rec.n_rows;
    }
}

bido_status step_end(bido_ctx* c, double* v, double* w, double* u, const PcgRun& ps, bido_stats* st) {
    bido_status e = pcg_result(c, ps, st);
    finish_collection(c, e == BIDO_OK);
    if (e && e != BIDO_ERR_NOT_CONVERGED) return e;
    step_write(c, v, w, u);
    return e;
}

bido_status step_once(bido_ctx* c, double* v, double* w, double* u, int64_t n, bido_stats* st) {
    PcgRun ps;
    step_begin(c, v, w, u, n, ps);
    while (!ps.done) {
        HIP_OK(hipStreamSynchronize(c->stream));
        pcg_advance(c, ps);
    }
    return step_end(c, v, w, u, ps, st);
}

// Weights: fan-in scaled normal, zero biases; the readout starts at zero so
// that an untrained correction is exactly the plain preconditioner.  Adam's
// moments start at zero.
bido_status gnn_init_weights(bido_ctx* c) {
    GnnState& g = c->gnn;
    std::vector<float> th(GNN_P, 0.0f);
    std::mt19937_64 rng(12345);
    std::normal_distribution<double> nd(0.0, 1.0);
    for (int k = 0; k < GNN_H * GNN_F; ++k) {
        th[GNN_OFF_W1S + k] = (float)(nd(rng) / std::sqrt((double)GNN_F));
        th[GNN_OFF_W1N + k] = (float)(nd(rng) / std::sqrt((double)GNN_F));
    }
    for (int k = 0; k < GNN_H * GNN_H; ++k) {
        th[GNN_OFF_W2S + k] = (float)(nd(rng) / std::sqrt((double)GNN_H));
        th[GNN_OFF_W2N + k] = (float)(nd(rng) / std::sqrt((double)GNN_H));
    }
    HIP_OK(hipMemcpy(g.theta, th.data(), GNN_P * sizeof(float), hipMemcpyHostToDevice));
    for (float* b : {g.m, g.v, g.grad}) HIP_OK(hipMemset(b, 0, GNN_P * sizeof(float)));
    launch_gnn_to_bf16(c->stream, g.theta, g.wbf);
    g.adam_step = 0;
    g.out_scale = 1.0f;
    return BIDO_OK;
}

bido_status gnn_setup(bido_ctx* c) {
    GnnState& g = c->gnn;
    const HostSetup& hs = c->hs;
    const int64_t NH = c->NH;
    std::vector<float> stat((size_t)NH * GNN_F, 0.0f);
    for (int64_t k = 0; k < NH; ++k)
        for (int j = 1; j < GNN_F; ++j) stat[hs.v_pos[k] * GNN_F + j] = (float)hs.gnn_static[k * 15 + j - 1];
    HIP_OK(upload(&g.stat, stat.data(), stat.size()));
    // neighbour weights in internal order, and the transpose
    const Csr& G = hs.gnn_agg;
    std::vector<std::vector<std::pair<int32_t, float>>> rows(NH), trows(NH);
    for (int64_t k = 0; k < NH; ++k)
        for (int64_t p = G.ptr[k]; p < G.ptr[k + 1]; ++p) {
            const int32_t i = (int32_t)hs.v_pos[k], j = (int32_t)hs.v_pos[G.col[p]];
            rows[i].push_back({j, (float)G.val[p]});
            trows[j].push_back({i, (float)G.val[p]});
        }
    auto up_graph = [&](std::vector<std::vector<std::pair<int32_t, float>>>& R, GnnGraph& out) -> bido_status {
        std::vector<int64_t> ptr(NH + 1, 0);
        std::vector<int32_t> col;
        std::vector<float> val;
        for (int64_t i = 0; i < NH; ++i) {
            std::sort(R[i].begin(), R[i].end());
            for (auto& e : R[i]) { col.push_back(e.first); val.push_back(e.second); }
            ptr[i + 1] = (int64_t)col.size();
        }
        out.n = NH;
        HIP_OK(upload(&out.ptr, ptr.data(), ptr.size()));
        HIP_OK(upload(&out.col, col.data(), std::max<size_t>(col.size(), 1)));
        HIP_OK(upload(&out.val, val.data(), std::max<size_t>(val.size(), 1)));
        return BIDO_OK;
    };
    bido_status e;
    if ((e = up_graph(rows, g.A))) return e;
    if ((e = up_graph(trows, g.At))) return e;
    // stored S_m pattern (= pattern of K_m) in internal order, and K_m itself
    {
        const Csr& Km = hs.km_int;
        std::vector<int32_t> row(Km.nnz()), tpos(Km.nnz());
        for (int64_t i = 0; i < NH; ++i)
            for (int64_t p = Km.ptr[i]; p < Km.ptr[i + 1]; ++p) row[p] = (int32_t)i;
        for (int64_t i = 0; i < NH; ++i)
            for (int64_t p = Km.ptr[i]; p < Km.ptr[i + 1]; ++p) {
                const int64_t j = Km.col[p];
                const auto b = Km.col.begin() + Km.ptr[j], e = Km.col.begin() + Km.ptr[j + 1];
                const auto it = std::lower_bound(b, e, (int32_t)i);
                if (it == e || *it != (int32_t)i) return fail(BIDO_ERR_ARG, "S_m pattern is not symmetric");
                tpos[p] = (int32_t)(it - Km.col.begin());
            }
        g.P.n = NH;
        g.P.nnz = Km.nnz();
        HIP_OK(upload(&g.P.ptr, Km.ptr.data(), Km.ptr.size()));
        HIP_OK(upload(&g.P.col, Km.col.data(), std::max<size_t>(Km.col.size(), 1)));
        HIP_OK(upload(&g.P.row, row.data(), std::max<size_t>(row.size(), 1)));
        HIP_OK(upload(&g.P.tpos, tpos.data(), std::max<size_t>(tpos.size(), 1)));
        HIP_OK(upload(&g.K.ptr, Km.ptr.data(), Km.ptr.size()));
        HIP_OK(upload(&g.K.col, Km.col.data(), std::max<size_t>(Km.col.size(), 1)));
        HIP_OK(upload(&g.K.val, Km.val.data(), std::max<size_t>(Km.val.size(), 1)));
        double dsum = 0.0;
        for (int64_t i = 0; i < NH; ++i)
            for (int64_t p = Km.ptr[i]; p < Km.ptr[i + 1]; ++p)
                if (Km.col[p] == i) dsum += Km.val[p];
        g.dbar = dsum / std::max<int64_t>(NH, 1);
        HIP_OK(hipMalloc((void**)&g.cval, std::max<int64_t>(Km.nnz(), 1) * sizeof(float)));
        HIP_OK(hipMalloc((void**)&g.G, std::max<int64_t>(Km.nnz(), 1) * sizeof(float)));
        HIP_OK(hipMalloc((void**)&g.r, std::max<int64_t>(NH, 1) * sizeof(float)));
    }
    // K_m = gamma M_H + S_m scaled to unit mean diagonal, internal order
    {
        const Csr& Sm = hs.A.Sm;
        std::vector<std::vector<std::pair<int32_t, float>>> wrows(NH);
        double dsum = 0.0;
        for (int64_t k = 0; k < NH; ++k) dsum += hs.gamma * hs.A.mH[k];
        for (int64_t k = 0; k < NH; ++k)
            for (int64_t p = Sm.ptr[k]; p < Sm.ptr[k + 1]; ++p)
                if (Sm.col[p] == k) dsum += Sm.val[p];
        const double dmean = dsum / std::max<int64_t>(NH, 1);
        for (int64_t k = 0; k < NH; ++k)
            for (int64_t p = Sm.ptr[k]; p < Sm.ptr[k + 1]; ++p) {
                double val = Sm.val[p] + (Sm.col[p] == k ? hs.gamma * hs.A.mH[k] : 0.0);
                wrows[hs.v_pos[k]].push_back({(int32_t)hs.v_pos[Sm.col[p]], (float)(val / dmean)});
            }
        if ((e = up_graph(wrows, g.Wk))) return e;
    }
    g.wk_like_k = g.Wk.n == NH && hs.km_int.ptr.size() == (size_t)NH + 1;
    if (g.wk_like_k) {       // the scaled copy shares K_m's stored pattern (a new step moves values only)
        std::vector<int64_t> wp(NH + 1);
        std::vector<int32_t> wc(std::max<int64_t>(hs.km_int.nnz(), 1));
        HIP_OK(hipMemcpy(wp.data(), g.Wk.ptr, wp.size() * sizeof(int64_t), hipMemcpyDeviceToHost));
        HIP_OK(hipMemcpy(wc.data(), g.Wk.col, wc.size() * sizeof(int32_t), hipMemcpyDeviceToHost));
        g.wk_like_k = wp == hs.km_int.ptr &&
                      std::equal(hs.km_int.col.begin(), hs.km_int.col.end(), wc.begin());
    }
    for (float** b : {&g.theta, &g.theta_best, &g.m, &g.v, &g.grad})
        HIP_OK(hipMalloc((void**)b, GNN_P * sizeof(float)));
    HIP_OK(hipMalloc((void**)&g.wbf, GNN_P * sizeof(uint16_t)));
    if ((e = gnn_init_weights(c))) return e;
    const int64_t nh = std::max<int64_t>(NH, 1);
    for (uint16_t** b : {&g.act.f, &g.act.m0}) HIP_OK(hipMalloc((void**)b, nh * GNN_F * sizeof(uint16_t)));
    for (uint16_t** b : {&g.act.h1, &g.act.m1, &g.act.h2}) HIP_OK(hipMalloc((void**)b, nh * GNN_H * sizeof(uint16_t)));
    for (float** b : {&g.act.o, &g.act.dout, &g.act.res, &g.act.zero, &g.ft, &g.fy})
        HIP_OK(hipMalloc((void**)b, nh * sizeof(float)));
    HIP_OK(hipMemset(g.act.zero, 0, nh * sizeof(float)));
    for (float** b : {&g.act.dz2, &g.act.g2, &g.act.dz1}) HIP_OK(hipMalloc((void**)b, nh * GNN_H * sizeof(float)));
    const int64_t np = (int64_t)GNN_WG_BLOCKS * GNN_P + (nh * GNN_H + 255) / 256 + 256;
    HIP_OK(hipMalloc((void**)&g.partials, np * sizeof(float)));
    HIP_OK(hipMalloc((void**)&g.dloss, 4 * sizeof(double)));
    HIP_OK(hipMalloc((void**)&g.tz, nh * sizeof(double)));
    return BIDO_OK;
}

// A new time step: K_m's values (its device copy, its mean diagonal and the
// loss weights K_m / mean diagonal) move with gamma, its pattern does not;
// the pairs, weights and stencil fitted at the old step are dropped and the
// weights start again from their initial values.
bido_status gnn_new_step(bido_ctx* c) {
    GnnState& g = c->gnn;
    const HostSetup& hs = c->hs;
    const Csr& Km = hs.km_int;
    const int64_t NH = c->NH;
    if (!g.wk_like_k) {                    // (not expected: a full set-up again)
        g.release();
        return gnn_setup(c);
    }
    HIP_OK(hipMemcpy(g.K.val, Km.val.data(), std::max<size_t>(Km.val.size(), 1) * sizeof(double),
                     hipMemcpyHostToDevice));
    double dsum = 0.0;
    for (int64_t i = 0; i < NH; ++i)
        for (int64_t p = Km.ptr[i]; p < Km.ptr[i + 1]; ++p)
            if (Km.col[p] == i) dsum += Km.val[p];
    g.dbar = dsum / std::max<int64_t>(NH, 1);
    double ds = 0.0;                       // the loss weights' scale, in the set-up's order
    for (int64_t k = 0; k < NH; ++k) ds += hs.gamma * hs.A.mH[k];
    for (int64_t k = 0; k < NH; ++k)
        for (int64_t p = hs.A.Sm.ptr[k]; p < hs.A.Sm.ptr[k + 1]; ++p)
            if (hs.A.Sm.col[p] == k) ds += hs.A.Sm.val[p];
    const double dmean = ds / std::max<int64_t>(NH, 1);
    std::vector<float> wv(std::max<int64_t>(Km.nnz(), 1), 0.0f);
    for (int64_t p = 0; p < Km.nnz(); ++p) wv[p] = (float)(Km.val[p] / dmean);
    HIP_OK(hipMemcpy(g.Wk.val, wv.data(), wv.size() * sizeof(float), hipMemcpyHostToDevice));
    if (bido_status e = gnn_init_weights(c)) return e;
    g.n_samples = 0;
    g.n_pending = 0;
    g.collecting = false;
    g.stencil_ready = false;
    g.increments = false;
    g.inc_ok = false;
    HIP_OK(hipStreamSynchronize(c->stream));
    return BIDO_OK;
}

bool dt_matches(const bido_ctx* c, double dt) {
    return std::fabs(dt - c->params.dt) <= 1e-12 * std::fabs(c->params.dt);
}

// ---------------------------------------------------------------------------
// Fused batch: the slices side by side in one union vector (slice s at
// off[s], its u rows then its v rows), one block-diagonal Lambda, S_i Pi and
// Pi^T S_i, and the merged forests of the slices' P1 and PK factors.  Each
// PCG phase is one launch sequence for all slices; the scalars and the
// stopping test stay per slice, and a finished slice is frozen
// (alpha = beta = 0) while the others go on.
// ---------------------------------------------------------------------------
constexpr int64_t SEG_ROWS = 1024;   // rows per block of the segmented kernels

enum { FR_RR = 0, FR_YY, FR_PQ, FR_RZ, FR_ZRO, FR_COUNT };

struct FusedBatch {
    hipStream_t stream = nullptr;
    Profiler prof;
    int precision = BIDO_PREC_FP64;
    int spmv_group = 8;
    bool graphs = true;
    int S = 0;
    int64_t n = 0;
    std::vector<int64_t> off, n2;
    CsrDev lam, avu, auv;
    FactorDev p1, pk;
    SegTable T, Tu, Tv;
    std::vector<void*> tables;          // device arrays of the three tables
    std::vector<SegSlice> slices;       // T's slices (host copy)
    double *x = nullptr, *r = nullptr, *z = nullptr, *p = nullptr, *q = nullptr, *Y = nullptr;
    double *tA = nullptr, *tB = nullptr, *tC = nullptr, *tD = nullptr, *r_old = nullptr;
    double* sc = nullptr;               // r.z (2 slots of S), p.q (S), then FR_COUNT partial regions
    double* sc_host = nullptr;          // pinned
    uint8_t *done = nullptr, *done_host = nullptr;
    // the stopping test on the device: per slice |Y|^2, tol, iteration cap,
    // and the test's outputs (iterations, status, |r| / |Y|), copied back
    // in one block (it_host points at the pinned copy)
    double *yy = nullptr, *tol = nullptr, *rel = nullptr;
    int *max_it = nullptr, *iters = nullptr, *status = nullptr;
    void* back_host = nullptr;            // pinned: done, iters, status, rel
    int last_iters = 0;                   // iterations of the latest step (first chunk of the next)
    int64_t n_steps = 0, host_waits = 0, iterations = 0, graph_kernels[3] = {0, 0, 0}, kernels = 0;
    hipGraphExec_t gx[3] = {nullptr, nullptr, nullptr};
    double setup_seconds = 0.0;
    // P_K by Chebyshev-accelerated Jacobi on the union K_m (one step count
    // for all slices, each slice with its own interval): cheb holds
    // inv_theta[S], then c1[S], c2[S] for each step after the first
    int pk_kind = BIDO_PK_CHOLESKY;
    int cheb_steps = 0;
    int64_t nv = 0;                     // v rows of all slices
    CsrDev km;
    double *km_dinv = nullptr, *cheb = nullptr, *ch_r = nullptr, *ch_d[2] = {nullptr, nullptr};

    int64_t region(int k) const { return 3 * (int64_t)S + (int64_t)k * T.nblocks; }
    double* part(int k) const { return sc + region(k); }
    double host_sum(int k, int s) const {
        double a = 0.0;
        for (int b = slices[s].b0; b < slices[s].b1; ++b) a += sc_host[region(k) + b];
        return a;
    }
    // each slice's preconditioner at creation (plain or the learned
    // stencil); the direction update is the flexible one in mixed precision
    // or with a learned slice, as for the slice run alone
    std::vector<int> precond;
    bool learned = false;
    bool flexible() const { return precision == BIDO_PREC_MIXED || learned; }
    void drop_graphs() {
        for (auto& g : gx)
            if (g) { hipGraphExecDestroy(g); g = nullptr; }
    }
    ~FusedBatch() {
        if (stream) hipStreamSynchronize(stream);
        drop_graphs();
        p1.release();
        pk.release();
        CsrHostView::release(lam);
        CsrHostView::release(avu);
        CsrHostView::release(auv);
        CsrHostView::release(km);
        for (void* t : tables) hipFree(t);
        for (double* b : {x, r, z, p, q, Y, tA, tB, tC, tD, r_old, sc, km_dinv, cheb, ch_r, ch_d[0], ch_d[1]})
            hipFree(b);
        hipFree(done);
        for (void* b : {(void*)yy, (void*)tol, (void*)rel, (void*)max_it, (void*)iters, (void*)status}) hipFree(b);
        if (back_host) hipHostFree(back_host);
        if (sc_host) hipHostFree(sc_host);
        if (done_host) hipHostFree(done_host);
        if (stream) hipStreamDestroy(stream);
    }
};

// Blocks of at most SEG_ROWS rows over the row range [start[s], start[s] +
// len[s]) of every slice.
void seg_layout(const std::vector<int64_t>& start, const std::vector<int64_t>& len, const std::vector<int64_t>& base,
                const std::vector<int64_t>& nu, std::vector<SegBlock>& blk, std::vector<SegSlice>& sl) {
    blk.clear();
    sl.assign(start.size(), SegSlice{});
    for (size_t s = 0; s < start.size(); ++s) {
        sl[s].base = base[s];
        sl[s].nu = nu[s];
        sl[s].b0 = (int32_t)blk.size();
        for (int64_t r = start[s]; r < start[s] + len[s]; r += SEG_ROWS)
            blk.push_back({r, std::min(r + SEG_ROWS, start[s] + len[s]), (int32_t)s, 0});
        sl[s].b1 = (int32_t)blk.size();
    }
}

bido_status seg_upload(FusedBatch* F, const std::vector<SegBlock>& blk, const std::vector<SegSlice>& sl,
                       SegTable& T) {
    SegBlock* db = nullptr;
    SegSlice* ds = nullptr;
    HIP_OK(upload(&db, blk.data(), blk.size()));
    F->tables.push_back(db);
    HIP_OK(upload(&ds, sl.data(), sl.size()));
    F->tables.push_back(ds);
    T.nblocks = (int)blk.size();
    T.blk = db;
    T.sl = ds;
    return BIDO_OK;
}

// Block-diagonal union of CSR blocks: block s at rows row_off[s] and columns
// col_off[s]; rows outside every block are empty.
bido_status union_csr(const std::vector<const Csr*>& parts, const std::vector<int64_t>& row_off,
                      const std::vector<int64_t>& col_off, int64_t n, CsrDev& d) {
    Csr u;
    u.n = n;
    u.ptr.assign(n + 1, 0);
    int64_t nnz = 0;
    for (const Csr* a : parts) nnz += a->nnz();
    u.col.reserve(nnz);
    u.val.reserve(nnz);
    std::vector<int64_t> order(parts.size());
    for (size_t s = 0; s < parts.size(); ++s) order[s] = (int64_t)s;
    std::sort(order.begin(), order.end(), [&](int64_t a, int64_t b) { return row_off[a] < row_off[b]; });
    int64_t row = 0;
    for (int64_t s : order) {
        const Csr& a = *parts[s];
        if (row_off[s] < row || row_off[s] + a.n > n) return fail(BIDO_ERR_ARG, "overlapping union blocks");
        for (; row < row_off[s]; ++row) u.ptr[row + 1] = (int64_t)u.col.size();
        for (int64_t i = 0; i < a.n; ++i, ++row) {
            for (int64_t k = a.ptr[i]; k < a.ptr[i + 1]; ++k) {
                u.col.push_back((int32_t)(a.col[k] + col_off[s]));
                u.val.push_back(a.val[k]);
            }
            u.ptr[row + 1] = (int64_t)u.col.size();
        }
    }
    for (; row < n; ++row) u.ptr[row + 1] = (int64_t)u.col.size();
    if (u.col.empty()) {                     // keep the device arrays non-null
        u.col.push_back(0);
        u.val.push_back(0.0);
    }
    return CsrHostView::up(u, d);
}

// Z2 = P_K^-1 t on the v rows of every active slice by Chebyshev steps
// (the same recurrence as pk_solve, with per-slice coefficients)
void fused_pk_cheb(FusedBatch* F, const double* in, double* out) {
    hipStream_t s = F->stream;
    const int S = F->S;
    const double nv = (double)F->nv, step_bytes = 12.0 * F->km.nnz + 8.0 * nv + 64.0 * nv;
    PROF(F, K_CHEB, 32.0 * nv,
         launch_seg_cheb_init(s, F->Tv, in, F->km_dinv, F->cheb, F->ch_d[0], out, F->done));
    for (int k = 1; k < F->cheb_steps; ++k) {
        const double* c1 = F->cheb + (int64_t)S * (1 + 2 * (k - 1));
        const bool last = k + 1 == F->cheb_steps;
        PROF(F, K_CHEB, last ? step_bytes - 16.0 * nv : step_bytes,
             launch_seg_cheb_step(s, F->Tv, F->km, F->spmv_group, F->km_dinv, k == 1 ? in : F->ch_r, F->ch_r,
                                  F->ch_d[(k - 1) & 1], F->ch_d[k & 1], out, c1, c1 + S, last, F->done));
    }
}

// z = P^-1 r for all slices (the same steps as precond_apply) and the
// partials of r.z (and r_old.z)
void fused_apply(FusedBatch* F, bool with_old) {
    hipStream_t s = F->stream;
    inner_solve(F, F->p1, F->r, F->tA);                                               // Z1 = P1^-1 R1
    launch_seg_csr(s, F->Tv, F->avu, F->spmv_group, F->tA, F->r, F->tB, F->done);      // R2 - S_i Pi Z1
    if (F->pk_kind == BIDO_PK_CHEBYSHEV) fused_pk_cheb(F, F->tB, F->z);                // Z2 = PK^-1 (...)
    else inner_solve(F, F->pk, F->tB, F->z);
    launch_seg_csr(s, F->Tu, F->auv, F->spmv_group, F->z, nullptr, F->tC, F->done);    // Pi^T S_i Z2
    inner_solve(F, F->p1, F->tC, F->tD);                                               // P1^-1 Pi^T S_i Z2
    launch_seg_combine(s, F->T, F->z, F->tA, F->tD, F->r, with_old ? F->r_old : nullptr, F->part(FR_RZ),
                       F->part(FR_ZRO), F->done);
}

// q = Lambda p, x += alpha p, r -= alpha q (alpha from r.z in slot `rho`);
// copy the scalars and the |r|^2 partials
void fused_tail(FusedBatch* F, int rho) {
    hipStream_t s = F->stream;
    const int S = F->S;
    launch_seg_spmv(s, F->T, F->lam, F->spmv_group, 0, F->p, nullptr, F->q, F->part(FR_PQ), nullptr, F->done);
    launch_seg_pcg_update(s, F->T, F->x, F->r, F->flexible() ? F->r_old : nullptr, F->p, F->q, F->part(FR_PQ),
                          F->part(FR_RR), F->sc + (int64_t)rho * S, F->done, F->sc + 2 * (int64_t)S);
    launch_seg_stop(s, S, F->T, F->part(FR_RR), F->sc, rho, F->yy, F->tol, F->max_it, F->done, F->iters, F->status,
                    F->rel);
}

// variant 0: the first iteration (p = z, r.z into slot 0); 1 and 2: a later
// one reading r.z from slot 0 or 1 and writing the other slot
void fused_seq(FusedBatch* F, int variant) {
    const int S = F->S;
    if (variant == 0) {
        fused_apply(F, false);
        launch_seg_p_update(F->stream, F->T, F->z, F->p, F->part(FR_RZ), nullptr, 1, 0, nullptr, F->sc, F->done);
        fused_tail(F, 0);
        return;
    }
    const int rho = variant - 1, next = 1 - rho;
    const bool flex = F->flexible();
    fused_apply(F, flex);
    launch_seg_p_update(F->stream, F->T, F->z, F->p, F->part(FR_RZ), F->part(FR_ZRO), 0, flex ? 1 : 0,
                        F->sc + (int64_t)rho * S, F->sc + (int64_t)next * S, F->done);
    fused_tail(F, next);
}

bido_status fused_launch(FusedBatch* F, int variant) {
    if (!F->graphs || F->prof.on || debug_on()) {
        fused_seq(F, variant);
        return BIDO_OK;
    }
    if (!F->gx[variant]) {
        HIP_OK(hipStreamBeginCapture(F->stream, hipStreamCaptureModeThreadLocal));
        fused_seq(F, variant);
        hipGraph_t g = nullptr;
        HIP_OK(hipStreamEndCapture(F->stream, &g));
        size_t nodes = 0;
        if (hipGraphGetNodes(g, nullptr, &nodes) == hipSuccess) F->graph_kernels[variant] = (int64_t)nodes;
        hipGraphExec_t x = nullptr;
        const hipError_t e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
        hipGraphDestroy(g);
        HIP_OK(e);
        F->gx[variant] = x;
    }
    HIP_OK(hipGraphLaunch(F->gx[variant], F->stream));
    return BIDO_OK;
}

struct SliceRun {
    double yy = 0.0, rel = 0.0;
    int it = 0;
    bool done = false, conv = false;
    bido_status status = BIDO_OK;
    std::string err;
};

// Step 2 for all slices of a fused batch (Steps 1 and 3 already launched):
// PCG from the present x with per-slice stopping tests.
bido_status fused_pcg(FusedBatch* F, const std::vector<bido_ctx*>& ctx, std::vector<SliceRun>& sr) {
    const int S = F->S;
    hipStream_t s = F->stream;
    launch_seg_spmv(s, F->T, F->lam, F->spmv_group, 1, F->x, F->Y, F->r, F->part(FR_RR), F->part(FR_YY), nullptr);
    HIP_OK(hipMemcpyAsync(F->sc_host, F->sc, F->region(FR_YY + 1) * sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_OK(hipStreamSynchronize(s));
    sr.assign(S, SliceRun());
    int active = 0;
    for (int i = 0; i < S; ++i) {
        SliceRun& q = sr[i];
        q.yy = F->host_sum(FR_YY, i);
        q.rel = q.yy > 0 ? std::sqrt(F->host_sum(FR_RR, i) / q.yy) : 0.0;
        if (q.yy == 0.0) {
            launch_fill(s, F->n2[i], F->x + F->off[i], 0.0);
            q.done = q.conv = true;
        } else if (q.rel <= ctx[i]->params.tol) {
            q.done = q.conv = true;
        }
        F->done_host[i] = q.done ? 1 : 0;
        active += !q.done;
    }
    // the iterations run without the host: each captured iteration ends with
    // the device stopping test; the host looks once per chunk (first chunk:
    // one less than the previous step's count, then one at a time)
    {
        std::vector<double> yy(S), tl(S);
        std::vector<int> mi(S);
        for (int i = 0; i < S; ++i) {
            yy[i] = sr[i].yy > 0.0 ? sr[i].yy : 1.0;
            tl[i] = ctx[i]->params.tol;
            mi[i] = ctx[i]->params.max_iter;
        }
        HIP_OK(hipMemcpyAsync(F->yy, yy.data(), S * sizeof(double), hipMemcpyHostToDevice, s));
        HIP_OK(hipMemcpyAsync(F->tol, tl.data(), S * sizeof(double), hipMemcpyHostToDevice, s));
        HIP_OK(hipMemcpyAsync(F->max_it, mi.data(), S * sizeof(int), hipMemcpyHostToDevice, s));
        HIP_OK(hipMemcpyAsync(F->done, F->done_host, S, hipMemcpyHostToDevice, s));
        HIP_OK(hipMemsetAsync(F->iters, 0, S * sizeof(int), s));
        HIP_OK(hipMemsetAsync(F->status, 0, S * sizeof(int), s));
    }
    uint8_t* bdone = (uint8_t*)F->back_host;
    int* biters = (int*)((char*)F->back_host + 64 * (((int64_t)S + 63) / 64));
    int* bstat = biters + S;
    double* brel = (double*)((char*)F->back_host + 64 * (((int64_t)S + 63) / 64) + 8 * (((int64_t)2 * S * 4 + 7) / 8));
    int rho = 0, launched = 0;
    int chunk = std::max(1, F->last_iters - 1);
    while (active > 0) {
        for (int k = 0; k < chunk; ++k) {
            bido_status e;
            int variant = 0;
            if (launched > 0) {
                variant = rho == 0 ? 1 : 2;
                rho = 1 - rho;
            }
            if ((e = fused_launch(F, variant))) return e;
            F->kernels += F->graph_kernels[variant];
            ++launched;
        }
        HIP_OK(hipMemcpyAsync(bdone, F->done, S, hipMemcpyDeviceToHost, s));
        HIP_OK(hipMemcpyAsync(biters, F->iters, S * sizeof(int), hipMemcpyDeviceToHost, s));
        HIP_OK(hipMemcpyAsync(bstat, F->status, S * sizeof(int), hipMemcpyDeviceToHost, s));
        HIP_OK(hipMemcpyAsync(brel, F->rel, S * sizeof(double), hipMemcpyDeviceToHost, s));
        HIP_OK(hipStreamSynchronize(s));
        ++F->host_waits;
        active = 0;
        for (int i = 0; i < S; ++i) {
            SliceRun& q = sr[i];
            if (q.done) continue;
            q.it = biters[i];
            q.rel = brel[i];
            if (bdone[i]) {
                q.done = true;
                if (bstat[i] == 0) {
                    q.conv = true;
                } else if (bstat[i] == 1) {
                    q.status = BIDO_ERR_NOT_SPD;
                    q.err = "CG breakdown (p.Ap or r.z not positive)";
                } else {
                    q.status = BIDO_ERR_NOT_CONVERGED;
                    q.err = "tolerance not reached within max_iter";
                }
            }
            active += !q.done;
        }
        chunk = 1;
    }
    int need = 0;
    for (int i = 0; i < S; ++i) need = std::max(need, sr[i].it);
    F->last_iters = need;
    F->iterations += launched;
    ++F->n_steps;
    return BIDO_OK;
}


}  // namespace

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

const char* bido_last_error(void) { return g_err.c_str(); }

void bido_default_params(bido_params* p) {
    if (!p) return;
    std::memset(p, 0, sizeof(*p));
    p->chi = 200.0;
    p->cm = 1.0;
    p->dt = 0.1;
    p->eps_h = 1e-3;
    p->eta = 2.0;
    p->tol = 1e-10;
    p->leaf = 64;
    p->max_iter = 200;
    p->precision = BIDO_PREC_FP64;
    p->precond = BIDO_PRECOND_PLAIN;
    p->ionic = 0;
    p->n_threads = 0;
    p->scheme = BIDO_SCHEME_EULER;
    p->guess_states = 8;
}

bido_status bido_create(const bido_mesh* mesh, const bido_tissue* tissue, const bido_params* params,
                        void* stream, bido_ctx** out) {
    if (!out) return fail(BIDO_ERR_ARG, "out is null");
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev == 0)
        return fail(BIDO_ERR_DEVICE, "no HIP device available");
    std::unique_ptr<bido_ctx> c(new bido_ctx());
    std::string err;
    if (!build_host(mesh, tissue, params, c->hs, err))
        return fail(err.find("pivot") != std::string::npos ? BIDO_ERR_NOT_SPD : BIDO_ERR_ARG, err);
    HostSetup& hs = c->hs;
    c->params = *params;
    c->precision = params->precision;
    c->stream = (hipStream_t)stream;
    HIP_OK(hipGetDevice(&c->device));
    {
        double* ws = nullptr;                 // the fixed workspace's address on this device
        HIP_OK(noalloc_scratch(c->device, &ws));
    }
    c->N = hs.A.N;
    c->NH = hs.A.NH;
    c->n2 = c->N + c->NH;
    // lanes per row of the sparse products: 2D rows hold ~7 (torso) or ~14
    // (heart) entries, so 4 lanes cover them in the two unconditional passes
    // without a pass of dropped loads (measured: the Lambda product 16.1 ->
    // 13.2 us on thorax200k, 346 -> 281 us on the batch64 union); 3D rows
    // (~15 and ~30 entries) keep 16
    c->spmv_group = hs.A.dim == 2 ? 4 : 16;
    c->heart_ids = hs.A.heart;
    bido_status e;
    if ((e = CsrHostView::up(hs.lam, c->lam))) return e;
    const bool compact = params->amg_columns == 0;
    if ((e = upload_lam_blk(hs, c->lamb, compact))) return e;
    {
        std::vector<int64_t> pos(std::max<int64_t>(c->NH, 1), 0);
        for (int64_t k = 0; k < c->NH; ++k)
            for (int64_t q = hs.lam.ptr[c->N + k]; q < hs.lam.ptr[c->N + k + 1]; ++q)
                if (hs.lam.col[q] == c->N + k) pos[k] = q;
        HIP_OK(upload(&c->lam_vdiag, pos.data(), pos.size()));
    }
    if ((e = CsrHostView::up(hs.avu, c->avu))) return e;
    if ((e = CsrHostView::up(hs.auv, c->auv))) return e;
    if (compact && (e = CsrHostView::compact(hs.avu, c->avu))) return e;
    if (compact && (e = CsrHostView::compact(hs.auv, c->auv))) return e;
    for (auto [src, dst] : {std::pair<const Csr*, float**>{&hs.avu, &c->avu32}, {&hs.auv, &c->auv32}}) {
        std::vector<float> v32(src->val.begin(), src->val.end());
        if (v32.empty()) v32.push_back(0.0f);
        HIP_OK(upload(dst, v32.data(), v32.size()));
    }
    if (hs.p1_factored) {
        if ((e = build_factor_dev(hs.p1, true, c->p1, hs.params.n_threads))) return e;
        hs.p1.trim_top_cache(c->p1.top_h);  // a fused batch reuses hierarchical tops
    } else {
        if ((e = upload_amg(hs.amg1, c->amg1, compact))) return e;
        hs.amg1 = Amg();                    // the device copy is the only one kept
    }
    if (hs.pk_factored) {
        if ((e = build_factor_dev(hs.pk, true, c->pk, hs.params.n_threads))) return e;
        hs.pk.trim_top_cache(c->pk.top_h);
    } else if (params->inner_pk == BIDO_PK_AMG) {
        if ((e = upload_amg(hs.amgk, c->amgk, compact))) return e;
        hs.amgk = Amg();                    // (a time-step change moves it on the device)
        c->pk_kind = BIDO_PK_AMG;
    }
    const int64_t n2 = c->n2;
    for (double** b : {&c->x, &c->r, &c->z, &c->p, &c->q, &c->Y, &c->r_old})
        HIP_OK(hipMalloc((void**)b, n2 * sizeof(double)));
    for (int k = 0; k < params->guess_states; ++k) {
        HIP_OK(hipMalloc((void**)&c->gw[k], n2 * sizeof(double)));
        HIP_OK(hipMalloc((void**)&c->gaw[k], n2 * sizeof(double)));
    }
    if (params->guess_states) {
        HIP_OK(hipMalloc((void**)&c->gG, GUESS_MAX * GUESS_MAX * sizeof(double)));
        HIP_OK(hipMalloc((void**)&c->gd, 3 * GUESS_MAX * sizeof(double)));
        c->gb = c->gd + GUESS_MAX;
        c->gc = c->gd + 2 * GUESS_MAX;
        c->grd.max_blocks = 1024;
        HIP_OK(hipMalloc((void**)&c->grd.partials, (size_t)GUESS_MAX * c->grd.max_blocks * sizeof(double)));
        HIP_OK(hipMalloc((void**)&c->grd.counter, sizeof(unsigned)));
        HIP_OK(hipMemset(c->grd.counter, 0, sizeof(unsigned)));
    }
    for (double** b : {&c->tA, &c->tC, &c->tD}) HIP_OK(hipMalloc((void**)b, c->N * sizeof(double)));
    HIP_OK(hipMalloc((void**)&c->tB, std::max<int64_t>(c->NH, 1) * sizeof(double)));
    if (hs.params.scheme == BIDO_SCHEME_STRANG)
        HIP_OK(hipMalloc((void**)&c->vs, std::max<int64_t>(c->NH, 1) * sizeof(double)));
    HIP_OK(hipMalloc((void**)&c->sc, pp_offset(PP_COUNT) * sizeof(double)));
    // Work vectors start as NaN (all-ones bit pattern): a kernel that reads
    // one before writing it shows up in every result instead of by chance.
    for (double* b : {c->x, c->r, c->z, c->p, c->q, c->Y, c->r_old})
        HIP_OK(hipMemset(b, 0xFF, n2 * sizeof(double)));
    for (double* b : {c->tA, c->tC, c->tD}) HIP_OK(hipMemset(b, 0xFF, c->N * sizeof(double)));
    HIP_OK(hipMemset(c->tB, 0xFF, std::max<int64_t>(c->NH, 1) * sizeof(double)));
    HIP_OK(hipMemset(c->sc, 0xFF, pp_offset(PP_COUNT) * sizeof(double)));
    if (hs.p1_factored) HIP_OK(poison_workspace(c->p1));
    if (hs.pk_factored) HIP_OK(poison_workspace(c->pk));
    HIP_OK(hipHostMalloc((void**)&c->sc_host, pp_offset(PP_COUNT) * sizeof(double), hipHostMallocDefault));
    HIP_OK(hipMalloc((void**)&c->rd.partials, 2 * c->rd.max_blocks * sizeof(double)));
    HIP_OK(hipMalloc((void**)&c->rd.counter, sizeof(unsigned)));
    HIP_OK(hipMemset(c->rd.counter, 0, sizeof(unsigned)));
    HIP_OK(upload(&c->u_pos, hs.u_pos.data(), hs.u_pos.size()));
    HIP_OK(upload(&c->v_pos, hs.v_pos.data(), hs.v_pos.size()));
    HIP_OK(upload(&c->m_int, hs.m_int.data(), hs.m_int.size()));
    HIP_OK(upload(&c->mh_loc, hs.mh_loc.data(), hs.mh_loc.size()));
    HIP_OK(upload(&c->stim_loc, hs.stim_loc.data(), hs.stim_loc.size()));
    HIP_OK(hipEventCreate(&c->ev0));
    HIP_OK(hipEventCreate(&c->ev1));
    HIP_OK(hipEventCreateWithFlags(&c->ev_in, hipEventDisableTiming));
    HIP_OK(hipEventCreateWithFlags(&c->ev_out, hipEventDisableTiming));
    HIP_OK(hipStreamCreateWithFlags(&c->work, hipStreamNonBlocking));
    if ((e = gnn_setup(c.get()))) return e;
    c->precond = params->precond == BIDO_PRECOND_LEARNED_ADDITIVE ? params->precond : BIDO_PRECOND_PLAIN;
    if (params->inner_pk == BIDO_PK_CHEBYSHEV &&
        (e = bido_set_pk(c.get(), BIDO_PK_CHEBYSHEV, 3, 0.0, 0.0)))   // K_m and an estimated interval
        return e;
    HIP_OK(hipDeviceSynchronize());
    *out = c.release();
    return BIDO_OK;
}

void batch_detach(bido_ctx* c);
// A context still in a batch leaves it first (the batch then refuses to run).
void bido_destroy(bido_ctx* ctx) {
    if (ctx && ctx->batch) batch_detach(ctx);
    delete ctx;
}

// ---------------------------------------------------------------------------
// Batched execution of independent slices: every context advances Steps 1-3
// in lockstep.  The slices' launches go to a few streams of the batch (the
// slices are packed onto them by size, largest first), so that small,
// latency-bound slices overlap on the device; the host waits once per PCG
// phase for the whole batch instead of once per slice.
// ---------------------------------------------------------------------------
struct bido_batch {
    std::vector<bido_ctx*> ctx;
    std::vector<hipStream_t> saved;    // the contexts' own streams
    std::vector<hipStream_t> own;      // the batch's streams
    std::vector<hipEvent_t> done;
    hipEvent_t start = nullptr;
    hipStream_t stream = nullptr;      // caller's stream
    std::unique_ptr<FusedBatch> fused; // fused batch (then no own streams)
    std::vector<double*> saved_x, saved_Y;
    // give slot i's context back its own stream and vectors
    void release_slot(size_t i) {
        bido_ctx* c = ctx[i];
        if (!c) return;
        hipStreamSynchronize(c->stream);
        c->stream = saved[i];
        c->batched = false;
        c->batch = nullptr;
        c->drop_graphs();
        if (i < saved_x.size()) {
            c->x = saved_x[i];
            c->Y = saved_Y[i];
        }
        ctx[i] = nullptr;
    }
    ~bido_batch() {
        if (fused) fused->drop_graphs();
        for (size_t i = 0; i < ctx.size(); ++i) release_slot(i);
        fused.reset();
        for (hipStream_t s : own) hipStreamDestroy(s);
        for (hipEvent_t e : done) hipEventDestroy(e);
        if (start) hipEventDestroy(start);
    }
};

void batch_detach(bido_ctx* c) {
    bido_batch* b = c->batch;
    if (b->fused) b->fused->drop_graphs();
    for (size_t i = 0; i < b->ctx.size(); ++i)
        if (b->ctx[i] == c) b->release_slot(i);
}

bido_status bido_batch_create(bido_ctx* const* ctxs, int n_ctx, int n_streams, void* stream,
                              bido_batch** out) {
    if (!ctxs || n_ctx < 1 || !out) return fail(BIDO_ERR_ARG, "null argument or empty batch");
    *out = nullptr;
    for (int i = 0; i < n_ctx; ++i) {
        if (!ctxs[i]) return fail(BIDO_ERR_ARG, "null context");
        if (ctxs[i]->batched) return fail(BIDO_ERR_STATE, "context already in a batch");
        for (int j = 0; j < i; ++j)
            if (ctxs[j] == ctxs[i]) return fail(BIDO_ERR_ARG, "context listed twice");
    }
    auto b = std::make_unique<bido_batch>();
    const int K = n_streams > 0 ? std::min(n_streams, n_ctx) : std::min(n_ctx, 4);
    b->stream = (hipStream_t)stream;
    HIP_OK(hipEventCreateWithFlags(&b->start, hipEventDisableTiming));
    for (int k = 0; k < K; ++k) {
        hipStream_t st;
        HIP_OK(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
        b->own.push_back(st);
        hipEvent_t ev;
        HIP_OK(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
        b->done.push_back(ev);
    }
    // largest slices first, each to the least loaded stream
    std::vector<int> order(n_ctx);
    for (int i = 0; i < n_ctx; ++i) order[i] = i;
    std::sort(order.begin(), order.end(), [&](int a, int c) { return ctxs[a]->n2 > ctxs[c]->n2; });
    std::vector<int64_t> load(K, 0);
    std::vector<int> which(n_ctx);
    for (int i : order) {
        const int k = (int)(std::min_element(load.begin(), load.end()) - load.begin());
        which[i] = k;
        load[k] += ctxs[i]->n2;
    }
    for (int i = 0; i < n_ctx; ++i) {
        b->ctx.push_back(ctxs[i]);
        b->saved.push_back(ctxs[i]->stream);
        ctxs[i]->stream = b->own[which[i]];
        ctxs[i]->batched = true;
        ctxs[i]->batch = b.get();
        ctxs[i]->drop_graphs();
    }
    *out = b.release();
    return BIDO_OK;
}

bido_status bido_batch_create_fused(bido_ctx* const* ctxs, int n_ctx, void* stream, bido_batch** out) {
    if (!ctxs || n_ctx < 1 || !out) return fail(BIDO_ERR_ARG, "null argument or empty batch");
    *out = nullptr;
    for (int i = 0; i < n_ctx; ++i) {
        if (!ctxs[i]) return fail(BIDO_ERR_ARG, "null context");
        if (ctxs[i]->batched) return fail(BIDO_ERR_STATE, "context already in a batch");
        for (int j = 0; j < i; ++j)
            if (ctxs[j] == ctxs[i]) return fail(BIDO_ERR_ARG, "context listed twice");
        // the learned stencil replaces K_m by K_m + C in the slice's P_K
        // tree of the forest; the additive network form stays per context
        const bool stencil = ctxs[i]->precond == BIDO_PRECOND_LEARNED && ctxs[i]->gnn.stencil_ready &&
                             ctxs[i]->pk_learned_host &&
                             ctxs[i]->pk_kind == BIDO_PK_CHOLESKY;
        if ((ctxs[i]->precond != BIDO_PRECOND_PLAIN && !stencil) || ctxs[i]->gnn.collecting)
            return fail(BIDO_ERR_STATE, "a fused batch runs the plain preconditioner or the learned stencil "
                                        "(with the factored P_K)");
        if (ctxs[i]->pk_kind != ctxs[0]->pk_kind ||
            (ctxs[i]->pk_kind == BIDO_PK_CHEBYSHEV && ctxs[i]->cheb_steps != ctxs[0]->cheb_steps))
            return fail(BIDO_ERR_STATE, "a fused batch needs one P_K choice (kind, Chebyshev steps) for all slices");
        if (ctxs[i]->precision != ctxs[0]->precision)
            return fail(BIDO_ERR_STATE, "a fused batch needs one precision for all slices");
        if (!ctxs[i]->hs.p1_factored || !ctxs[i]->hs.pk_factored || ctxs[i]->pk_kind == BIDO_PK_AMG)
            return fail(BIDO_ERR_STATE, "a fused batch sweeps the forest of the slices' factors: every slice "
                                        "needs factored P_1 and K_m");
    }
    auto t0 = std::chrono::steady_clock::now();
    auto b = std::make_unique<bido_batch>();
    b->stream = (hipStream_t)stream;
    HIP_OK(hipEventCreateWithFlags(&b->start, hipEventDisableTiming));
    hipEvent_t ev;
    HIP_OK(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    b->done.push_back(ev);
    auto F = std::make_unique<FusedBatch>();
    const int S = n_ctx;
    F->S = S;
    F->precision = ctxs[0]->precision;
    F->spmv_group = ctxs[0]->spmv_group;
    for (int i = 0; i < n_ctx; ++i) {
        F->precond.push_back(ctxs[i]->precond);
        F->learned = F->learned || ctxs[i]->precond == BIDO_PRECOND_LEARNED;
    }
    int64_t n = 0;
    int big = 0;
    for (int i = 0; i < S; ++i) {
        F->off.push_back(n);
        F->n2.push_back(ctxs[i]->n2);
        n += ctxs[i]->n2;
        if (ctxs[i]->n2 > ctxs[big]->n2) big = i;
        F->spmv_group = std::max(F->spmv_group, ctxs[i]->spmv_group);
    }
    if (n >= INT32_MAX) return fail(BIDO_ERR_ARG, "fused batch too large for 32-bit column indices");
    F->n = n;
    std::vector<const Csr*> lam, avu, auv;
    std::vector<int64_t> o, ou, ov;
    for (int i = 0; i < S; ++i) {
        lam.push_back(&ctxs[i]->hs.lam);
        avu.push_back(&ctxs[i]->hs.avu);
        auv.push_back(&ctxs[i]->hs.auv);
        o.push_back(F->off[i]);
        ov.push_back(F->off[i] + ctxs[i]->N);
    }
    bido_status e;
    if ((e = union_csr(lam, o, o, n, F->lam))) return e;
    if ((e = union_csr(avu, ov, o, n, F->avu))) return e;
    if ((e = union_csr(auv, o, ov, n, F->auv))) return e;
    if (ctxs[0]->pk_kind == BIDO_PK_CHEBYSHEV) {
        const int m = ctxs[0]->cheb_steps;
        std::vector<const Csr*> km;
        std::vector<double> dinv(std::max<int64_t>(n, 1), 0.0);
        std::vector<double> cf((size_t)S * (1 + 2 * (m - 1)));
        for (int i = 0; i < S; ++i) {
            const Csr& K = ctxs[i]->hs.km_int;
            km.push_back(&K);
            for (int64_t r = 0; r < K.n; ++r) {
                double dg = 0.0;
                for (int64_t q = K.ptr[r]; q < K.ptr[r + 1]; ++q)
                    if (K.col[q] == r) dg += K.val[q];
                if (!(dg > 0.0)) return fail(BIDO_ERR_NOT_SPD, "K_m has a non-positive diagonal entry");
                dinv[ov[i] + r] = 1.0 / dg;
            }
            F->nv += K.n;
            const ChebCoef& c = ctxs[i]->cheb;
            cf[i] = c.inv_theta;
            for (int k = 1; k < m; ++k) {
                cf[(size_t)S * (1 + 2 * (k - 1)) + i] = c.c1[k - 1];
                cf[(size_t)S * (2 + 2 * (k - 1)) + i] = c.c2[k - 1];
            }
        }
        if ((e = union_csr(km, ov, ov, n, F->km))) return e;
        HIP_OK(upload(&F->km_dinv, dinv.data(), dinv.size()));
        HIP_OK(upload(&F->cheb, cf.data(), cf.size()));
        for (double** v : {&F->ch_r, &F->ch_d[0], &F->ch_d[1]})
            HIP_OK(hipMalloc((void**)v, std::max<int64_t>(n, 1) * sizeof(double)));
        F->pk_kind = BIDO_PK_CHEBYSHEV;
        F->cheb_steps = m;
    }
    {
        // merged forests; each tree keeps the cut of its own plan (and its
        // hierarchical top), the tiles are those of the largest slice
        std::vector<const Factor*> f1, fk;
        for (int i = 0; i < S; ++i) {
            f1.push_back(&ctxs[i]->hs.p1);
            fk.push_back(&ctxs[i]->hs.pk);
        }
        const bool want32 = F->precision == BIDO_PREC_MIXED;
        const int nth = ctxs[0]->hs.params.n_threads;
        Factor m;
        merge_factors(f1, o, n, m);
        for (int i = 0; i < S; ++i) m.part_top_h[i] = ctxs[i]->p1.top_h;
        // 512 subtrees shared over the union in proportion to the trees'
        // sizes (each tree's cut kept below its top cut) instead of 256 per
        // tree: the union has subtrees enough to fill the device anyway, and
        // bigger ones keep the waves of a workgroup busy (batch64 FP64:
        // 627 -> 802 slice-steps/s); a slice's plan option sub_total > 0
        // (of the largest slice) replaces the 512
        const int sub_total = ctxs[big]->p1.opts.sub_total > 0 ? ctxs[big]->p1.opts.sub_total : 512;
        PlanOptions op = ctxs[big]->p1.opts;
        op.top_h = -1;
        op.sub_h = -1;
        op.sub_total = sub_total;
        if ((e = build_factor_dev(m, want32, F->p1, nth, &op))) return e;
        m = Factor();
        for (int i = 0; i < S; ++i)           // a learned slice brings its factor of K_m + C
            if (ctxs[i]->precond == BIDO_PRECOND_LEARNED) fk[i] = ctxs[i]->pk_learned_host.get();
        merge_factors(fk, ov, n, m);
        for (int i = 0; i < S; ++i)
            m.part_top_h[i] = ctxs[i]->precond == BIDO_PRECOND_LEARNED ? ctxs[i]->pk_learned.top_h : ctxs[i]->pk.top_h;
        op = ctxs[big]->pk.opts;
        op.top_h = -1;
        op.sub_h = -1;
        op.sub_total = sub_total;
        if ((e = build_factor_dev(m, want32, F->pk, nth, &op))) return e;
    }
    {
        std::vector<int64_t> nu, nh, len;
        for (int i = 0; i < S; ++i) {
            nu.push_back(ctxs[i]->N);
            nh.push_back(ctxs[i]->NH);
        }
        std::vector<SegBlock> blk;
        std::vector<SegSlice> sl;
        seg_layout(o, F->n2, o, nu, blk, sl);
        if ((e = seg_upload(F.get(), blk, sl, F->T))) return e;
        F->slices = sl;
        seg_layout(o, nu, o, nu, blk, sl);
        if ((e = seg_upload(F.get(), blk, sl, F->Tu))) return e;
        seg_layout(ov, nh, o, nu, blk, sl);
        if ((e = seg_upload(F.get(), blk, sl, F->Tv))) return e;
    }
    for (double** v : {&F->x, &F->r, &F->z, &F->p, &F->q, &F->Y, &F->tA, &F->tB, &F->tC, &F->tD, &F->r_old}) {
        HIP_OK(hipMalloc((void**)v, std::max<int64_t>(n, 1) * sizeof(double)));
        HIP_OK(hipMemset(*v, 0xFF, std::max<int64_t>(n, 1) * sizeof(double)));
    }
    const int64_t nsc = F->region(FR_COUNT);
    HIP_OK(hipMalloc((void**)&F->sc, nsc * sizeof(double)));
    HIP_OK(hipMemset(F->sc, 0xFF, nsc * sizeof(double)));
    HIP_OK(hipHostMalloc((void**)&F->sc_host, nsc * sizeof(double), hipHostMallocDefault));
    HIP_OK(hipMalloc((void**)&F->done, S));
    HIP_OK(hipHostMalloc((void**)&F->done_host, S, hipHostMallocDefault));
    for (double** b : {&F->yy, &F->tol, &F->rel}) HIP_OK(hipMalloc((void**)b, S * sizeof(double)));
    for (int** b : {&F->max_it, &F->iters, &F->status}) HIP_OK(hipMalloc((void**)b, S * sizeof(int)));
    HIP_OK(hipHostMalloc(&F->back_host, 64 * (((int64_t)S + 63) / 64) + 8 * (((int64_t)2 * S * 4 + 7) / 8) + 8 * S,
                         hipHostMallocDefault));
    for (FactorDev* f : {&F->p1, &F->pk}) {
        HIP_OK(poison_workspace(*f));
    }
    HIP_OK(hipStreamCreateWithFlags(&F->stream, hipStreamNonBlocking));
    HIP_OK(hipMemset(F->done, 0, S));
    F->p1.plan.skip = F->done;         // the sweeps leave frozen slices' trees alone
    F->pk.plan.skip = F->done;
    HIP_OK(hipDeviceSynchronize());
    for (int i = 0; i < S; ++i) {
        bido_ctx* c = ctxs[i];
        b->ctx.push_back(c);
        b->saved.push_back(c->stream);
        b->saved_x.push_back(c->x);
        b->saved_Y.push_back(c->Y);
        c->stream = F->stream;
        c->x = F->x + F->off[i];
        c->Y = F->Y + F->off[i];
        c->batched = true;
        c->batch = b.get();
        c->drop_graphs();
    }
    F->setup_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    b->fused = std::move(F);
    *out = b.release();
    return BIDO_OK;
}

bido_status bido_batch_set_graphs(bido_batch* b, int on) {
    if (!b) return fail(BIDO_ERR_ARG, "null batch");
    if (!b->fused) return fail(BIDO_ERR_STATE, "not a fused batch (its contexts' bido_set_graphs applies)");
    b->fused->drop_graphs();
    b->fused->graphs = on != 0;
    return BIDO_OK;
}

bido_status bido_batch_info(const bido_batch* b, int* fused, int64_t* n_union, double* setup_seconds) {
    if (!b) return fail(BIDO_ERR_ARG, "null batch");
    if (fused) *fused = b->fused ? 1 : 0;
    if (n_union) *n_union = b->fused ? b->fused->n : 0;
    if (setup_seconds) *setup_seconds = b->fused ? b->fused->setup_seconds : 0.0;
    return BIDO_OK;
}

bido_status bido_batch_counters(const bido_batch* b, int64_t* steps, int64_t* iterations, int64_t* host_waits,
                                int64_t* kernels) {
    if (!b) return fail(BIDO_ERR_ARG, "null batch");
    if (!b->fused) return fail(BIDO_ERR_STATE, "not a fused batch");
    const FusedBatch* F = b->fused.get();
    if (steps) *steps = F->n_steps;
    if (iterations) *iterations = F->iterations;
    if (host_waits) *host_waits = F->host_waits;
    if (kernels) *kernels = F->kernels;
    return BIDO_OK;
}

bido_status bido_batch_profile(bido_batch* b, int enable) {
    if (!b) return fail(BIDO_ERR_ARG, "null batch");
    if (!b->fused) return fail(BIDO_ERR_STATE, "only a fused batch has a profiler (profile its contexts instead)");
    FusedBatch* F = b->fused.get();
    HIP_OK(hipStreamSynchronize(F->stream));
    F->prof.recs.clear();
    F->prof.used = 0;
    F->prof.on = enable != 0;
    return BIDO_OK;
}

bido_status bido_batch_profile_read(bido_batch* b, bido_kprof* out, int cap, int* n) {
    if (!b || !n) return fail(BIDO_ERR_ARG, "null argument");
    if (!b->fused) return fail(BIDO_ERR_STATE, "only a fused batch has a profiler");
    HIP_OK(hipStreamSynchronize(b->fused->stream));
    return profile_aggregate(b->fused->prof, out, cap, n);
}

void bido_batch_destroy(bido_batch* b) {
    if (!b) return;
    for (hipStream_t s : b->own) hipStreamSynchronize(s);
    delete b;
}

static bido_status fused_run(bido_batch* b, double* const* v, double* const* w, double* const* u, int64_t n0,
                             int64_t n_steps, bido_stats* per_ctx, bido_stats* total) {
    FusedBatch* F = b->fused.get();
    const int S = (int)b->ctx.size();
    for (int i = 0; i < S; ++i) {
        const bido_ctx* c = b->ctx[i];
        if (c->precond != F->precond[i] || c->precision != F->precision || c->gnn.collecting)
            return fail(BIDO_ERR_STATE, "a slice of the fused batch changed its preconditioner or precision");
    }
    auto t0 = std::chrono::steady_clock::now();
    HIP_OK(hipEventRecord(b->start, b->stream));
    HIP_OK(hipStreamWaitEvent(F->stream, b->start, 0));
    std::vector<SliceRun> sr;
    std::vector<int64_t> tot(S, 0);
    std::vector<int> last_it(S, 0);
    int max_it = 0;
    bido_status err = BIDO_OK;
    std::string err_msg;
    for (int64_t k = 0; k < n_steps && !err; ++k) {
        const int64_t n = n0 + k;
        for (int i = 0; i < S; ++i) step_prepare(b->ctx[i], v[i], w[i], u[i], n);
        const bido_status e = fused_pcg(F, b->ctx, sr);
        if (e) return e;
        for (int i = 0; i < S; ++i) {
            tot[i] += sr[i].it;
            last_it[i] = sr[i].it;
            max_it = std::max(max_it, sr[i].it);
            if (sr[i].status && !err) {
                err = sr[i].status;
                err_msg = "slice " + std::to_string(i) + ": " + sr[i].err;
            }
            if (!sr[i].status || sr[i].status == BIDO_ERR_NOT_CONVERGED) step_write(b->ctx[i], v[i], w[i], u[i]);
        }
    }
    HIP_OK(hipEventRecord(b->done[0], F->stream));
    HIP_OK(hipStreamWaitEvent(b->stream, b->done[0], 0));
    HIP_OK(hipStreamSynchronize(F->stream));
    const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    int64_t all = 0;
    bool all_conv = true;
    double worst = 0.0;
    for (int i = 0; i < S; ++i) {
        all += tot[i];
        const bool conv = !sr.empty() && sr[i].conv;
        all_conv = all_conv && (n_steps == 0 || conv);
        if (!sr.empty()) worst = std::max(worst, sr[i].rel);
        if (per_ctx) {
            std::memset(&per_ctx[i], 0, sizeof(per_ctx[i]));
            per_ctx[i].iterations = last_it[i];
            per_ctx[i].rel_residual = sr.empty() ? 0.0 : sr[i].rel;
            per_ctx[i].converged = conv ? 1 : 0;
            per_ctx[i].total_iterations = tot[i];
            per_ctx[i].ms = ms;
        }
    }
    if (total) {
        std::memset(total, 0, sizeof(*total));
        total->iterations = max_it;
        total->converged = all_conv ? 1 : 0;
        total->rel_residual = worst;
        total->ms = ms;
        total->total_iterations = all;
    }
    return err ? fail(err, err_msg) : BIDO_OK;
}

bido_status bido_batch_run(bido_batch* b, double* const* v, double* const* w, double* const* u, double dt,
                           int64_t n0, int64_t n_steps, bido_stats* per_ctx, bido_stats* total) {
    if (!b || !v || !w || !u || n_steps < 0) return fail(BIDO_ERR_ARG, "null argument");
    const int S = (int)b->ctx.size();
    for (int i = 0; i < S; ++i)
        if (!b->ctx[i]) return fail(BIDO_ERR_STATE, "a context of the batch was destroyed");
    for (int i = 0; i < S; ++i) {
        bido_ctx* c = b->ctx[i];
        if (!v[i] || !w[i] || !u[i]) return fail(BIDO_ERR_ARG, "null state pointer");
        if (!dt_matches(c, dt)) return fail(BIDO_ERR_DT_MISMATCH, "dt differs from the factored time step");
        if (c->precond == BIDO_PRECOND_LEARNED_ADDITIVE)
            return fail(BIDO_ERR_STATE, "the additive learned mode needs a host check inside the apply; "
                                        "not available in a batch");
    }
    if (b->fused) return fused_run(b, v, w, u, n0, n_steps, per_ctx, total);
    auto t0 = std::chrono::steady_clock::now();
    HIP_OK(hipEventRecord(b->start, b->stream));
    for (hipStream_t s : b->own) HIP_OK(hipStreamWaitEvent(s, b->start, 0));
    std::vector<PcgRun> ps(S);
    std::vector<bido_stats> last(S);
    std::vector<int64_t> tot(S, 0);
    std::vector<int> fb(S, 0);
    int max_it = 0;
    bido_status err = BIDO_OK;
    bool all_conv = true;
    double worst = 0.0;
    for (int64_t k = 0; k < n_steps && !err; ++k) {
        const int64_t n = n0 + k;
        for (int i = 0; i < S; ++i) step_begin(b->ctx[i], v[i], w[i], u[i], n, ps[i]);
        for (;;) {
            for (hipStream_t s : b->own) HIP_OK(hipStreamSynchronize(s));
            int active = 0;
            for (int i = 0; i < S; ++i)
                if (!ps[i].done) {
                    pcg_advance(b->ctx[i], ps[i]);
                    active += !ps[i].done;
                }
            if (active == 0) break;
        }
        for (int i = 0; i < S; ++i) {
            const bido_status e = step_end(b->ctx[i], v[i], w[i], u[i], ps[i], &last[i]);
            tot[i] += last[i].iterations;
            fb[i] += last[i].fallbacks;
            max_it = std::max(max_it, last[i].iterations);
            worst = std::max(worst, last[i].rel_residual);
            all_conv = all_conv && last[i].converged;
            if (e && e != BIDO_ERR_NOT_CONVERGED && !err) err = e;
            if (e == BIDO_ERR_NOT_CONVERGED && !err) err = e;
        }
    }
    for (size_t k = 0; k < b->own.size(); ++k) {
        HIP_OK(hipEventRecord(b->done[k], b->own[k]));
        HIP_OK(hipStreamWaitEvent(b->stream, b->done[k], 0));
        HIP_OK(hipStreamSynchronize(b->own[k]));
    }
    const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    int64_t all = 0;
    int all_fb = 0;
    for (int i = 0; i < S; ++i) {
        all += tot[i];
        all_fb += fb[i];
        if (per_ctx) {
            per_ctx[i] = last[i];
            per_ctx[i].total_iterations = tot[i];
            per_ctx[i].fallbacks = fb[i];
            per_ctx[i].ms = ms;
        }
    }
    if (total) {
        std::memset(total, 0, sizeof(*total));
        total->iterations = max_it;
        total->converged = all_conv ? 1 : 0;
        total->rel_residual = worst;
        total->ms = ms;
        total->fallbacks = all_fb;
        total->total_iterations = all;
    }
    return err;
}

bido_status bido_get_info(const bido_ctx* c, bido_info* info) {
    if (!c || !info) return fail(BIDO_ERR_ARG, "null argument");
    std::memset(info, 0, sizeof(*info));
    info->n_nodes = c->N;
    info->n_heart = c->NH;
    info->n_elems = 0;
    info->nnz_lambda = c->lam.nnz;
    // one Lambda product: values + columns + row pointers + x read + y write
    // (the blocked form when there is one)
    info->bytes_lambda = c->lamb.on() ? (int64_t)blk_bytes(c->lamb, 0)
                                      : c->lam.nnz * 12 + (c->n2 + 1) * 8 + c->n2 * 16;
    const int64_t w = c->precision == BIDO_PREC_MIXED ? 4 : 8;
    info->bytes_p1 = c->p1.panel_entries * w + c->p1.meta_bytes;
    info->bytes_pk = c->pk.panel_entries * w + c->pk.meta_bytes;
    info->dense_bytes_p1 = c->p1.dense_entries * 8;
    info->dense_bytes_pk = c->pk.dense_entries * 8;
    info->levels_p1 = c->p1.height + 1;
    info->levels_pk = c->pk.height + 1;
    info->launches_per_sweep_p1 = (int)c->p1.top.size() + (c->p1.plan.n_sub > 0);
    info->launches_per_sweep_pk = (int)c->pk.top.size() + (c->pk.plan.n_sub > 0);
    info->lowrank_blocks = c->p1.top_lowrank + c->pk.top_lowrank;
    info->setup_seconds = c->hs.setup_seconds + c->p1.top_seconds + c->pk.top_seconds;
    info->ground_index = (int)c->hs.p1.ground;
    if (c->amg1.on()) {
        info->bytes_p1 = (int64_t)c->amg1.bytes(c->precision == BIDO_PREC_MIXED ? 4 : 8);
        info->levels_p1 = (int)c->amg1.lv.size();
        info->launches_per_sweep_p1 = 0;
    }
    if (c->amgk.on()) {
        info->bytes_pk = (int64_t)c->amgk.bytes(c->precision == BIDO_PREC_MIXED ? 4 : 8);
        info->levels_pk = (int)c->amgk.lv.size();
        info->launches_per_sweep_pk = 0;
    }
    return BIDO_OK;
}

bido_status bido_heart_nodes(const bido_ctx* c, const int64_t** ids, int64_t* n_h) {
    if (!c || !ids || !n_h) return fail(BIDO_ERR_ARG, "null argument");
    *ids = c->heart_ids.data();
    *n_h = (int64_t)c->heart_ids.size();
    return BIDO_OK;
}

bido_status bido_set_precision(bido_ctx* c, int precision) {
    if (!c) return fail(BIDO_ERR_ARG, "null context");
    if (precision != BIDO_PREC_FP64 && precision != BIDO_PREC_MIXED)
        return fail(BIDO_ERR_ARG, "bad precision");
    c->precision = precision;
    return BIDO_OK;
}

bido_status bido_profile(bido_ctx* c, int enable) {
    if (!c) return fail(BIDO_ERR_ARG, "null context");
    HIP_OK(hipStreamSynchronize(c->stream));
    c->prof.recs.clear();
    c->prof.used = 0;
    c->prof.on = enable != 0;
    return BIDO_OK;
}


bido_status bido_profile_read(bido_ctx* c, bido_kprof* out, int cap, int* n) {
    if (!c || !n) return fail(BIDO_ERR_ARG, "null argument");
    HIP_OK(hipStreamSynchronize(c->stream));
    return profile_aggregate(c->prof, out, cap, n);
}

bido_status bido_inner_solve(bido_ctx* c, int which, const double* b, double* x) {
    if (!c || !b || !x || (which != 0 && which != 1)) return fail(BIDO_ERR_ARG, "bad argument");
    if (which == 0) p1_solve(c, b, x);
    else pk_solve(c, b, x);
    HIP_OK(hipGetLastError());
    HIP_OK(hipStreamSynchronize(c->stream));
    return BIDO_OK;
}

// The same apply with every work array of the sweeps (the intermediate y,
// the update workspace, the partial sums of split tiles, the top's gathered
// vector and projections; the Chebyshev P_K's three vectors) carved from the
// fixed per-GPU workspace instead of the context's own buffers.  Allocates
// nothing; clears the one entry that must start at zero (the update
// workspace's constant 0.0) with a fill kernel.  Calls on one GPU share the
// workspace: overlapping calls race.
bido_status bido_inner_solve_noalloc(bido_ctx* c, int which, const double* b, double* x, int64_t* need) {
    if (!c || !b || !x || (which != 0 && which != 1)) return fail(BIDO_ERR_ARG, "bad argument");
    if ((which == 0 && !c->hs.p1_factored) || (which == 1 && c->pk_kind == BIDO_PK_AMG))
        return fail(BIDO_ERR_STATE, "the allocation-free apply covers the factor sweeps and the Chebyshev P_K");
    const bool cheb = which == 1 && c->pk_kind == BIDO_PK_CHEBYSHEV;
    const FactorDev& src = which == 0 ? c->p1 : c->pk;
    auto up = [](int64_t n) { return (std::max<int64_t>(n, 1) + 31) / 32 * 32; };   // 256-byte slots
    int64_t total = 0;
    if (cheb) total = 3 * up(c->NH);
    else total = up(src.n) + up(src.upd_size) + up(src.scratch_size) + up(src.plan.n_top) + up(src.ht_size);
    if (need) *need = total;
    if (total > NOALLOC_SCRATCH_DOUBLES)
        return fail(BIDO_ERR_RANGE, "inner solve needs " + std::to_string(total) +
                                        " doubles of workspace; the fixed workspace holds " +
                                        std::to_string(NOALLOC_SCRATCH_DOUBLES));
    double* ws = nullptr;
    HIP_OK(noalloc_scratch(c->device, &ws));
    if (cheb) {
        const int64_t m = up(c->NH);
        pk_solve(c, b, x, ws, ws + m, ws + 2 * m);
    } else {
        FactorDev f = src;                         // shallow view: same factor, other workspace
        double* q = ws;
        f.ytmp = q;        q += up(src.n);
        f.upd = q;         q += up(src.upd_size);
        f.plan.scratch = q; q += up(src.scratch_size);
        f.plan.top_w = src.plan.n_top > 0 ? q : nullptr; q += up(src.plan.n_top);
        f.plan.ht = src.ht_size > 0 ? q : nullptr;
        launch_fill(c->stream, 1, f.upd, 0.0);     // the constant 0.0 entry
        inner_solve(c, f, b, x);
    }
    HIP_OK(hipGetLastError());
    HIP_OK(hipStreamSynchronize(c->stream));
    return BIDO_OK;
}

// Interval of the Chebyshev P_K for the current K_m (host Lanczos).
static bido_status estimate_pk_interval(bido_ctx* c, double* lo, double* hi) {
    std::vector<double> gm(c->NH);
    for (int64_t l = 0; l < c->NH; ++l) gm[c->hs.v_pos[l]] = c->hs.gamma * c->hs.mh_loc[l];
    ChebInterval iv;
    std::string err;
    if (!chebyshev_interval(c->hs.km_int, gm, BIDO_PK_LANCZOS_STEPS, iv, err)) return fail(BIDO_ERR_ARG, err);
    *lo = iv.lo;
    *hi = iv.hi;
    return BIDO_OK;
}

bido_status bido_set_pk(bido_ctx* c, int kind, int steps, double lo, double hi) {
    if (!c) return fail(BIDO_ERR_ARG, "null context");
    if (kind != BIDO_PK_CHOLESKY && kind != BIDO_PK_CHEBYSHEV && kind != BIDO_PK_AMG)
        return fail(BIDO_ERR_ARG, "bad P_K kind");
    if (c->batched) return fail(BIDO_ERR_STATE, "context is in a batch");
    if (kind == BIDO_PK_CHOLESKY && !c->hs.pk_factored)
        return fail(BIDO_ERR_STATE, "K_m was not factored (inner_pk at create)");
    if (kind == BIDO_PK_AMG && !c->amgk.on())
        return fail(BIDO_ERR_STATE, "no multigrid hierarchy of K_m (inner_pk = BIDO_PK_AMG at create)");
    HIP_OK(hipStreamSynchronize(c->stream));
    c->drop_graphs();
    if (kind == BIDO_PK_CHOLESKY || kind == BIDO_PK_AMG) {
        c->pk_kind = kind;
        return BIDO_OK;
    }
    if (steps < 1 || steps > BIDO_PK_MAX_STEPS) return fail(BIDO_ERR_ARG, "Chebyshev steps out of range");
    if (!(lo >= 0.0) || !(hi >= 0.0) || (lo == 0.0) != (hi == 0.0) || (lo > 0.0 && !(hi > lo)))
        return fail(BIDO_ERR_ARG, "bad Chebyshev interval (0 < lo < hi, or both 0 to estimate)");
    const Csr& K = c->hs.km_int;
    if (K.n != c->NH) return fail(BIDO_ERR_STATE, "K_m is not available");
    const bool estimate = lo == 0.0;
    if (estimate) {
        if (bido_status e = estimate_pk_interval(c, &lo, &hi)) return e;
    }
    if (!c->km.ptr && c->NH > 0) {
        if (bido_status e = CsrHostView::up(K, c->km)) return e;
        std::vector<double> dinv(c->NH, 0.0);
        for (int64_t i = 0; i < c->NH; ++i)
            for (int64_t p = K.ptr[i]; p < K.ptr[i + 1]; ++p)
                if (K.col[p] == i) dinv[i] += K.val[p];
        for (auto& x : dinv) {
            if (!(x > 0.0)) return fail(BIDO_ERR_NOT_SPD, "K_m has a non-positive diagonal entry");
            x = 1.0 / x;
        }
        HIP_OK(upload(&c->km_dinv, dinv.data(), dinv.size()));
        for (double** b : {&c->ch_r, &c->ch_d[0], &c->ch_d[1]}) HIP_OK(hipMalloc((void**)b, c->NH * sizeof(double)));
    }
    c->pk_kind = kind;
    c->cheb_steps = steps;
    c->cheb_lo = lo;
    c->cheb_hi = hi;
    c->cheb_auto = estimate;
    c->cheb = chebyshev_coefficients(lo, hi, steps);
    return BIDO_OK;
}

// Device side of a time-step change (the host state is already updated):
// Lambda's values, the K_m factor or the Chebyshev P_K's copies, and the
// learned correction set up again.
// One dot product on the device, read back (set-up paths only: it waits).
static bido_status device_dot(bido_ctx* c, int64_t n, const double* a, const double* b, double* out) {
    launch_dot_reduce(c->stream, n, a, b, c->rd, c->sc + S_LZ);
    HIP_OK(hipMemcpyAsync(out, c->sc + S_LZ, sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIP_OK(hipStreamSynchronize(c->stream));
    return BIDO_OK;
}

// The largest eigenvalue of D^-1 A of a level by the host's Lanczos estimate
// (same start vector, same steps, same recurrence), run on the device with
// the level's work vectors.
static bido_status device_lambda_max(bido_ctx* c, const AmgDev& M, AmgDev::Lev& L, double* lmax) {
    hipStream_t s = c->stream;
    const int64_t n = L.n;
    std::vector<double> dinv(n), v0;
    HIP_OK(hipMemcpy(dinv.data(), L.dinv, n * sizeof(double), hipMemcpyDeviceToHost));
    if (!lanczos_start(dinv, v0)) {
        *lmax = 1.0;
        return BIDO_OK;
    }
    double *v = L.x, *vp = L.r, *w = L.xp, *t = L.d0, *y = L.d1;
    HIP_OK(hipMemcpy(v, v0.data(), n * sizeof(double), hipMemcpyHostToDevice));
    launch_fill(s, n, vp, 0.0);
    const AmgMat<double> A = L.mat<double>(L.A, L.A32, L.gA);
    std::vector<double> al, be;
    double beta = 0.0;
    const int steps = (int)std::min<int64_t>(M.lanczos_steps, n);
    for (int j = 0; j < steps; ++j) {
        launch_lz_in(s, n, L.dinv, v, t);
        launch_amg_spmv<double>(s, A, t, (const double*)nullptr, 1.0, y);
        launch_lz_w(s, n, L.dinv, y, beta, vp, w);
        double a = 0.0, b = 0.0;
        if (bido_status e = device_dot(c, n, w, v, &a)) return e;
        launch_axpy(s, n, -a, v, w);
        if (bido_status e = device_dot(c, n, w, w, &b)) return e;
        al.push_back(a);
        b = std::sqrt(b);
        if (j + 1 == steps || b <= 1e-14 * std::fabs(a)) break;
        be.push_back(b);
        beta = b;
        launch_lz_next(s, n, w, 1.0 / b, v, vp);
    }
    *lmax = tridiag_largest(al, be);
    return BIDO_OK;
}

// A new gamma for a multigrid hierarchy of K_m, on the device: every level's
// matrix moves by (gamma' - gamma) times its Galerkin mass part (FP64 and
// FP32 copies), then D^-1, the smoother's column-scaled copy, the smoother
// interval (the host's Lanczos estimate) and the coarsest inverse (Gauss-
// Jordan, one pivot per launch).  The aggregation and the transfer
// operators stay.
static bido_status amg_refresh_device(bido_ctx* c, AmgDev& M, double gamma) {
    if (!M.refreshable()) return fail(BIDO_ERR_STATE, "multigrid hierarchy without mass parts");
    hipStream_t s = c->stream;
    const double dg = gamma - M.gamma;
    for (size_t l = 0; l < M.lv.size(); ++l) {
        AmgDev::Lev& L = M.lv[l];
        const bool last = l + 1 == M.lv.size();
        const int64_t excl = l == 0 ? M.excluded : -1;
        launch_amg_shift(s, L.nnz_A, dg, L.mass, L.A.val, last ? nullptr : L.A32);
        if (last) {
            launch_amg_dense_inverse(s, L.n, L.A.ptr, L.A.col, L.A.val, excl, M.cinv, L.x);
            break;
        }
        launch_amg_dinv(s, L.n, L.A.ptr, L.A.col, L.A.val, excl, L.dinv, L.dinv32);
        launch_amg_colscale(s, L.nnz_A, L.A.col, L.A.val, L.dinv, L.As64, L.As32);
        double lmax = 1.0;
        if (bido_status e = device_lambda_max(c, M, L, &lmax)) return e;
        L.hi = 1.1 * lmax;
        L.lo = L.hi / M.smooth_ratio;
        L.cf = chebyshev_coefficients(L.lo, L.hi, std::max(2, L.steps));
    }
    HIP_OK(hipStreamSynchronize(s));
    M.gamma = gamma;
    return BIDO_OK;
}

static bido_status set_dt_device(bido_ctx* c, bool refactor) {
    // Lambda: only its v-v diagonal changed; its new values go to their
    // positions (and gm of the blocked form)
    {
        const Csr& L = c->hs.lam;
        const int64_t N = c->N, NH = c->NH;
        std::vector<double> dv(NH);
        for (int64_t k = 0; k < NH; ++k)
            for (int64_t q = L.ptr[N + k]; q < L.ptr[N + k + 1]; ++q)
                if (L.col[q] == N + k) dv[k] = L.val[q];
        HIP_OK(hipMemcpy(c->tB, dv.data(), NH * sizeof(double), hipMemcpyHostToDevice));
        launch_scatter_in(c->stream, NH, c->lam_vdiag, c->tB, c->lam.val);
        if (c->lamb.on())
            HIP_OK(hipMemcpyAsync(c->lamb.gm, c->hs.lamb.gm.data(), c->lamb.n * sizeof(double),
                                  hipMemcpyHostToDevice, c->stream));
        HIP_OK(hipStreamSynchronize(c->stream));
    }
    if (c->amgk.on())      // (also when another P_K is active: kept at the current gamma)
        if (bido_status e = amg_refresh_device(c, c->amgk, c->hs.gamma)) return e;
    if (refactor && c->pk_kind == BIDO_PK_CHOLESKY) {
        const PlanOptions opts = c->pk.opts;
        c->pk.release();
        if (bido_status e = build_factor_dev(c->hs.pk, true, c->pk, c->hs.params.n_threads, &opts)) return e;
        c->hs.pk.trim_top_cache(c->pk.top_h);
        HIP_OK(poison_workspace(c->pk));
    }
    if (c->km.ptr) {      // the Chebyshev P_K's copy of K_m and its inverse diagonal
        const Csr& K = c->hs.km_int;
        HIP_OK(hipMemcpy(c->km.val, K.val.data(), K.val.size() * sizeof(double), hipMemcpyHostToDevice));
        std::vector<double> dinv(c->NH, 0.0);
        for (int64_t i = 0; i < c->NH; ++i)
            for (int64_t p = K.ptr[i]; p < K.ptr[i + 1]; ++p)
                if (K.col[p] == i) dinv[i] += K.val[p];
        for (auto& x : dinv) x = 1.0 / x;
        HIP_OK(hipMemcpy(c->km_dinv, dinv.data(), dinv.size() * sizeof(double), hipMemcpyHostToDevice));
    }
    if (c->pk_kind == BIDO_PK_CHEBYSHEV && c->cheb_auto) {
        if (bido_status e = estimate_pk_interval(c, &c->cheb_lo, &c->cheb_hi)) return e;
        c->cheb = chebyshev_coefficients(c->cheb_lo, c->cheb_hi, c->cheb_steps);
    }
    // the learned correction (samples, loss weight, stencil and its factor)
    // was fitted to K_m at the old step: set it up again from scratch
    if (c->pk_learned.nodes) c->pk_learned.release();
    c->pk_learned_host.reset();
    c->amgk_learned.release();
    if (bido_status e = gnn_new_step(c)) return e;
    c->precond = BIDO_PRECOND_PLAIN;
    HIP_OK(hipDeviceSynchronize());
    return BIDO_OK;
}

bido_status bido_set_dt(bido_ctx* c, double dt, double* seconds) {
    if (!c) return fail(BIDO_ERR_ARG, "null context");
    if (!(dt > 0.0) || !std::isfinite(dt)) return fail(BIDO_ERR_ARG, "dt must be > 0");
    if (c->batched) return fail(BIDO_ERR_STATE, "context is in a batch");
    auto t0 = std::chrono::steady_clock::now();
    HIP_OK(hipStreamSynchronize(c->stream));
    if (seconds) *seconds = 0.0;
    if (dt_matches(c, dt)) return BIDO_OK;
    // the factored K_m is factored again on the host; a multigrid K_m moves
    // to the new gamma on the device (amg_refresh_device), the host copy of
    // its hierarchy is not kept
    const bool refactor = c->pk_kind == BIDO_PK_CHOLESKY;
    std::string err;
    if (!host_set_dt(c->hs, dt, refactor, err)) return fail(BIDO_ERR_NOT_SPD, err);
    // from here on the host state is at the new step: a failure below leaves
    // the context refusing every step (dt NaN) until a later call succeeds
    c->params.dt = std::nan("");
    c->drop_graphs();
    c->g_n = -2;                  // the states of another dt leave the projection
    bido_status e = set_dt_device(c, refactor);
    if (e) return e;
    c->params.dt = dt;
    if (seconds) *seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    return BIDO_OK;
}

bido_status bido_record(bido_ctx* c, double v_act, int n_probes, const double* xyz, int64_t max_steps) {
    if (!c) return fail(BIDO_ERR_ARG, "null context");
    if (n_probes < 0 || (n_probes > 0 && (!xyz || max_steps < 1)) || max_steps < 0)
        return fail(BIDO_ERR_ARG, "bad probe arguments");
    if (std::isinf(v_act)) return fail(BIDO_ERR_ARG, "v_act must be finite (or NaN for none)");
    if (c->batched) return fail(BIDO_ERR_STATE, "context is in a batch");
    if ((int64_t)n_probes * std::max<int64_t>(max_steps, 1) > (int64_t)1 << 31)
        return fail(BIDO_ERR_ARG, "recording too large");
    const int dim = c->hs.A.dim, nv = dim + 1;
    std::vector<int64_t> ids;
    std::vector<double> wts;
    std::string err;
    if (n_probes > 0 && !locate_points(dim, c->hs.xyz, c->hs.elems, xyz, n_probes, ids, wts, err))
        return fail(BIDO_ERR_ARG, err);
    HIP_OK(hipStreamSynchronize(c->stream));
    auto& rec = c->rec;
    rec.release();
    rec.v_act = v_act;
    rec.act_on = !std::isnan(v_act);
    if (rec.act_on && c->NH > 0) {
        HIP_OK(hipMalloc((void**)&rec.act, c->NH * sizeof(double)));
        launch_fill(c->stream, c->NH, rec.act, -1.0);
    }
    rec.np = n_probes;
    rec.nv = nv;
    if (n_probes > 0) {
        HIP_OK(upload(&rec.ids, ids.data(), ids.size()));
        HIP_OK(upload(&rec.wts, wts.data(), wts.size()));
        HIP_OK(hipMalloc((void**)&rec.rows, (size_t)n_probes * max_steps * sizeof(double)));
        launch_fill(c->stream, (int64_t)n_probes * max_steps, rec.rows, std::nan(""));
    }
    rec.max_steps = n_probes > 0 ? max_steps : 0;
    rec.on = rec.act_on || n_probes > 0;
    HIP_OK(hipStreamSynchronize(c->stream));
    return BIDO_OK;
}

bido_status bido_record_read(bido_ctx* c, double* act, double* probes, int64_t* n_rows) {
    if (!c) return fail(BIDO_ERR_ARG, "null context");
    const auto& rec = c->rec;
    HIP_OK(hipStreamSynchronize(c->stream));
    if (act) {
        if (!rec.act_on) return fail(BIDO_ERR_STATE, "no activation times are being recorded");
        HIP_OK(hipMemcpy(act, rec.act, c->NH * sizeof(double), hipMemcpyDeviceToHost));
    }
    if (probes && rec.np > 0 && rec.n_rows > 0)
        HIP_OK(hipMemcpy(probes, rec.rows, (size_t)rec.n_rows * rec.np * sizeof(double), hipMemcpyDeviceToHost));
    if (n_rows) *n_rows = rec.n_rows;
    return BIDO_OK;
}

bido_status bido_get_pk(const bido_ctx* c, int* kind, int* steps, double* lo, double* hi) {
    if (!c) return fail(BIDO_ERR_ARG, "null context");
    if (kind) *kind = c->pk_kind;
    if (steps) *steps = c->pk_kind == BIDO_PK_CHEBYSHEV ? c->cheb_steps : 0;
    if (lo) *lo = c->pk_kind == BIDO_PK_CHEBYSHEV ? c->cheb_lo : 0.0;
    if (hi) *hi = c->pk_kind == BIDO_PK_CHEBYSHEV ? c->cheb_hi : 0.0;
    return BIDO_OK;
}

bido_status bido_reset_guess(bido_ctx* c) {
    if (!c) return fail(BIDO_ERR_ARG, "null context");
    c->g_n = -2;
    c->g_len = 0;
    return BIDO_OK;
}

bido_status bido_set_precond(bido_ctx* c, int precond) {
    if (!c) return fail(BIDO_ERR_ARG, "null context");
    if (precond != BIDO_PRECOND_PLAIN && precond != BIDO_PRECOND_LEARNED &&
        precond != BIDO_PRECOND_LEARNED_ADDITIVE)
        return fail(BIDO_ERR_ARG, "bad precond");
    if (precond == BIDO_PRECOND_LEARNED && !c->gnn.stencil_ready)
        return fail(BIDO_ERR_STATE, "the learned stencil has not been trained (or K_m + C was not SPD)");
    if (c->batch && c->batch->fused && precond != c->precond)
        return fail(BIDO_ERR_STATE, "context belongs to a fused batch (its preconditioner is fixed there)");
    c->precond = precond;
    return BIDO_OK;
}

bido_status bido_learn_collect(bido_ctx* c, double* v, double* w, double* u, double dt, int64_t n0,
                               int64_t n_steps, int max_samples, bido_stats* st) {
    if (!c || max_samples < 1) return fail(BIDO_ERR_ARG, "bad argument");
    if (c->batched) return fail(BIDO_ERR_STATE, "context is in a batch");
    GnnState& g = c->gnn;
    if (max_samples > g.max_samples) {
        hipStreamSynchronize(c->stream);
        auto grow = [&](float** buf) -> bido_status {
            float* nb = nullptr;
            HIP_OK(hipMalloc((void**)&nb, (size_t)max_samples * std::max<int64_t>(c->NH, 1) * sizeof(float)));
            if (g.n_samples > 0)
                HIP_OK(hipMemcpy(nb, *buf, (size_t)g.n_samples * c->NH * sizeof(float), hipMemcpyDeviceToDevice));
            hipFree(*buf);
            *buf = nb;
            return BIDO_OK;
        };
        auto growd = [&](double** buf) -> bido_status {
            double* nb = nullptr;
            HIP_OK(hipMalloc((void**)&nb, (size_t)max_samples * sizeof(double)));
            if (g.n_samples > 0)
                HIP_OK(hipMemcpy(nb, *buf, (size_t)g.n_samples * sizeof(double), hipMemcpyDeviceToDevice));
            hipFree(*buf);
            *buf = nb;
            return BIDO_OK;
        };
        bido_status e1;
        for (float** b : {&g.s_t, &g.s_y, &g.s_z, &g.s_b})
            if ((e1 = grow(b))) return e1;
        for (double** b : {&g.s_tn2, &g.s_zz})
            if ((e1 = growd(b))) return e1;
        g.max_samples = max_samples;
    }
    for (double** b : {&g.pend, &g.pend_t, &g.pend_v})
        if (!*b) HIP_OK(hipMalloc((void**)b, (size_t)g.max_pending * std::max<int64_t>(c->NH, 1) * sizeof(double)));
    // with a multigrid P_1 the Schur right-hand side of a PCG iterate is not
    // exact, so the stencil pairs come from consecutive converged steps
    g.increments = !c->hs.p1_factored;
    if (g.increments) {
        for (double** b : {&g.inc_v, &g.inc_y})
            if (!*b) HIP_OK(hipMalloc((void**)b, std::max<int64_t>(c->NH, 1) * sizeof(double)));
        g.inc_ok = false;
    }
    g.collecting = true;
    g.n_pending = 0;
    bido_status e = bido_run(c, v, w, u, dt, n0, n_steps, st);
    g.collecting = false;
    return e;
}

bido_status bido_learn_samples(const bido_ctx* c, int* n_samples) {
    if (!c || !n_samples) return fail(BIDO_ERR_ARG, "null argument");
    *n_samples = c->gnn.n_samples;
    return BIDO_OK;
}

static bido_status train_additive(bido_ctx* c, int epochs, int batch, float lr, uint64_t seed, int n_val,
                                  bido_train_stats* ts) {
    GnnState& g = c->gnn;
    const int n_tr = g.n_samples - n_val;
    hipStream_t s = c->stream;
    const int64_t NH = c->NH;
    auto t0 = std::chrono::steady_clock::now();
    double hl[4];
    // loss of the zero correction on the training and validation sets; the
    // network learns targets in units of their RMS per vertex (out_scale)
    HIP_OK(hipMemsetAsync(g.dloss, 0, 4 * sizeof(double), s));
    for (int k = 0; k < g.n_samples; ++k)
        launch_gnn_sumsq(s, NH, g.s_y + (int64_t)k * NH, g.partials, g.dloss + (k < n_tr ? 0 : 1));
    HIP_OK(hipMemcpyAsync(hl, g.dloss, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_OK(hipStreamSynchronize(s));
    const double rms = std::sqrt(hl[0] / ((double)n_tr * std::max<int64_t>(NH, 1)));
    g.out_scale = rms > 0 ? (float)rms : 1.0f;
    const float yinv = 1.0f / g.out_scale;
    HIP_OK(hipMemsetAsync(g.dloss, 0, 2 * sizeof(double), s));
    for (int k = 0; k < g.n_samples; ++k)
        launch_gnn_energy0(s, NH, g.s_y + (int64_t)k * NH, g.Wk, g.act, g.partials,
                           g.dloss + (k < n_tr ? 0 : 1), yinv);
    auto eval = [&](int k0, int k1, double* dst) {
        for (int k = k0; k < k1; ++k) {
            launch_gnn_forward_sample(s, NH, g.s_t + (int64_t)k * NH, g.stat, g.A, g.wbf, g.act);
            launch_gnn_loss(s, NH, g.s_y + (int64_t)k * NH, g.Wk, g.act, g.partials, dst, yinv);
        }
    };
    HIP_OK(hipMemsetAsync(g.dloss + 2, 0, 2 * sizeof(double), s));
    eval(0, n_tr, g.dloss + 2);
    HIP_OK(hipMemcpyAsync(hl, g.dloss, 4 * sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_OK(hipStreamSynchronize(s));
    if (ts) {
        std::memset(ts, 0, sizeof(*ts));
        ts->samples = g.n_samples;
        ts->train_samples = n_tr;
        ts->loss_zero = hl[0] / n_tr;
        ts->loss_zero_val = n_val ? hl[1] / n_val : 0.0;
        ts->loss_first = hl[2] / n_tr;
    }
    std::mt19937_64 rng(seed);
    std::vector<int> order(n_tr);
    for (int k = 0; k < n_tr; ++k) order[k] = k;
    for (int ep = 0; ep < epochs; ++ep) {
        std::shuffle(order.begin(), order.end(), rng);
        for (int b0 = 0; b0 < n_tr; b0 += batch) {
            const int b1 = std::min(n_tr, b0 + batch);
            HIP_OK(hipMemsetAsync(g.grad, 0, GNN_P * sizeof(float), s));
            for (int q = b0; q < b1; ++q) {
                const int k = order[q];
                launch_gnn_forward_sample(s, NH, g.s_t + (int64_t)k * NH, g.stat, g.A, g.wbf, g.act);
                launch_gnn_backward(s, NH, g.s_y + (int64_t)k * NH, g.Wk, g.At, g.wbf, g.act, g.partials,
                                    g.grad, nullptr, yinv);
            }
            launch_gnn_adam(s, g.theta, g.m, g.v, g.grad, 1.0f / (float)(b1 - b0), lr, ++g.adam_step, g.wbf);
        }
    }
    HIP_OK(hipMemsetAsync(g.dloss, 0, 4 * sizeof(double), s));
    eval(0, n_tr, g.dloss + 2);
    eval(n_tr, g.n_samples, g.dloss + 3);
    HIP_OK(hipMemcpyAsync(hl, g.dloss, 4 * sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_OK(hipStreamSynchronize(s));
    if (ts) {
        ts->epochs = epochs;
        ts->loss_last = hl[2] / n_tr;
        ts->loss_val = n_val ? hl[3] / n_val : 0.0;
        ts->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
    return BIDO_OK;
}

// Learned Schur-complement stencil: regression C z*_k ~ t_k - K_m z*_k over
// the recorded pairs, then the factor of K_m + C replaces P_K in the learned
// mode (the plain factor stays, and is kept if K_m + C is not SPD).
static bido_status train_stencil(bido_ctx* c, int epochs, int batch, float lr, uint64_t seed, int n_val,
                                 bido_train_stats* ts) {
    GnnState& g = c->gnn;
    const int n_tr = g.n_samples - n_val;
    hipStream_t s = c->stream;
    const int64_t NH = c->NH;
    auto t0 = std::chrono::steady_clock::now();
    double hl[4];
    auto eval = [&](int k0, int k1, double* dst, bool zero_c) {
        if (zero_c) HIP_OK(hipMemsetAsync(g.cval, 0, std::max<int64_t>(g.P.nnz, 1) * sizeof(float), s));
        for (int k = k0; k < k1; ++k)
            launch_stencil_sample_loss(s, g.P, g.cval, g.s_z + (int64_t)k * NH, g.s_b + (int64_t)k * NH, g.r,
                                       nullptr, g.partials, dst);
        return BIDO_OK;
    };
    HIP_OK(hipMemsetAsync(g.dloss, 0, 4 * sizeof(double), s));
    eval(0, n_tr, g.dloss + 0, true);
    eval(n_tr, g.n_samples, g.dloss + 1, true);
    launch_gnn_embed(s, NH, g.stat, g.A, g.wbf, g.act);
    launch_stencil_values(s, g.P, g.act.h2, g.wbf, g.cval);
    eval(0, n_tr, g.dloss + 2, false);
    eval(n_tr, g.n_samples, g.dloss + 3, false);
    HIP_OK(hipMemcpyAsync(hl, g.dloss, 4 * sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_OK(hipStreamSynchronize(s));
    // model selection: the weights of the epoch with the lowest held-out
    // loss (training loss without held-out pairs), those before training
    // included
    const int sel0 = n_val > 0 ? n_tr : 0, sel1 = n_val > 0 ? g.n_samples : n_tr;
    double best = n_val > 0 ? hl[3] : hl[2];
    int best_epoch = 0;
    HIP_OK(hipMemcpyAsync(g.theta_best, g.theta, GNN_P * sizeof(float), hipMemcpyDeviceToDevice, s));
    if (ts) {
        std::memset(ts, 0, sizeof(*ts));
        ts->samples = g.n_samples;
        ts->train_samples = n_tr;
        ts->loss_zero = hl[0] / n_tr;
        ts->loss_zero_val = n_val ? hl[1] / n_val : 0.0;
        ts->loss_first = hl[2] / n_tr;
    }
    std::mt19937_64 rng(seed);
    std::vector<int> order(n_tr);
    for (int k = 0; k < n_tr; ++k) order[k] = k;
    for (int ep = 0; ep < epochs; ++ep) {
        std::shuffle(order.begin(), order.end(), rng);
        for (int b0 = 0; b0 < n_tr; b0 += batch) {
            const int b1 = std::min(n_tr, b0 + batch);
            launch_gnn_embed(s, NH, g.stat, g.A, g.wbf, g.act);
            launch_stencil_values(s, g.P, g.act.h2, g.wbf, g.cval);
            HIP_OK(hipMemsetAsync(g.G, 0, std::max<int64_t>(g.P.nnz, 1) * sizeof(float), s));
            for (int q = b0; q < b1; ++q) {
                const int k = order[q];
                launch_stencil_sample_loss(s, g.P, g.cval, g.s_z + (int64_t)k * NH, g.s_b + (int64_t)k * NH,
                                           g.r, g.G, g.partials, g.dloss + 3);
            }
            HIP_OK(hipMemsetAsync(g.grad, 0, GNN_P * sizeof(float), s));
            launch_stencil_backward(s, g.P, g.At, g.G, g.wbf, g.act, g.partials, g.grad);
            launch_gnn_adam(s, g.theta, g.m, g.v, g.grad, 1.0f / (float)(b1 - b0), lr, ++g.adam_step, g.wbf);
        }
        launch_gnn_embed(s, NH, g.stat, g.A, g.wbf, g.act);
        launch_stencil_values(s, g.P, g.act.h2, g.wbf, g.cval);
        HIP_OK(hipMemsetAsync(g.dloss, 0, sizeof(double), s));
        eval(sel0, sel1, g.dloss, false);
        double l = 0.0;
        HIP_OK(hipMemcpyAsync(&l, g.dloss, sizeof(double), hipMemcpyDeviceToHost, s));
        HIP_OK(hipStreamSynchronize(s));
        if (l < best) {
            best = l;
            best_epoch = ep + 1;
            HIP_OK(hipMemcpyAsync(g.theta_best, g.theta, GNN_P * sizeof(float), hipMemcpyDeviceToDevice, s));
        }
    }
    if (best_epoch != epochs) {            // back to the kept weights
        HIP_OK(hipMemcpyAsync(g.theta, g.theta_best, GNN_P * sizeof(float), hipMemcpyDeviceToDevice, s));
        launch_gnn_to_bf16(s, g.theta, g.wbf);
    }
    launch_gnn_embed(s, NH, g.stat, g.A, g.wbf, g.act);
    launch_stencil_values(s, g.P, g.act.h2, g.wbf, g.cval);
    HIP_OK(hipMemsetAsync(g.dloss, 0, 4 * sizeof(double), s));
    eval(0, n_tr, g.dloss + 2, false);
    eval(n_tr, g.n_samples, g.dloss + 3, false);
    std::vector<float> cv(std::max<int64_t>(g.P.nnz, 1));
    HIP_OK(hipMemcpyAsync(hl, g.dloss, 4 * sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_OK(hipMemcpyAsync(cv.data(), g.cval, cv.size() * sizeof(float), hipMemcpyDeviceToHost, s));
    HIP_OK(hipStreamSynchronize(s));
    if (ts) {
        ts->epochs = epochs;
        ts->loss_last = hl[2] / n_tr;
        ts->loss_val = n_val ? hl[3] / n_val : 0.0;
        ts->best_epoch = best_epoch;
    }
    // factor K_m + C on the host and upload it as the learned P_K (without a
    // factored K_m: a multigrid hierarchy of K_m + C instead)
    auto t1 = std::chrono::steady_clock::now();
    Csr Kt = c->hs.km_int;
    for (int64_t p = 0; p < Kt.nnz(); ++p) Kt.val[p] += g.dbar * (double)cv[p];
    Factor f;
    f.tree = c->hs.pk.tree;
    std::string err;
    bool spd = false;
    if (!c->hs.pk_factored) {
        Amg am;
        spd = amg_build(Kt, -1, AmgOptions(), am, err);
        if (spd) {
            if (bido_status e = upload_amg(am, c->amgk_learned, c->params.amg_columns == 0)) return e;
        }
    } else if ((spd = multifrontal(Kt, f, -1, c->params.n_threads, err))) {
        set_top_compression(f, c->hs.pk.xyz.data(), c->hs.pk.dim, c->hs.pk.eps);
        c->pk_learned.release();
        bido_status e = build_factor_dev(f, true, c->pk_learned, c->params.n_threads);
        if (e) return e;
        for (FactorDev* fd : {&c->pk_learned}) {
            HIP_OK(poison_workspace(*fd));
        }
        f.trim_top_cache(c->pk_learned.top_h);
        c->pk_learned_host = std::make_unique<Factor>(std::move(f));
    }
    g.stencil_ready = spd;
    if (ts) {
        ts->spd = spd ? 1 : 0;
        ts->refactor_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t1).count();
        ts->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
    return BIDO_OK;
}

bido_status bido_learn_train(bido_ctx* c, int kind, int epochs, int batch, float lr, uint64_t seed, int n_val,
                             bido_train_stats* ts) {
    if (!c || epochs < 0 || batch < 1 || !(lr > 0)) return fail(BIDO_ERR_ARG, "bad argument");
    if (c->batched) return fail(BIDO_ERR_STATE, "context is in a batch");
    const int n_tr = c->gnn.n_samples - n_val;
    if (n_val < 0 || n_tr < 1) return fail(BIDO_ERR_STATE, "not enough collected samples");
    if (kind == BIDO_LEARN_STENCIL) return train_stencil(c, epochs, batch, lr, seed, n_val, ts);
    if (kind == BIDO_LEARN_ADDITIVE && c->gnn.increments)
        return fail(BIDO_ERR_STATE, "the pairs were collected as step increments (multigrid P_1): stencil only");
    if (kind == BIDO_LEARN_ADDITIVE) return train_additive(c, epochs, batch, lr, seed, n_val, ts);
    return fail(BIDO_ERR_ARG, "unknown learning target");
}

bido_status bido_weights_io(bido_ctx* c, float* buf, int n, int dir) {
    if (!c || !buf || n != GNN_P || (dir != 0 && dir != 1)) return fail(BIDO_ERR_ARG, "bad argument");
    GnnState& g = c->gnn;
    HIP_OK(hipStreamSynchronize(c->stream));
    if (dir == 0) {
        HIP_OK(hipMemcpy(buf, g.theta, GNN_P * sizeof(float), hipMemcpyDeviceToHost));
    } else {
        HIP_OK(hipMemcpy(g.theta, buf, GNN_P * sizeof(float), hipMemcpyHostToDevice));
        HIP_OK(hipMemset(g.m, 0, GNN_P * sizeof(float)));
        HIP_OK(hipMemset(g.v, 0, GNN_P * sizeof(float)));
        g.adam_step = 0;
        launch_gnn_to_bf16(c->stream, g.theta, g.wbf);
        g.out_scale = 1.0f;
        HIP_OK(hipStreamSynchronize(c->stream));
    }
    return BIDO_OK;
}

bido_status bido_gnn_eval(bido_ctx* c, const double* t, double* out) {
    if (!c || !t || !out) return fail(BIDO_ERR_ARG, "null argument");
    hipStream_t s = c->stream;
    GnnState& g = c->gnn;
    const int64_t NH = c->NH;
    launch_scatter_in(s, NH, c->v_pos, t, c->tB);
    launch_dot_reduce(s, NH, c->tB, c->tB, c->rd, c->sc + S_TN2);
    launch_fill(s, NH, g.tz, 0.0);
    launch_gnn_forward(s, NH, c->tB, c->sc + S_TN2, g.stat, g.A, g.wbf, g.act, 0, g.tz, g.out_scale);
    launch_gather_out(s, NH, c->v_pos, g.tz, out, c->sc, -1, 1.0);
    HIP_OK(hipGetLastError());
    HIP_OK(hipStreamSynchronize(s));
    return BIDO_OK;
}

bido_status bido_gnn_loss_grad(bido_ctx* c, const float* that, const float* y, double* loss, float* grad) {
    if (!c || !that || !y || !loss || !grad) return fail(BIDO_ERR_ARG, "null argument");
    hipStream_t s = c->stream;
    GnnState& g = c->gnn;
    const int64_t NH = c->NH;
    launch_scatter_in_f(s, NH, c->v_pos, that, g.ft);
    launch_scatter_in_f(s, NH, c->v_pos, y, g.fy);
    HIP_OK(hipMemsetAsync(g.grad, 0, GNN_P * sizeof(float), s));
    HIP_OK(hipMemsetAsync(g.dloss, 0, sizeof(double), s));
    launch_gnn_forward_sample(s, NH, g.ft, g.stat, g.A, g.wbf, g.act);
    launch_gnn_backward(s, NH, g.fy, g.Wk, g.At, g.wbf, g.act, g.partials, g.grad, g.dloss, 1.0f);
    HIP_OK(hipMemcpyAsync(loss, g.dloss, sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_OK(hipMemcpyAsync(grad, g.grad, GNN_P * sizeof(float), hipMemcpyDeviceToHost, s));
    HIP_OK(hipGetLastError());
    HIP_OK(hipStreamSynchronize(s));
    return BIDO_OK;
}

bido_status bido_stencil_check(bido_ctx* c, const float* zh, const float* bh, float* r, double* loss,
                               float* grad) {
    if (!c || !zh || !bh || !loss) return fail(BIDO_ERR_ARG, "null argument");
    hipStream_t s = c->stream;
    GnnState& g = c->gnn;
    const int64_t NH = c->NH;
    launch_scatter_in_f(s, NH, c->v_pos, zh, g.ft);
    launch_scatter_in_f(s, NH, c->v_pos, bh, g.fy);
    HIP_OK(hipMemsetAsync(g.grad, 0, GNN_P * sizeof(float), s));
    HIP_OK(hipMemsetAsync(g.dloss, 0, sizeof(double), s));
    HIP_OK(hipMemsetAsync(g.G, 0, std::max<int64_t>(g.P.nnz, 1) * sizeof(float), s));
    launch_gnn_embed(s, NH, g.stat, g.A, g.wbf, g.act);
    launch_stencil_values(s, g.P, g.act.h2, g.wbf, g.cval);
    launch_stencil_sample_loss(s, g.P, g.cval, g.ft, g.fy, g.r, g.G, g.partials, g.dloss);
    if (grad) launch_stencil_backward(s, g.P, g.At, g.G, g.wbf, g.act, g.partials, g.grad);
    if (r) launch_gather_f(s, NH, c->v_pos, g.r, r);
    HIP_OK(hipMemcpyAsync(loss, g.dloss, sizeof(double), hipMemcpyDeviceToHost, s));
    if (grad) HIP_OK(hipMemcpyAsync(grad, g.grad, GNN_P * sizeof(float), hipMemcpyDeviceToHost, s));
    HIP_OK(hipGetLastError());
    HIP_OK(hipStreamSynchronize(s));
    return BIDO_OK;
}

// Mean time of one application of factor f over `reps` back-to-back solves
// on the context's stream [ms].
double time_factor(bido_ctx* c, const FactorDev& f, const double* in, double* out, int reps) {
    inner_solve(c, f, in, out);
    hipEventRecord(c->ev0, c->stream);
    for (int r = 0; r < reps; ++r) inner_solve(c, f, in, out);
    hipEventRecord(c->ev1, c->stream);
    hipEventSynchronize(c->ev1);
    float ms = 0.f;
    hipEventElapsedTime(&ms, c->ev0, c->ev1);
    return ms / reps;
}

bido_status bido_autotune(bido_ctx* c, int reps, bido_tune_report* rep) {
    if (!c) return fail(BIDO_ERR_ARG, "null context");
    if (c->batched) return fail(BIDO_ERR_STATE, "context belongs to a batch");
    reps = reps > 0 ? reps : 10;
    auto t0 = std::chrono::steady_clock::now();
    bido_tune_report r{};
    const int nth = c->hs.params.n_threads;
    for (int which = 0; which < 2; ++which) {
        if (!(which == 0 ? c->hs.p1_factored : c->hs.pk_factored)) continue;   // nothing to tune
        FactorDev& cur = which == 0 ? c->p1 : c->pk;
        const Factor& f = which == 0 ? c->hs.p1 : c->hs.pk;
        launch_fill(c->stream, cur.n, c->r, 1.0);
        double best = time_factor(c, cur, c->r, c->z, reps);
        r.us_before[which] = best * 1e3;
        auto attempt = [&](PlanOptions o) {
            FactorDev cand;
            if (build_factor_dev(f, true, cand, nth, &o) == BIDO_OK) {
                ++r.candidates;
                const double ms = time_factor(c, cand, c->r, c->z, reps);
                if (ms < 0.98 * best) {
                    best = ms;
                    std::swap(cur, cand);
                }
            }
            cand.release();
        };
        // the cut first, with the present tiles; then the tiles at the best cut
        const PlanOptions start = cur.opts;
        for (int d : {-2, -1, 1, 2}) {
            PlanOptions o = start;
            o.top_h = start.top_h + d;
            if (o.top_h >= 0) attempt(o);
        }
        const PlanOptions at = cur.opts;
        for (int fc : {64, 128, 256})
            for (int wide : {1, 0})
                for (int br : {0, wide ? 1024 : 256}) {
                    PlanOptions o = at;
                    o.fwd_cols = fc;
                    o.bwd_rows = br;
                    o.bwd_wide = wide;
                    if (o.fwd_cols == at.fwd_cols && o.bwd_rows == at.bwd_rows && o.bwd_wide == at.bwd_wide) continue;
                    attempt(o);
                }
        f.trim_top_cache(cur.top_h);
        HIP_OK(poison_workspace(cur));
        r.us_after[which] = best * 1e3;
        r.top_h[which] = cur.opts.top_h;
        r.fwd_cols[which] = cur.opts.fwd_cols;
        r.bwd_rows[which] = cur.opts.bwd_rows;
    }
    c->drop_graphs();
    HIP_OK(hipStreamSynchronize(c->stream));
    r.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (rep) *rep = r;
    return BIDO_OK;
}

void bido_default_plan(bido_plan* q) {
    if (!q) return;
    *q = bido_plan{};
    q->top_h = -1;
    q->bwd_wide = -1;
    q->level_items = -1;
    q->sub_h = -1;
}

bido_status bido_set_plan(bido_ctx* c, int which, const bido_plan* q) {
    if (!c || !q) return fail(BIDO_ERR_ARG, "null argument");
    if (which != 0 && which != 1) return fail(BIDO_ERR_ARG, "unknown factor");
    if (q->spmv_group != 0 && q->spmv_group != 4 && q->spmv_group != 8 && q->spmv_group != 16 &&
        q->spmv_group != 32)
        return fail(BIDO_ERR_ARG, "spmv_group must be 4, 8, 16 or 32");
    if (c->batched) return fail(BIDO_ERR_STATE, "context belongs to a batch");
    if (!(which == 0 ? c->hs.p1_factored : c->hs.pk_factored))
        return fail(BIDO_ERR_STATE, "that block is not factored (inner_p1 / inner_pk at create)");
    HIP_OK(hipStreamSynchronize(c->stream));
    c->drop_graphs();
    PlanOptions o;
    o.top_h = q->top_h;
    o.fwd_cols = q->fwd_cols;
    o.bwd_rows = q->bwd_rows;
    o.bwd_wide = q->bwd_wide;
    o.level_items = q->level_items;
    o.sub_h = q->sub_h;
    o.sub_want = q->sub_want;
    o.sub_total = q->sub_total;
    o.bwd_group_max = q->bwd_group_max;
    FactorDev& cur = which == 0 ? c->p1 : c->pk;
    const Factor& f = which == 0 ? c->hs.p1 : c->hs.pk;
    FactorDev cand;
    bido_status e = build_factor_dev(f, true, cand, c->hs.params.n_threads, &o);
    if (e != BIDO_OK) {
        cand.release();
        return e;
    }
    std::swap(cur, cand);
    cand.release();
    f.trim_top_cache(cur.top_h);
    HIP_OK(poison_workspace(cur));
    if (q->spmv_group) c->spmv_group = q->spmv_group;
    HIP_OK(hipStreamSynchronize(c->stream));
    return BIDO_OK;
}

bido_status bido_get_plan(const bido_ctx* c, int which, bido_plan* q) {
    if (!c || !q) return fail(BIDO_ERR_ARG, "null argument");
    if (which != 0 && which != 1) return fail(BIDO_ERR_ARG, "unknown factor");
    const PlanOptions& o = (which == 0 ? c->p1 : c->pk).opts;
    bido_default_plan(q);
    q->top_h = o.top_h;
    q->fwd_cols = o.fwd_cols;
    q->bwd_rows = o.bwd_rows;
    q->bwd_wide = o.bwd_wide;
    q->level_items = o.level_items;
    q->sub_h = o.sub_h;
    q->sub_want = o.sub_want;
    q->sub_total = o.sub_total;
    q->bwd_group_max = o.bwd_group_max;
    q->spmv_group = c->spmv_group;
    return BIDO_OK;
}

bido_status bido_set_graphs(bido_ctx* c, int on) {
    if (!c) return fail(BIDO_ERR_ARG, "null context");
    c->drop_graphs();
    c->graph_mode = on < 0 ? -1 : (on != 0);
    return BIDO_OK;
}

bido_status bido_set_solver(bido_ctx* c, double tol, int max_iter) {
    if (!c) return fail(BIDO_ERR_ARG, "null context");
    if (tol > 0) c->params.tol = tol;
    if (max_iter > 0) c->params.max_iter = max_iter;
    return BIDO_OK;
}

bido_status bido_step(bido_ctx* c, double* v, double* w, double* u, double dt, int64_t n,
                      bido_stats* st) {
    return bido_run(c, v, w, u, dt, n, 1, st);
}

bido_status bido_run(bido_ctx* c, double* v, double* w, double* u, double dt, int64_t n0,
                     int64_t n_steps, bido_stats* st) {
    if (!c || !v || !w || !u || n_steps < 0) return fail(BIDO_ERR_ARG, "null argument");
    if (!dt_matches(c, dt))
        return fail(BIDO_ERR_DT_MISMATCH, "dt differs from the factored time step");
    bido_stats local{};
    auto t0 = std::chrono::steady_clock::now();
    // steps run on the context's own (capturable) stream, ordered after and
    // before the caller's stream by events
    hipStream_t user = c->stream;
    if (!c->batched) {
        HIP_OK(hipEventRecord(c->ev_in, user));
        HIP_OK(hipStreamWaitEvent(c->work, c->ev_in, 0));
        c->stream = c->work;
    }
    HIP_OK(hipEventRecord(c->ev0, c->stream));
    bido_status e = BIDO_OK;
    int64_t total = 0;
    int fb = 0;
    for (int64_t k = 0; k < n_steps; ++k) {
        e = step_once(c, v, w, u, n0 + k, &local);
        total += local.iterations;
        fb += local.fallbacks;
        if (e) break;
    }
    HIP_OK(hipEventRecord(c->ev1, c->stream));
    if (!c->batched) {
        c->stream = user;
        HIP_OK(hipEventRecord(c->ev_out, c->work));
        HIP_OK(hipStreamWaitEvent(user, c->ev_out, 0));
    }
    HIP_OK(hipStreamSynchronize(c->stream));
    float ms = 0.f;
    hipEventElapsedTime(&ms, c->ev0, c->ev1);
    if (st) {
        *st = local;
        st->total_iterations = total;
        st->fallbacks = fb;
        st->ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    }
    (void)ms;
    return e;
}

bido_status bido_solve(bido_ctx* c, const double* rhs, double* x, double tol, bido_stats* st) {
    if (!c || !rhs || !x) return fail(BIDO_ERR_ARG, "null argument");
    hipStream_t s = c->stream;
    const int64_t N = c->N, NH = c->NH;
    auto t0 = std::chrono::steady_clock::now();
    launch_scatter_in(s, N, c->u_pos, rhs, c->Y);
    launch_scatter_in(s, NH, c->v_pos, rhs + N, c->Y + N);
    launch_dot_reduce(s, N, c->Y, nullptr, c->rd, c->sc + S_Y1SUM);
    launch_dot_reduce(s, c->n2, c->Y, c->Y, c->rd, c->sc + S_YY);
    bido_status e = read_scalars(c);
    if (e) return e;
    const double y1sum = c->sc_host[S_Y1SUM], ynorm = std::sqrt(c->sc_host[S_YY]);
    const double removed = std::fabs(y1sum) / std::sqrt((double)N);
    if (removed > 1e-8 * ynorm)
        return fail(BIDO_ERR_RANGE, "rhs not in the range of Lambda: its u part has a mean (Prop. 1)");
    launch_shift(s, N, c->Y, c->sc, S_Y1SUM, (double)N);   // project Y1 on 1^perp
    launch_scatter_in(s, N, c->u_pos, x, c->x);
    launch_scatter_in(s, NH, c->v_pos, x + N, c->x + N);
    bido_stats local{};
    e = pcg(c, tol > 0 ? tol : c->params.tol, &local);
    finish_collection(c, e == BIDO_OK);
    if (e && e != BIDO_ERR_NOT_CONVERGED) return e;
    launch_dot_reduce(s, N, c->m_int, c->x, c->rd, c->sc + S_MU);
    launch_gather_out(s, N, c->u_pos, c->x, x, c->sc, S_MU, c->hs.msum);
    launch_gather_out(s, NH, c->v_pos, c->x + N, x + N, c->sc, -1, 1.0);
    HIP_OK(hipStreamSynchronize(s));
    if (st) {
        *st = local;
        st->range_removed = removed;
        st->total_iterations = local.iterations;
        st->ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    }
    return e;
}

}  // extern "C"
