// Host-only inspection entry points (include/bido_host.h).
#include <algorithm>
#include <cstring>
#include <memory>
#include <string>

#include "../../include/bido_host.h"
#include "plan.h"
#include "setup.h"

struct bido_host {
    bido::HostSetup hs;
    bido::PlanOptions opt[2];   // plan options of the P_1 and P_K queries
};

namespace {
thread_local std::string h_err;
bido_status hfail(bido_status c, const std::string& m) {
    h_err = m;
    return c;
}
}  // namespace

extern "C" {

const char* bido_host_last_error(void) { return h_err.c_str(); }

bido_status bido_host_setup(const bido_mesh* mesh, const bido_tissue* tissue,
                            const bido_params* params, bido_host** out) {
    if (!out) return hfail(BIDO_ERR_ARG, "out is null");
    *out = nullptr;
    std::unique_ptr<bido_host> h(new bido_host());
    std::string err;
    if (!bido::build_host(mesh, tissue, params, h->hs, err))
        return hfail(err.find("pivot") != std::string::npos ? BIDO_ERR_NOT_SPD : BIDO_ERR_ARG, err);
    *out = h.release();
    return BIDO_OK;
}

void bido_host_free(bido_host* h) { delete h; }

bido_status bido_host_csr(const bido_host* h, int which, int64_t* n, int64_t* nnz,
                          const int64_t** ptr, const int32_t** col, const double** val) {
    if (!h || !n || !nnz || !ptr || !col || !val) return hfail(BIDO_ERR_ARG, "null argument");
    const bido::Csr* a = nullptr;
    switch (which) {
        case BIDO_MAT_S1: a = &h->hs.A.S1; break;
        case BIDO_MAT_SI: a = &h->hs.A.Si; break;
        case BIDO_MAT_SM: a = &h->hs.A.Sm; break;
        case BIDO_MAT_LAMBDA: a = &h->hs.lam; break;
        case BIDO_MAT_GNN_AGG: a = &h->hs.gnn_agg; break;
        case BIDO_MAT_KM: a = &h->hs.km_int; break;
        default: return hfail(BIDO_ERR_ARG, "unknown matrix");
    }
    *n = a->n;
    *nnz = a->nnz();
    *ptr = a->ptr.data();
    *col = a->col.data();
    *val = a->val.data();
    return BIDO_OK;
}

bido_status bido_host_pk_interval(const bido_host* h, int lanczos_steps, double* out) {
    if (!h || !out || lanczos_steps < 1) return hfail(BIDO_ERR_ARG, "bad argument");
    const bido::HostSetup& hs = h->hs;
    std::vector<double> gm(hs.km_int.n, 0.0);
    for (size_t l = 0; l < hs.mh_loc.size(); ++l) gm[hs.v_pos[l]] = hs.gamma * hs.mh_loc[l];
    bido::ChebInterval iv;
    std::string err;
    if (!bido::chebyshev_interval(hs.km_int, gm, lanczos_steps, iv, err)) return hfail(BIDO_ERR_ARG, err);
    const double v[6] = {iv.lo, iv.hi, iv.ritz_lo, iv.ritz_hi, iv.bound_lo, iv.bound_hi};
    std::copy(v, v + 6, out);
    return BIDO_OK;
}

bido_status bido_host_pk_emulate(const bido_host* h, int steps, double lo, double hi, const double* b, double* x) {
    if (!h || !b || !x || steps < 1 || !(lo > 0.0) || !(hi > lo)) return hfail(BIDO_ERR_ARG, "bad argument");
    const bido::Csr& K = h->hs.km_int;
    const int64_t n = K.n;
    std::vector<double> dinv(n, 0.0), r(b, b + n), d(n), dn(n);
    for (int64_t i = 0; i < n; ++i)
        for (int64_t p = K.ptr[i]; p < K.ptr[i + 1]; ++p)
            if (K.col[p] == i) dinv[i] += K.val[p];
    for (auto& v : dinv) v = 1.0 / v;
    const bido::ChebCoef c = bido::chebyshev_coefficients(lo, hi, steps);
    for (int64_t i = 0; i < n; ++i) x[i] = d[i] = c.inv_theta * dinv[i] * b[i];
    for (int k = 1; k < steps; ++k) {          // r -= K d; d = c1 d + c2 D^-1 r; x += d
        for (int64_t i = 0; i < n; ++i) {
            double s = 0.0;
            for (int64_t p = K.ptr[i]; p < K.ptr[i + 1]; ++p) s += K.val[p] * d[K.col[p]];
            r[i] -= s;
            dn[i] = c.c1[k - 1] * d[i] + c.c2[k - 1] * dinv[i] * r[i];
        }
        for (int64_t i = 0; i < n; ++i) x[i] += dn[i];
        d.swap(dn);
    }
    return BIDO_OK;
}

bido_status bido_host_set_dt(bido_host* h, double dt, int refactor) {
    if (!h) return hfail(BIDO_ERR_ARG, "null argument");
    std::string err;
    if (!bido::host_set_dt(h->hs, dt, refactor != 0, err)) return hfail(BIDO_ERR_ARG, err);
    return BIDO_OK;
}

bido_status bido_host_locate(const bido_host* h, int n, const double* pts, int64_t* ids, double* wts) {
    if (!h || n < 0 || (n > 0 && (!pts || !ids || !wts))) return hfail(BIDO_ERR_ARG, "bad argument");
    std::vector<int64_t> vi;
    std::vector<double> vw;
    std::string err;
    if (!bido::locate_points(h->hs.A.dim, h->hs.xyz, h->hs.elems, pts, n, vi, vw, err))
        return hfail(BIDO_ERR_ARG, err);
    std::copy(vi.begin(), vi.end(), ids);
    std::copy(vw.begin(), vw.end(), wts);
    return BIDO_OK;
}

bido_status bido_host_vec(const bido_host* h, int which, int64_t* n, const double** data) {
    if (!h || !n || !data) return hfail(BIDO_ERR_ARG, "null argument");
    const std::vector<double>* v = nullptr;
    if (which == BIDO_VEC_M) v = &h->hs.A.m;
    else if (which == BIDO_VEC_MH) v = &h->hs.A.mH;
    else if (which == BIDO_VEC_GNN_STATIC) v = &h->hs.gnn_static;
    else return hfail(BIDO_ERR_ARG, "unknown vector");
    *n = (int64_t)v->size();
    *data = v->data();
    return BIDO_OK;
}

bido_status bido_host_index(const bido_host* h, int which, int64_t* n, const int64_t** data) {
    if (!h || !n || !data) return hfail(BIDO_ERR_ARG, "null argument");
    const std::vector<int64_t>* v = nullptr;
    if (which == BIDO_IDX_UPOS) v = &h->hs.u_pos;
    else if (which == BIDO_IDX_VPOS) v = &h->hs.v_pos;
    else if (which == BIDO_IDX_HEART) v = &h->hs.A.heart;
    else return hfail(BIDO_ERR_ARG, "unknown index");
    *n = (int64_t)v->size();
    *data = v->data();
    return BIDO_OK;
}

bido_status bido_host_factor_stats(const bido_host* h, int which, int64_t* entries, int* height,
                                   int* max_sep) {
    if (!h) return hfail(BIDO_ERR_ARG, "null argument");
    const bido::Factor* f = which == BIDO_FACTOR_P1 ? &h->hs.p1 : which == BIDO_FACTOR_PK ? &h->hs.pk : nullptr;
    if (!f) return hfail(BIDO_ERR_ARG, "unknown factor");
    if (entries) *entries = f->dense_entries();
    if (height) *height = f->tree.height;
    if (max_sep) {
        int m = 0;
        for (const auto& fr : f->fronts) m = fr.nI > m ? fr.nI : m;
        *max_sep = m;
    }
    return BIDO_OK;
}

bido_status bido_host_factor_nodes(const bido_host* h, int which, int64_t* n_nodes, int32_t* out,
                                   int64_t cap) {
    if (!h || !n_nodes) return hfail(BIDO_ERR_ARG, "null argument");
    const bido::Factor* f = which == BIDO_FACTOR_P1 ? &h->hs.p1 : which == BIDO_FACTOR_PK ? &h->hs.pk : nullptr;
    if (!f) return hfail(BIDO_ERR_ARG, "unknown factor");
    const int64_t nn = (int64_t)f->fronts.size();
    *n_nodes = nn;
    if (out)
        for (int64_t i = 0; i < nn && i < cap; ++i) {
            const auto& nd = f->tree.nodes[i];
            out[i * 5 + 0] = f->fronts[i].nI;
            out[i * 5 + 1] = f->fronts[i].nB;
            out[i * 5 + 2] = nd.height;
            out[i * 5 + 3] = nd.depth;
            out[i * 5 + 4] = nd.parent;
        }
    return BIDO_OK;
}

bido_status bido_host_factor_emulate(const bido_host* h, int which, const double* b, double* x) {
    if (!h || !b || !x) return hfail(BIDO_ERR_ARG, "null argument");
    const bido::Factor* f = which == BIDO_FACTOR_P1 ? &h->hs.p1 : which == BIDO_FACTOR_PK ? &h->hs.pk : nullptr;
    if (!f) return hfail(BIDO_ERR_ARG, "unknown factor");
    bido::FactorPlan p;
    std::string err;
    if (!bido::build_plan(*f, p, err, h->hs.params.n_threads, &h->opt[which])) return hfail(BIDO_ERR_ARG, err);
    try {
        bido::emulate_plan(p, b, x);
    } catch (const std::exception& e) {
        return hfail(BIDO_ERR_STATE, std::string("plan emulation: ") + e.what());
    }
    return BIDO_OK;
}

bido_status bido_host_factor_plan(const bido_host* h, int which, int* hc, int* n_sub, int* n_levels,
                                  int64_t* n_fwd_items, int64_t* n_bwd_items, int64_t* n_bwd_split) {
    if (!h) return hfail(BIDO_ERR_ARG, "null argument");
    const bido::Factor* f = which == BIDO_FACTOR_P1 ? &h->hs.p1 : which == BIDO_FACTOR_PK ? &h->hs.pk : nullptr;
    if (!f) return hfail(BIDO_ERR_ARG, "unknown factor");
    bido::FactorPlan p;
    std::string err;
    if (!bido::build_plan(*f, p, err, 0, &h->opt[which])) return hfail(BIDO_ERR_ARG, err);
    if (hc) *hc = p.hc;
    if (n_sub) *n_sub = p.n_sub;
    if (n_levels) *n_levels = (int)p.spans.size();
    if (n_fwd_items) *n_fwd_items = (int64_t)p.fwd_items.size();
    if (n_bwd_items) *n_bwd_items = (int64_t)p.bwd_items.size();
    if (n_bwd_split) *n_bwd_split = (int64_t)p.bwd_comb.size();
    return BIDO_OK;
}

static const bido::Amg* host_amg(const bido_host* h, int which) {
    const bido::Amg* m = which == BIDO_FACTOR_P1 ? &h->hs.amg1 : which == BIDO_FACTOR_PK ? &h->hs.amgk : nullptr;
    return m && !m->levels.empty() ? m : nullptr;
}

bido_status bido_host_amg_info(const bido_host* h, int which, int* levels, int64_t* n_coarse, double* op_complexity,
                               double* seconds, int* smooth_steps) {
    if (!h) return hfail(BIDO_ERR_ARG, "null argument");
    const bido::Amg* m = host_amg(h, which);
    if (!m) return hfail(BIDO_ERR_STATE, "no multigrid hierarchy for that block");
    if (levels) *levels = (int)m->levels.size();
    if (n_coarse) *n_coarse = m->levels.back().A.n;
    if (op_complexity) *op_complexity = m->op_complexity;
    if (seconds) *seconds = m->setup_seconds;
    if (smooth_steps) *smooth_steps = m->smooth_steps;
    return BIDO_OK;
}

bido_status bido_host_lambda_blocked(const bido_host* h, int64_t* n, int64_t* npos, const int64_t** ptr,
                                     const int32_t** col, const double** val, const double** gm) {
    if (!h || !n || !npos || !ptr || !col || !val || !gm) return hfail(BIDO_ERR_ARG, "null argument");
    const bido::LamBlocked& b = h->hs.lamb;
    if (b.n == 0) return hfail(BIDO_ERR_STATE, "no blocked form of Lambda (torso rows or two orders)");
    *n = b.n;
    *npos = (int64_t)b.col.size();
    *ptr = b.ptr.data();
    *col = b.col.data();
    *val = b.val.data();
    *gm = b.gm.data();
    return BIDO_OK;
}

bido_status bido_host_amg_level(const bido_host* h, int which, int level, int what, int64_t* n, int64_t* nnz,
                                const int64_t** ptr, const int32_t** col, const double** val) {
    if (!h || !n || !nnz || !ptr || !col || !val) return hfail(BIDO_ERR_ARG, "null argument");
    const bido::Amg* m = host_amg(h, which);
    if (!m) return hfail(BIDO_ERR_STATE, "no multigrid hierarchy for that block");
    if (level < 0 || level >= (int)m->levels.size()) return hfail(BIDO_ERR_ARG, "level out of range");
    const bido::AmgLevel& L = m->levels[level];
    if (what != 0 && level + 1 == (int)m->levels.size()) return hfail(BIDO_ERR_ARG, "the coarsest level has no P");
    const bido::Csr& a = what == 0 ? L.A : L.P;
    if (what != 0 && what != 1) return hfail(BIDO_ERR_ARG, "what: 0 = A, 1 = P");
    *n = a.n;
    *nnz = a.nnz();
    *ptr = a.ptr.data();
    *col = a.col.data();
    *val = a.val.data();
    return BIDO_OK;
}

bido_status bido_host_amg_smoother(const bido_host* h, int which, int level, const double** dinv, double* lo,
                                   double* hi, int* steps) {
    if (!h || !dinv || !lo || !hi || !steps) return hfail(BIDO_ERR_ARG, "null argument");
    const bido::Amg* m = host_amg(h, which);
    if (!m) return hfail(BIDO_ERR_STATE, "no multigrid hierarchy for that block");
    if (level < 0 || level >= (int)m->levels.size()) return hfail(BIDO_ERR_ARG, "level out of range");
    const bido::AmgLevel& L = m->levels[level];
    *dinv = L.dinv.data();
    *steps = L.steps;
    *lo = L.lo;
    *hi = L.hi;
    return BIDO_OK;
}

bido_status bido_host_amg_apply(const bido_host* h, int which, const double* b, double* x) {
    if (!h || !b || !x) return hfail(BIDO_ERR_ARG, "null argument");
    const bido::Amg* m = host_amg(h, which);
    if (!m) return hfail(BIDO_ERR_STATE, "no multigrid hierarchy for that block");
    bido::amg_apply(*m, b, x);
    return BIDO_OK;
}

bido_status bido_host_set_plan(bido_host* h, int which, const bido_plan* q) {
    if (!h || !q) return hfail(BIDO_ERR_ARG, "null argument");
    if (which != BIDO_FACTOR_P1 && which != BIDO_FACTOR_PK) return hfail(BIDO_ERR_ARG, "unknown factor");
    bido::PlanOptions o;
    o.top_h = q->top_h;
    o.fwd_cols = q->fwd_cols;
    o.bwd_rows = q->bwd_rows;
    o.bwd_wide = q->bwd_wide;
    o.level_items = q->level_items;
    o.sub_h = q->sub_h;
    o.sub_want = q->sub_want;
    o.sub_total = q->sub_total;
    o.bwd_group_max = q->bwd_group_max;
    h->opt[which] = o;
    return BIDO_OK;
}

bido_status bido_host_merge(const bido_host* const* hs, int n, bido_host** out) {
    if (!hs || n < 1 || !out) return hfail(BIDO_ERR_ARG, "null argument");
    auto m = std::make_unique<bido_host>();
    std::vector<const bido::Factor*> f1, fk;
    std::vector<int64_t> o1, ok;
    int64_t off = 0;
    for (int s = 0; s < n; ++s) {
        if (!hs[s]) return hfail(BIDO_ERR_ARG, "null host set-up");
        const bido::HostSetup& h = hs[s]->hs;
        f1.push_back(&h.p1);
        fk.push_back(&h.pk);
        o1.push_back(off);
        ok.push_back(off + h.A.N);
        off += h.A.N + h.A.NH;
    }
    bido::merge_factors(f1, o1, off, m->hs.p1);
    bido::merge_factors(fk, ok, off, m->hs.pk);
    m->hs.params = hs[0]->hs.params;
    *out = m.release();
    return BIDO_OK;
}

bido_status bido_host_factor_top(const bido_host* h, int which, int* top_h, int64_t* n_top, double* seconds,
                                 int64_t* stored_entries, int* max_rank, int64_t* n_lowrank) {
    if (!h) return hfail(BIDO_ERR_ARG, "null argument");
    const bido::Factor* f = which == BIDO_FACTOR_P1 ? &h->hs.p1 : which == BIDO_FACTOR_PK ? &h->hs.pk : nullptr;
    if (!f) return hfail(BIDO_ERR_ARG, "unknown factor");
    bido::FactorPlan p;
    std::string err;
    if (!bido::build_plan(*f, p, err, h->hs.params.n_threads, &h->opt[which])) return hfail(BIDO_ERR_ARG, err);
    if (top_h) *top_h = p.top_h;
    if (n_top) *n_top = p.n_top;
    if (seconds) *seconds = p.top_seconds;
    if (stored_entries) *stored_entries = p.top_hodlr ? (int64_t)p.hodlr.val.size() : p.n_top * p.n_top;
    if (max_rank) *max_rank = p.top_hodlr ? p.hodlr.max_rank : -1;
    if (n_lowrank) {
        int64_t k = 0;
        if (p.top_hodlr)
            for (const auto& b : p.hodlr.blocks) k += b.k > 0;
        *n_lowrank = k;
    }
    return BIDO_OK;
}

bido_status bido_host_factor_apply(const bido_host* h, int which, const double* b, double* x) {
    if (!h || !b || !x) return hfail(BIDO_ERR_ARG, "null argument");
    const bido::Factor* f = which == BIDO_FACTOR_P1 ? &h->hs.p1 : which == BIDO_FACTOR_PK ? &h->hs.pk : nullptr;
    if (!f) return hfail(BIDO_ERR_ARG, "unknown factor");
    bido::host_solve(*f, b, x);
    return BIDO_OK;
}

}  // extern "C"
