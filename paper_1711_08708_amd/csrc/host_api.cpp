// Host-only inspection entry points (include/bido_host.h).
#include <cstring>
#include <memory>
#include <string>

#include "../../include/bido_host.h"
#include "setup.h"

struct bido_host {
    bido::HostSetup hs;
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
        default: return hfail(BIDO_ERR_ARG, "unknown matrix");
    }
    *n = a->n;
    *nnz = a->nnz();
    *ptr = a->ptr.data();
    *col = a->col.data();
    *val = a->val.data();
    return BIDO_OK;
}

bido_status bido_host_vec(const bido_host* h, int which, int64_t* n, const double** data) {
    if (!h || !n || !data) return hfail(BIDO_ERR_ARG, "null argument");
    const std::vector<double>* v = nullptr;
    if (which == BIDO_VEC_M) v = &h->hs.A.m;
    else if (which == BIDO_VEC_MH) v = &h->hs.A.mH;
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

bido_status bido_host_factor_stats(const bido_host* h, int which, int64_t* dense_entries,
                                   int64_t* stored_entries, int64_t* n_lowrank, int* height,
                                   int* max_sep) {
    if (!h) return hfail(BIDO_ERR_ARG, "null argument");
    const bido::Factor* f = which == BIDO_FACTOR_P1 ? &h->hs.p1 : which == BIDO_FACTOR_PK ? &h->hs.pk : nullptr;
    if (!f) return hfail(BIDO_ERR_ARG, "unknown factor");
    if (dense_entries) *dense_entries = f->dense_entries();
    if (stored_entries) *stored_entries = f->stored_entries();
    if (n_lowrank) *n_lowrank = f->n_lowrank();
    if (height) *height = f->tree.height;
    if (max_sep) {
        int m = 0;
        for (const auto& fr : f->fronts) m = fr.nI > m ? fr.nI : m;
        *max_sep = m;
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
