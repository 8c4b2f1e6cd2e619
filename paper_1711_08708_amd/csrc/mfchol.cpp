// Multifrontal Cholesky on the nested-dissection tree, and the host
// application of the resulting factor (used only by the set-up checks).
//
// Node t eliminates its own indices I_t.  Its front gathers the original
// entries of the columns I_t and the update matrices of its children; the
// partial factorisation gives L_tt, L_Bt = F_Bt L_tt^-T and the update
// matrix F_BB - L_Bt L_Bt^T passed to the parent.  The stored panel is
// P_t = [L_tt^-1 ; L_Bt L_tt^-1], which turns both triangular solves into
// matrix-vector products (see host.h).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <unordered_map>

#ifdef _OPENMP
#include <omp.h>
#endif

#include "dense.h"
#include "host.h"

namespace bido {

int64_t Factor::dense_entries() const {
    int64_t s = 0;
    for (const auto& f : fronts)
        s += (int64_t)f.nI * (f.nI + 1) / 2 + (int64_t)f.nB * f.nI;
    return s;
}

namespace {

// Pattern/values of the grounded matrix: row and column g reduced to the
// unit diagonal.
Csr grounded_copy(const Csr& a, int64_t g) {
    if (g < 0) return a;
    Csr b;
    b.n = a.n;
    b.ptr.assign(a.n + 1, 0);
    b.col.reserve(a.col.size());
    b.val.reserve(a.val.size());
    for (int64_t r = 0; r < a.n; ++r) {
        for (int64_t p = a.ptr[r]; p < a.ptr[r + 1]; ++p) {
            int64_t c = a.col[p];
            if (r == g || c == g) {
                if (r == g && c == g) {
                    b.col.push_back((int32_t)c);
                    b.val.push_back(1.0);
                }
                continue;
            }
            b.col.push_back(a.col[p]);
            b.val.push_back(a.val[p]);
        }
        if (r == g && (b.col.empty() || b.col.back() != g)) {
            // diagonal was structurally missing: insert it in order
            std::vector<std::pair<int32_t, double>> row;
            for (int64_t p = b.ptr[r]; p < (int64_t)b.col.size(); ++p) row.emplace_back(b.col[p], b.val[p]);
            row.emplace_back((int32_t)g, 1.0);
            std::sort(row.begin(), row.end());
            b.col.resize(b.ptr[r]);
            b.val.resize(b.ptr[r]);
            for (auto& e : row) { b.col.push_back(e.first); b.val.push_back(e.second); }
        }
        b.ptr[r + 1] = (int64_t)b.col.size();
    }
    return b;
}

}  // namespace

bool multifrontal(const Csr& a0, Factor& f, int64_t ground, int n_threads,
                  std::string& err) {
    const Csr a = grounded_copy(a0, ground);
    const NdTree& t = f.tree;
    const int nn = (int)t.nodes.size();
    f.n = a.n;
    f.ground = ground;
    f.grounds.clear();
    if (ground >= 0) f.grounds.push_back(ground);
    f.fronts.assign(nn, Front());

    // ---- symbolic: boundary sets, children first (post-order) -----------
    for (int id = 0; id < nn; ++id) {
        const NdNode& nd = t.nodes[id];
        Front& fr = f.fronts[id];
        fr.node = id;
        fr.off = nd.begin;
        fr.nI = (int)(nd.end - nd.begin);
        std::vector<int64_t> b;
        for (int64_t i = nd.begin; i < nd.end; ++i)
            for (int64_t p = a.ptr[i]; p < a.ptr[i + 1]; ++p)
                if (a.col[p] >= nd.end) b.push_back(a.col[p]);
        for (int c = 0; c < 2; ++c) {
            int ch = nd.child[c];
            if (ch < 0) continue;
            for (int64_t j : f.fronts[ch].B)
                if (j >= nd.end) b.push_back(j);
        }
        std::sort(b.begin(), b.end());
        b.erase(std::unique(b.begin(), b.end()), b.end());
        fr.B.swap(b);
        fr.nB = (int)fr.B.size();
    }

    // ---- numeric: level by level from the leaves -------------------------
    std::vector<std::vector<double>> upd(nn);   // update matrices (nB x nB)
    std::vector<std::vector<int>> by_height(t.height + 1);
    for (int id = 0; id < nn; ++id) by_height[t.nodes[id].height].push_back(id);
#ifdef _OPENMP
    const int nth = n_threads > 0 ? n_threads : omp_get_max_threads();
#else
    const int nth = 1;
    (void)n_threads;
#endif
    int failed = -1;
    int64_t fail_pivot = -1;

    auto factor_node = [&](int id, bool par) -> bool {
        const NdNode& nd = t.nodes[id];
        Front& fr = f.fronts[id];
        const int nI = fr.nI, nB = fr.nB, nF = nI + nB;
        std::vector<double> F((size_t)nF * nF, 0.0);
        auto pos_of = [&](int64_t j) -> int {   // front position of index j
            if (j < nd.end) return (int)(j - nd.begin);
            return nI + (int)(std::lower_bound(fr.B.begin(), fr.B.end(), j) - fr.B.begin());
        };
        // original entries of the columns I_t (lower triangle of the front)
        for (int64_t i = nd.begin; i < nd.end; ++i) {
            const int ci = (int)(i - nd.begin);
            for (int64_t p = a.ptr[i]; p < a.ptr[i + 1]; ++p) {
                int64_t j = a.col[p];
                if (j < nd.begin) continue;     // eliminated in the subtree
                int pj = pos_of(j);
                if (pj >= ci) F[(size_t)pj * nF + ci] = a.val[p];
            }
        }
        // extend-add of the children's update matrices
        for (int c = 0; c < 2; ++c) {
            int ch = nd.child[c];
            if (ch < 0) continue;
            const Front& cf = f.fronts[ch];
            std::vector<int> map(cf.nB);
            for (int r = 0; r < cf.nB; ++r) map[r] = pos_of(cf.B[r]);
            const std::vector<double>& U = upd[ch];
            for (int r = 0; r < cf.nB; ++r)
                for (int s = 0; s <= r; ++s) {
                    int pr = map[r], ps = map[s];
                    double v = U[(size_t)r * cf.nB + s];
                    if (pr >= ps) F[(size_t)pr * nF + ps] += v;
                    else F[(size_t)ps * nF + pr] += v;
                }
            std::vector<double>().swap(upd[ch]);
        }
        // partial factorisation
        int64_t bad = dense::potrf_lower(nI, F.data(), nF, par);
        if (bad >= 0) {
#pragma omp critical
            {
                failed = id;
                fail_pivot = nd.begin + bad;
            }
            return false;
        }
        double* LB = F.data() + (size_t)nI * nF;       // rows nI.., cols 0..nI
        if (nB > 0) {
            dense::trsm_right_lower_t(nB, nI, F.data(), nF, LB, nF, par);
            // update matrix = F_BB - L_Bt L_Bt^T (lower part)
            dense::gemm_nt_sub(nB, nB, nI, LB, nF, LB, nF, F.data() + (size_t)nI * nF + nI, nF,
                               true, par);
            std::vector<double>& U = upd[id];
            U.assign((size_t)nB * nB, 0.0);
            for (int r = 0; r < nB; ++r)
                for (int s = 0; s <= r; ++s)
                    U[(size_t)r * nB + s] = F[(size_t)(nI + r) * nF + nI + s];
        }
        // panel: [L^-1 ; L_Bt L^-1]
        fr.P.assign((size_t)nF * nI, 0.0);
        std::vector<double> Y((size_t)nI * nI, 0.0);   // Y = L^-T
        for (int i = 0; i < nI; ++i) Y[(size_t)i * nI + i] = 1.0;
        dense::trsm_right_lower_t(nI, nI, F.data(), nF, Y.data(), nI, par);
        for (int i = 0; i < nI; ++i)
            for (int j = 0; j <= i; ++j) fr.P[(size_t)i * nI + j] = Y[(size_t)j * nI + i];
        if (nB > 0) {
            // M = L_Bt L^-1 = L_Bt Y^T ;  gemm_nt_sub computes C -= A B^T
            std::vector<double> Mneg((size_t)nB * nI, 0.0);
            dense::gemm_nt_sub(nB, nI, nI, LB, nF, Y.data(), nI, Mneg.data(), nI, false, par);
            for (size_t q = 0; q < Mneg.size(); ++q) fr.P[(size_t)nI * nI + q] = -Mneg[q];
        }
        return true;
    };

    for (int h = 0; h <= t.height && failed < 0; ++h) {
        const auto& ids = by_height[h];
        if ((int)ids.size() >= nth) {
#pragma omp parallel for schedule(dynamic, 1) num_threads(nth)
            for (size_t q = 0; q < ids.size(); ++q) {
                if (failed >= 0) continue;
                factor_node(ids[q], false);
            }
        } else {
            for (int id : ids) {
                if (failed >= 0) break;
                factor_node(id, true);
            }
        }
    }
    if (failed >= 0) {
        err = "non-positive pivot at index " + std::to_string(fail_pivot) +
              " during the multifrontal Cholesky";
        return false;
    }
    return true;
}

// ---------------------------------------------------------------------------
// Host solve with the panels (forward: post-order; backward: reverse).
// ---------------------------------------------------------------------------
namespace {

void panel_apply(const Front& fr, const double* w, double* out) {
    // out = P_t w   (nI + nB rows)
    const int nI = fr.nI, nF = fr.nI + fr.nB;
    for (int r = 0; r < nF; ++r) {
        const double* p = &fr.P[(size_t)r * nI];
        int len = r < nI ? r + 1 : nI;
        double s = 0.0;
        for (int c = 0; c < len; ++c) s += p[c] * w[c];
        out[r] = s;
    }
}

void panel_apply_t(const Front& fr, const double* z, double* out) {
    // out = P_t^T z   (nI entries), z has nI + nB entries
    const int nI = fr.nI, nF = fr.nI + fr.nB;
    std::fill(out, out + nI, 0.0);
    for (int r = 0; r < nF; ++r) {
        const double* p = &fr.P[(size_t)r * nI];
        int len = r < nI ? r + 1 : nI;
        for (int c = 0; c < len; ++c) out[c] += p[c] * z[r];
    }
}

}  // namespace

void host_solve(const Factor& f, const double* b, double* x) {
    const int64_t n = f.n;
    std::vector<double> acc(n, 0.0), y(n, 0.0), w, out;
    std::vector<char> gnd(n, 0);
    for (int64_t g : f.grounds) gnd[g] = 1;
    for (const Front& fr : f.fronts) {   // post-order
        w.resize(fr.nI);
        out.resize(fr.nI + fr.nB);
        for (int i = 0; i < fr.nI; ++i) {
            int64_t g = fr.off + i;
            w[i] = gnd[g] ? 0.0 : b[g] - acc[g];
        }
        panel_apply(fr, w.data(), out.data());
        for (int i = 0; i < fr.nI; ++i) y[fr.off + i] = out[i];
        for (int r = 0; r < fr.nB; ++r) acc[fr.B[r]] += out[fr.nI + r];
    }
    for (int64_t i = 0; i < n; ++i) x[i] = 0.0;
    for (auto it = f.fronts.rbegin(); it != f.fronts.rend(); ++it) {
        const Front& fr = *it;
        w.resize(fr.nI + fr.nB);
        out.resize(fr.nI);
        for (int i = 0; i < fr.nI; ++i) w[i] = y[fr.off + i];
        for (int r = 0; r < fr.nB; ++r) w[fr.nI + r] = -x[fr.B[r]];
        panel_apply_t(fr, w.data(), out.data());
        for (int i = 0; i < fr.nI; ++i) x[fr.off + i] = out[i];
    }
}

}  // namespace bido

namespace bido {

// Disjoint union of factors (the factor of a block-diagonal matrix): factor
// s occupies indices [offs[s], offs[s] + n_s) of an index space of n_total
// entries (indices outside every factor are never touched); tree nodes and
// boundary indices are shifted and the trees become one forest.
void merge_factors(const std::vector<const Factor*>& fs, const std::vector<int64_t>& offs, int64_t n_total,
                   Factor& out) {
    out = Factor();
    out.n = n_total;
    out.ground = -1;
    out.eps = fs.empty() ? 0.0 : fs[0]->eps;
    out.dim = fs.empty() ? 0 : fs[0]->dim;
    bool coords = out.dim > 0;
    for (const Factor* f : fs) coords = coords && f->dim == out.dim && (int64_t)f->xyz.size() >= f->n * f->dim;
    if (coords) out.xyz.assign((size_t)n_total * out.dim, 0.0);
    else out.dim = 0;
    int node_off = 0;
    for (size_t s = 0; s < fs.size(); ++s) {
        const Factor& f = *fs[s];
        const int64_t o = offs[s];
        out.parts.push_back(&f);
        out.part_off.push_back(o);
        out.part_node0.push_back(node_off);
        // a single cached top names the cut the slice's own plan uses
        out.part_top_h.push_back(f.top_cache.size() == 1 ? f.top_cache.begin()->first : -1);
        for (int64_t g : f.grounds) out.grounds.push_back(g + o);
        if (coords)
            for (int64_t i = 0; i < f.n * f.dim; ++i) out.xyz[o * f.dim + i] = f.xyz[i];
        for (const NdNode& nd : f.tree.nodes) {
            NdNode m = nd;
            m.begin += o;
            m.end += o;
            m.sub_begin += o;
            if (m.parent >= 0) m.parent += node_off;
            for (int& ch : m.child)
                if (ch >= 0) ch += node_off;
            out.tree.nodes.push_back(m);
        }
        for (const Front& fr : f.fronts) {
            Front m = fr;
            m.node += node_off;
            m.off += o;
            for (int64_t& b : m.B) b += o;
            out.fronts.push_back(std::move(m));
        }
        out.tree.height = std::max(out.tree.height, f.tree.height);
        node_off += (int)f.tree.nodes.size();
    }
    out.tree.root = -1;
}

}  // namespace bido
