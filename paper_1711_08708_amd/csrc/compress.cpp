// Hierarchical low-rank compression (Sec. 5.3): the explicit inverse of the
// top separators' Schur complement is held as a symmetric hierarchical
// off-diagonal low-rank matrix.  The top vertices are ordered by recursive
// geometric bisection; every off-diagonal block of the bisection tree is
// truncated at relative accuracy eps by a rank-revealing (column-pivoted
// Householder) QR, and the leaves stay dense.
#include <omp.h>

#include <algorithm>
#include <cfloat>
#include <cmath>
#include <numeric>
#include <stdexcept>

#include "host.h"

namespace bido {

void set_top_compression(Factor& f, const double* xyz, int dim, double eps) {
    f.dim = dim;
    f.eps = eps;
    f.xyz.assign(xyz, xyz + (size_t)f.n * dim);
}

// B (m x n, row-major, leading dimension ld) ~ U V^T with U (m x k) and
// V (n x k) column-major: Householder QR with column pivoting, stopped at the
// first pivot |R_jj| <= max(eps |R_00|, abs_tol) (a block far below the
// matrix it belongs to gets rank 0 instead of a basis of rounding noise).
void rrqr_lowrank(const double* B, int64_t ld, int m, int n, double eps, std::vector<double>& U,
                  std::vector<double>& V, int& k, double abs_tol) {
    std::vector<double> A((size_t)m * n);          // column-major work copy
    for (int i = 0; i < m; ++i)
        for (int j = 0; j < n; ++j) A[(size_t)j * m + i] = B[(size_t)i * ld + j];
    std::vector<double> nrm(n), beta, diag;
    std::vector<int> piv(n);
    std::iota(piv.begin(), piv.end(), 0);
    for (int j = 0; j < n; ++j) {
        double s = 0.0;
        for (int i = 0; i < m; ++i) s += A[(size_t)j * m + i] * A[(size_t)j * m + i];
        nrm[j] = s;
    }
    const int kmax = std::min(m, n);
    double r00 = 0.0;
    k = 0;
    for (int j = 0; j < kmax; ++j) {
        const int p = (int)(std::max_element(nrm.begin() + j, nrm.end()) - nrm.begin());
        const double np = std::sqrt(nrm[p]);
        if (j == 0) r00 = np;
        if (!(np > abs_tol) || np <= eps * r00 || !std::isfinite(np)) break;
        if (p != j) {
            std::swap_ranges(A.begin() + (size_t)j * m, A.begin() + (size_t)(j + 1) * m, A.begin() + (size_t)p * m);
            std::swap(nrm[j], nrm[p]);
            std::swap(piv[j], piv[p]);
        }
        double* x = &A[(size_t)j * m];
        double xx = 0.0;
        for (int i = j; i < m; ++i) xx += x[i] * x[i];
        const double alpha = x[j] >= 0.0 ? -std::sqrt(xx) : std::sqrt(xx);
        x[j] -= alpha;                                  // x[j:m] is now the reflector v
        double vtv = 0.0;
        for (int i = j; i < m; ++i) vtv += x[i] * x[i];
        const double bt = vtv > 0.0 ? 2.0 / vtv : 0.0;
#pragma omp parallel for schedule(static) if ((int64_t)(n - j) * (m - j) > 200000)
        for (int l = j + 1; l < n; ++l) {
            double* y = &A[(size_t)l * m];
            double s = 0.0;
            for (int i = j; i < m; ++i) s += x[i] * y[i];
            s *= bt;
            for (int i = j; i < m; ++i) y[i] -= s * x[i];
            double t = 0.0;
            for (int i = j + 1; i < m; ++i) t += y[i] * y[i];
            nrm[l] = t;
        }
        beta.push_back(bt);
        diag.push_back(alpha);
        ++k;
    }
    // U = Q e_c (c < k): apply the reflectors in reverse order
    U.assign((size_t)m * k, 0.0);
    for (int c = 0; c < k; ++c) {
        double* q = &U[(size_t)c * m];
        q[c] = 1.0;
        for (int i = c; i >= 0; --i) {
            const double* v = &A[(size_t)i * m];
            double s = 0.0;
            for (int r = i; r < m; ++r) s += v[r] * q[r];
            s *= beta[i];
            for (int r = i; r < m; ++r) q[r] -= s * v[r];
        }
    }
    // V[piv[l]][c] = R[c][l]
    V.assign((size_t)n * k, 0.0);
    for (int c = 0; c < k; ++c)
        for (int l = c; l < n; ++l) V[(size_t)c * n + piv[l]] = l == c ? diag[c] : A[(size_t)l * m + c];
}

namespace {

void bisect(std::vector<int64_t>& ord, int64_t a, int64_t e, const double* xyz, int dim, int leaf) {
    if (e - a <= leaf) return;
    double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
    for (int64_t i = a; i < e; ++i)
        for (int d = 0; d < dim; ++d) {
            lo[d] = std::min(lo[d], xyz[ord[i] * dim + d]);
            hi[d] = std::max(hi[d], xyz[ord[i] * dim + d]);
        }
    int ax = 0;
    for (int d = 1; d < dim; ++d)
        if (hi[d] - lo[d] > hi[ax] - lo[ax]) ax = d;
    const int64_t m = (a + e) / 2;
    std::nth_element(ord.begin() + a, ord.begin() + m, ord.begin() + e, [&](int64_t p, int64_t q) {
        const double xp = xyz[p * dim + ax], xq = xyz[q * dim + ax];
        return xp < xq || (xp == xq && p < q);
    });
    bisect(ord, a, m, xyz, dim, leaf);
    bisect(ord, m, e, xyz, dim, leaf);
}

}  // namespace

void hodlr_order(int64_t n, const double* xyz, int dim, int leaf, std::vector<int64_t>& ord) {
    ord.resize(n);
    std::iota(ord.begin(), ord.end(), 0);
    bisect(ord, 0, n, xyz, dim, leaf);
}

// A: n x n row-major, symmetric, already in the bisection order.
void hodlr_build(const std::vector<double>& A, int64_t n, double eps, int leaf, int n_threads, Hodlr& h) {
    h = Hodlr();
    h.n = n;
    struct Node { int64_t a, m, e; };
    std::vector<Node> internal;
    std::vector<std::pair<int64_t, int64_t>> leaves;
    // the bisection tree: ranges halve exactly as in hodlr_order
    std::vector<std::pair<int64_t, int64_t>> todo{{0, n}};
    while (!todo.empty()) {
        auto [a, e] = todo.back();
        todo.pop_back();
        if (e - a <= leaf) {
            leaves.push_back({a, e});
            continue;
        }
        const int64_t m = (a + e) / 2;
        internal.push_back({a, m, e});
        todo.push_back({m, e});
        todo.push_back({a, m});
    }
    std::sort(leaves.begin(), leaves.end());
    const int nb = (int)internal.size();
    std::vector<std::vector<double>> Us(nb), Vs(nb);
    std::vector<int> ks(nb, 0);
    (void)n_threads;
    // blocks are truncated relative to themselves, but never below eps (at
    // least the square of the machine epsilon) times the largest entry
    double scale = 0.0;
    for (double v : A) scale = std::max(scale, std::fabs(v));
    const double abs_tol = std::max(eps, DBL_EPSILON * DBL_EPSILON) * scale;
    for (int b = 0; b < nb; ++b) {
        const Node& nd = internal[b];
        rrqr_lowrank(&A[(size_t)nd.a * n + nd.m], n, (int)(nd.m - nd.a), (int)(nd.e - nd.m), eps, Us[b], Vs[b],
                     ks[b], abs_tol);
    }
    int64_t toff = 0;
    for (int b = 0; b < nb; ++b) {
        const Node& nd = internal[b];
        HodlrBlock hb{};
        hb.a = (int32_t)nd.a;
        hb.m = (int32_t)nd.m;
        hb.e = (int32_t)nd.e;
        hb.k = ks[b];
        hb.u = (int64_t)h.val.size();
        h.val.insert(h.val.end(), Us[b].begin(), Us[b].end());
        hb.v = (int64_t)h.val.size();
        h.val.insert(h.val.end(), Vs[b].begin(), Vs[b].end());
        hb.t = (int32_t)toff;
        toff += 2 * ks[b];
        h.max_rank = std::max(h.max_rank, ks[b]);
        h.blocks.push_back(hb);
    }
    h.t_size = std::max<int64_t>(toff, 1);
    for (auto [a, e] : leaves) {
        HodlrLeaf lf{};
        lf.a = (int32_t)a;
        lf.e = (int32_t)e;
        lf.d = (int64_t)h.val.size();
        for (int64_t j = a; j < e; ++j)                  // column-major diagonal block
            for (int64_t i = a; i < e; ++i) h.val.push_back(A[(size_t)i * n + j]);
        lf.anc = (int32_t)h.anc.size();
        for (int b = 0; b < nb; ++b) {
            const Node& nd = internal[b];
            if (a >= nd.a && e <= nd.e) h.anc.push_back(2 * b + (a >= nd.m ? 1 : 0));
        }
        lf.nanc = (int32_t)(h.anc.size() - lf.anc);
        h.leaves.push_back(lf);
    }
    if (h.anc.empty()) h.anc.push_back(0);
}

// y = A w with the hierarchical form (reference for the plan emulation;
// bounds-checked accesses).
void hodlr_apply(const Hodlr& h, const double* w, double* y) {
    std::vector<double> t(h.t_size, 0.0);
    for (const HodlrBlock& b : h.blocks) {
        const int64_t mi = b.m - b.a, mj = b.e - b.m;
        for (int c = 0; c < b.k; ++c) {
            double sj = 0.0, si = 0.0;
            for (int64_t r = 0; r < mj; ++r) sj += h.val.at(b.v + c * mj + r) * w[b.m + r];
            for (int64_t r = 0; r < mi; ++r) si += h.val.at(b.u + c * mi + r) * w[b.a + r];
            t.at(b.t + c) = sj;
            t.at(b.t + b.k + c) = si;
        }
    }
    for (const HodlrLeaf& lf : h.leaves) {
        const int64_t len = lf.e - lf.a;
        for (int64_t i = 0; i < len; ++i) {
            double s = 0.0;
            for (int64_t j = 0; j < len; ++j) s += h.val.at(lf.d + j * len + i) * w[lf.a + j];
            for (int q = 0; q < lf.nanc; ++q) {
                const int code = h.anc.at(lf.anc + q);
                const HodlrBlock& b = h.blocks.at(code >> 1);
                if ((code & 1) == 0) {                 // rows in [a, m): U (V^T w[m:e))
                    const int64_t mi = b.m - b.a, r = lf.a + i - b.a;
                    if (r < 0 || r >= mi) throw std::runtime_error("leaf outside its ancestor block");
                    for (int c = 0; c < b.k; ++c) s += h.val.at(b.u + c * mi + r) * t.at(b.t + c);
                } else {                               // rows in [m, e): V (U^T w[a:m))
                    const int64_t mj = b.e - b.m, r = lf.a + i - b.m;
                    if (r < 0 || r >= mj) throw std::runtime_error("leaf outside its ancestor block");
                    for (int c = 0; c < b.k; ++c) s += h.val.at(b.v + c * mj + r) * t.at(b.t + b.k + c);
                }
            }
            y[lf.a + i] = s;
        }
    }
}

}  // namespace bido
