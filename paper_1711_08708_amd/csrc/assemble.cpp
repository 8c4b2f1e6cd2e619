// P1 assembly of the bidomain matrices (Sec. 3.1, Sec. 5.2).
//
// Element stiffness K_e = |e| G sigma G^T with G the gradients of the
// barycentric functions; the lumped mass gives |e|/(d+1) to each vertex of e
// (the diagonal mass of the paper's CVFE runs).  Tensors (Sec. 2):
//   sigma_i, sigma_e = Q diag(g) Q^T in the element's fibre frame Q,
//   sigma_1 = sigma_i + sigma_e on heart elements, k(x) Id on torso ones,
//   sigma_m = (sigma_e^-1 + sigma_i^-1)^-1 (monodomain, Sec. 5.2).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>

#include "host.h"

namespace bido {
namespace {

int inv_small(int d, const double* a, double* ai, double* det_out) {
    if (d == 2) {
        double det = a[0] * a[3] - a[1] * a[2];
        if (det == 0.0) return -1;
        ai[0] = a[3] / det; ai[1] = -a[1] / det;
        ai[2] = -a[2] / det; ai[3] = a[0] / det;
        *det_out = det;
        return 0;
    }
    double c00 = a[4] * a[8] - a[5] * a[7];
    double c01 = a[5] * a[6] - a[3] * a[8];
    double c02 = a[3] * a[7] - a[4] * a[6];
    double det = a[0] * c00 + a[1] * c01 + a[2] * c02;
    if (det == 0.0) return -1;
    double id = 1.0 / det;
    ai[0] = c00 * id;
    ai[1] = (a[2] * a[7] - a[1] * a[8]) * id;
    ai[2] = (a[1] * a[5] - a[2] * a[4]) * id;
    ai[3] = c01 * id;
    ai[4] = (a[0] * a[8] - a[2] * a[6]) * id;
    ai[5] = (a[2] * a[3] - a[0] * a[5]) * id;
    ai[6] = c02 * id;
    ai[7] = (a[1] * a[6] - a[0] * a[7]) * id;
    ai[8] = (a[0] * a[4] - a[1] * a[3]) * id;
    *det_out = det;
    return 0;
}

// Q diag(g) Q^T for a row-major frame Q whose columns are the axes.
void frame_tensor(int d, const double* Q, const double* g, double* s) {
    for (int i = 0; i < d; ++i)
        for (int j = 0; j < d; ++j) {
            double acc = 0.0;
            for (int k = 0; k < d; ++k) acc += Q[i * d + k] * g[k] * Q[j * d + k];
            s[i * d + j] = acc;
        }
}

struct ElemGeo {
    std::vector<double> vol;   // E
    std::vector<double> G;     // E x (d+1) x d
};

bool element_geometry(const MeshIn& in, ElemGeo& g, std::string& err) {
    const int d = in.dim, k = d + 1;
    const int64_t E = in.n_elems;
    g.vol.resize(E);
    g.G.resize((size_t)E * k * d);
    const double fact = (d == 2) ? 2.0 : 6.0;
    int bad = 0;
#pragma omp parallel for schedule(static) reduction(+ : bad)
    for (int64_t e = 0; e < E; ++e) {
        const int32_t* v = in.elems + e * k;
        double J[9], Ji[9], det;
        // J[i][c] = x_{c+1}[i] - x_0[i]  (columns are edge vectors)
        for (int i = 0; i < d; ++i)
            for (int c = 0; c < d; ++c)
                J[i * d + c] = in.xyz[(int64_t)v[c + 1] * d + i] - in.xyz[(int64_t)v[0] * d + i];
        if (inv_small(d, J, Ji, &det)) { ++bad; continue; }
        g.vol[e] = std::fabs(det) / fact;
        double* G = &g.G[(size_t)e * k * d];
        // grad of barycentric c+1 = row c of J^-1; grad of barycentric 0 = -sum
        for (int i = 0; i < d; ++i) {
            double s = 0.0;
            for (int c = 0; c < d; ++c) {
                G[(c + 1) * d + i] = Ji[c * d + i];
                s += Ji[c * d + i];
            }
            G[i] = -s;
        }
    }
    if (bad) { err = "degenerate element(s) in the mesh"; return false; }
    return true;
}

// Generic row-wise assembly of sum_e |e| G sigma_e G^T over the elements
// with use_elem[e] != 0, rows/cols mapped through idx (global -> local, -1
// = not present), n local rows.  tensor(e, out) writes sigma_e.
template <class TensorFn>
void assemble_stiffness(const MeshIn& in, const ElemGeo& geo,
                        const std::vector<int64_t>& n2e_ptr,
                        const std::vector<int64_t>& n2e,
                        const std::vector<char>& use_elem,
                        const std::vector<int64_t>& idx,    // global->local
                        const std::vector<int64_t>& rows,   // local->global
                        TensorFn tensor, Csr& out) {
    const int d = in.dim, k = d + 1;
    const int64_t n = (int64_t)rows.size();
    out.n = n;
    out.ptr.assign(n + 1, 0);
    // pass 1: count distinct columns per row
#pragma omp parallel
    {
        std::vector<int64_t> cols;
#pragma omp for schedule(dynamic, 256)
        for (int64_t r = 0; r < n; ++r) {
            int64_t gi = rows[r];
            cols.clear();
            for (int64_t p = n2e_ptr[gi]; p < n2e_ptr[gi + 1]; ++p) {
                int64_t e = n2e[p];
                if (!use_elem[e]) continue;
                for (int b = 0; b < k; ++b) cols.push_back(idx[in.elems[e * k + b]]);
            }
            std::sort(cols.begin(), cols.end());
            out.ptr[r + 1] = std::unique(cols.begin(), cols.end()) - cols.begin();
        }
    }
    for (int64_t r = 0; r < n; ++r) out.ptr[r + 1] += out.ptr[r];
    out.col.resize(out.ptr[n]);
    out.val.assign(out.ptr[n], 0.0);
    // pass 2: fill
#pragma omp parallel
    {
        std::vector<int64_t> cols;
        double sig[9];
#pragma omp for schedule(dynamic, 256)
        for (int64_t r = 0; r < n; ++r) {
            int64_t gi = rows[r];
            cols.clear();
            for (int64_t p = n2e_ptr[gi]; p < n2e_ptr[gi + 1]; ++p) {
                int64_t e = n2e[p];
                if (!use_elem[e]) continue;
                for (int b = 0; b < k; ++b) cols.push_back(idx[in.elems[e * k + b]]);
            }
            std::sort(cols.begin(), cols.end());
            cols.erase(std::unique(cols.begin(), cols.end()), cols.end());
            int64_t base = out.ptr[r];
            for (size_t c = 0; c < cols.size(); ++c) out.col[base + c] = (int32_t)cols[c];
            for (int64_t p = n2e_ptr[gi]; p < n2e_ptr[gi + 1]; ++p) {
                int64_t e = n2e[p];
                if (!use_elem[e]) continue;
                const int32_t* v = in.elems + e * k;
                int a = 0;
                while (v[a] != gi) ++a;
                tensor(e, sig);
                const double* G = &geo.G[(size_t)e * k * d];
                double sg[3];   // sigma * grad_a
                for (int i = 0; i < d; ++i) {
                    double s = 0.0;
                    for (int j = 0; j < d; ++j) s += sig[i * d + j] * G[a * d + j];
                    sg[i] = s;
                }
                for (int b = 0; b < k; ++b) {
                    double val = 0.0;
                    for (int i = 0; i < d; ++i) val += G[b * d + i] * sg[i];
                    val *= geo.vol[e];
                    int64_t c = idx[v[b]];
                    int64_t pos = std::lower_bound(cols.begin(), cols.end(), c) - cols.begin();
                    out.val[base + pos] += val;
                }
            }
        }
    }
}

}  // namespace

bool assemble(const MeshIn& in, Assembled& out, std::string& err) {
    const int d = in.dim;
    if (d != 2 && d != 3) { err = "dim must be 2 or 3"; return false; }
    const int k = d + 1;
    const int64_t N = in.n_nodes, E = in.n_elems;
    if (N <= 0 || E <= 0 || !in.xyz || !in.elems || !in.region) {
        err = "empty mesh or missing arrays";
        return false;
    }
    for (int64_t e = 0; e < E * k; ++e)
        if (in.elems[e] < 0 || in.elems[e] >= N) { err = "element vertex out of range"; return false; }
    for (int64_t i = 0; i < N * d; ++i)
        if (!std::isfinite(in.xyz[i])) { err = "non-finite vertex coordinate"; return false; }
    std::vector<char> is_heart_e(E, 0);
    for (int64_t e = 0; e < E; ++e) {
        int r = in.region[e];
        if (r == 1) { is_heart_e[e] = 1; continue; }
        if (r < 0 || r >= in.n_region_sigma || !in.region_sigma) {
            err = "torso region code without a conductivity";
            return false;
        }
        if (!(in.region_sigma[r] > 0.0) || !std::isfinite(in.region_sigma[r])) {
            err = "torso conductivity must be finite and > 0";
            return false;
        }
    }
    bool any_heart = false;
    for (int64_t e = 0; e < E; ++e) any_heart |= is_heart_e[e] != 0;
    if (!any_heart) { err = "mesh has no heart element"; return false; }
    if (!in.fibre) { err = "missing fibre frames"; return false; }
    for (int i = 0; i < d; ++i)
        if (!(in.sigma_i[i] > 0.0) || !(in.sigma_e[i] > 0.0) || !std::isfinite(in.sigma_i[i]) ||
            !std::isfinite(in.sigma_e[i])) {
            err = "heart conductivities must be finite and > 0";
            return false;
        }
    for (int64_t e = 0; e < E; ++e) {
        if (!is_heart_e[e]) continue;
        for (int q = 0; q < d * d; ++q)
            if (!std::isfinite(in.fibre[e * d * d + q])) { err = "non-finite fibre frame"; return false; }
    }

    ElemGeo geo;
    if (!element_geometry(in, geo, err)) return false;

    // vertex -> element incidence
    std::vector<int64_t> cnt(N + 1, 0);
    for (int64_t e = 0; e < E * k; ++e) cnt[in.elems[e] + 1]++;
    for (int64_t i = 0; i < N; ++i) cnt[i + 1] += cnt[i];
    std::vector<int64_t> n2e(cnt[N]);
    {
        std::vector<int64_t> pos(cnt.begin(), cnt.end() - 1);
        for (int64_t e = 0; e < E; ++e)
            for (int a = 0; a < k; ++a) n2e[pos[in.elems[e * k + a]]++] = e;
    }
    for (int64_t i = 0; i < N; ++i)
        if (cnt[i + 1] == cnt[i]) { err = "vertex not used by any element"; return false; }

    // heart vertices, ascending global id
    std::vector<char> hn(N, 0);
    for (int64_t e = 0; e < E; ++e)
        if (is_heart_e[e])
            for (int a = 0; a < k; ++a) hn[in.elems[e * k + a]] = 1;
    out.dim = d;
    out.N = N;
    out.heart.clear();
    out.heart_loc.assign(N, -1);
    for (int64_t i = 0; i < N; ++i)
        if (hn[i]) { out.heart_loc[i] = (int64_t)out.heart.size(); out.heart.push_back(i); }
    out.NH = (int64_t)out.heart.size();

    std::vector<int64_t> ident(N), all_rows(N);
    std::iota(ident.begin(), ident.end(), 0);
    std::iota(all_rows.begin(), all_rows.end(), 0);
    std::vector<char> all_e(E, 1);

    auto heart_tensors = [&](int64_t e, double* si, double* se) {
        const double* Q = in.fibre + e * d * d;
        frame_tensor(d, Q, in.sigma_i, si);
        frame_tensor(d, Q, in.sigma_e, se);
    };
    auto t_sigma1 = [&](int64_t e, double* s) {
        if (is_heart_e[e]) {
            double si[9], se[9];
            heart_tensors(e, si, se);
            for (int i = 0; i < d * d; ++i) s[i] = si[i] + se[i];
        } else {
            double kt = in.region_sigma[in.region[e]];
            for (int i = 0; i < d; ++i)
                for (int j = 0; j < d; ++j) s[i * d + j] = (i == j) ? kt : 0.0;
        }
    };
    auto t_sigmai = [&](int64_t e, double* s) {
        double se[9];
        heart_tensors(e, s, se);
    };
    auto t_sigmam = [&](int64_t e, double* s) {
        double si[9], se[9], ii[9], ie[9], sum[9], det;
        heart_tensors(e, si, se);
        inv_small(d, si, ii, &det);
        inv_small(d, se, ie, &det);
        for (int i = 0; i < d * d; ++i) sum[i] = ii[i] + ie[i];
        inv_small(d, sum, s, &det);
    };

    assemble_stiffness(in, geo, cnt, n2e, all_e, ident, all_rows, t_sigma1, out.S1);
    assemble_stiffness(in, geo, cnt, n2e, is_heart_e, out.heart_loc, out.heart, t_sigmai, out.Si);
    assemble_stiffness(in, geo, cnt, n2e, is_heart_e, out.heart_loc, out.heart, t_sigmam, out.Sm);

    out.m.assign(N, 0.0);
    out.mH.assign(out.NH, 0.0);
    for (int64_t e = 0; e < E; ++e) {
        double share = geo.vol[e] / k;
        for (int a = 0; a < k; ++a) {
            int64_t v = in.elems[e * k + a];
            out.m[v] += share;
            if (is_heart_e[e]) out.mH[out.heart_loc[v]] += share;
        }
    }
    return true;
}

}  // namespace bido
