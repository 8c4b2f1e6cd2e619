// Host set-up (no HIP): assembly (Sec. 3.1), orderings, the system matrix
// Lambda (Sec. 3.2) in the internal order, and the inner-solve factors of
// the block-LU preconditioner (Def. 2 with K ~ K_m, Sec. 5.2-5.3).
#include "setup.h"

#include <algorithm>
#include <array>
#include <chrono>
#include <cmath>

#ifdef _OPENMP
#include <omp.h>
#endif

namespace bido {
namespace {

// the vertex nearest the centroid of the n vertices (coordinates n x d)
int64_t central_vertex(const double* xyz, int64_t n, int d) {
    double c[3] = {0.0, 0.0, 0.0};
    for (int64_t i = 0; i < n; ++i)
        for (int a = 0; a < d; ++a) c[a] += xyz[i * d + a];
    for (int a = 0; a < d; ++a) c[a] /= (double)std::max<int64_t>(n, 1);
    int64_t best = 0;
    double bd = INFINITY;
    for (int64_t i = 0; i < n; ++i) {
        double r = 0.0;
        for (int a = 0; a < d; ++a) r += (xyz[i * d + a] - c[a]) * (xyz[i * d + a] - c[a]);
        if (r < bd) { bd = r; best = i; }
    }
    return best;
}

Csr add_diag(const Csr& a, const std::vector<double>& d, double scale) {
    Csr b = a;
    for (int64_t r = 0; r < a.n; ++r) {
        bool found = false;
        for (int64_t p = a.ptr[r]; p < a.ptr[r + 1]; ++p)
            if (a.col[p] == r) { b.val[p] += scale * d[r]; found = true; }
        if (!found) { b.n = -1; return b; }   // P1 matrices always store the diagonal
    }
    return b;
}

// Features of the learned correction (see setup.h).
void gnn_inputs(const MeshIn& in, const Assembled& A, HostSetup& hs) {
    const int d = A.dim, k = d + 1;
    const int64_t NH = A.NH, E = in.n_elems;
    const int nent = d == 2 ? 3 : 6;
    static const int iu2[3][2] = {{0, 0}, {0, 1}, {1, 1}};
    static const int iu3[6][2] = {{0, 0}, {0, 1}, {0, 2}, {1, 1}, {1, 2}, {2, 2}};
    hs.gnn_static.assign((size_t)NH * 15, 0.0);
    std::vector<double> cnt(NH, 0.0);
    double scale = 0.0;
    for (int a = 0; a < d; ++a) scale = std::max(scale, std::max(in.sigma_i[a], in.sigma_e[a]));
    std::vector<std::array<int32_t, 3>> facets;
    facets.reserve((size_t)E * k);
    for (int64_t e = 0; e < E; ++e) {
        if (in.region[e] != 1) continue;
        const double* Q = in.fibre + e * d * d;
        double si[9], se[9];
        for (int i = 0; i < d; ++i)
            for (int j = 0; j < d; ++j) {
                double a = 0.0, b = 0.0;
                for (int q = 0; q < d; ++q) {
                    a += Q[i * d + q] * in.sigma_i[q] * Q[j * d + q];
                    b += Q[i * d + q] * in.sigma_e[q] * Q[j * d + q];
                }
                si[i * d + j] = a;
                se[i * d + j] = b;
            }
        double ent[12];
        for (int q = 0; q < nent; ++q) {
            const int i = d == 2 ? iu2[q][0] : iu3[q][0], j = d == 2 ? iu2[q][1] : iu3[q][1];
            ent[q] = si[i * d + j];
            ent[nent + q] = se[i * d + j];
        }
        const int32_t* v = in.elems + e * k;
        for (int a = 0; a < k; ++a) {
            const int64_t l = A.heart_loc[v[a]];
            for (int q = 0; q < 2 * nent; ++q) hs.gnn_static[l * 15 + q] += ent[q];
            cnt[l] += 1.0;
        }
        for (int skip = 0; skip < k; ++skip) {
            std::array<int32_t, 3> f{-1, -1, -1};
            int o = 0;
            for (int a = 0; a < k; ++a)
                if (a != skip) f[o++] = (int32_t)A.heart_loc[v[a]];
            std::sort(f.begin(), f.begin() + o);
            facets.push_back(f);
        }
    }
    for (int64_t l = 0; l < NH; ++l)
        for (int q = 0; q < 2 * nent; ++q) hs.gnn_static[l * 15 + q] /= (cnt[l] * scale);
    // boundary of the heart sub-mesh: facets owned by one heart element
    std::sort(facets.begin(), facets.end());
    std::vector<int> dist(NH, -1);
    std::vector<int64_t> queue;
    for (size_t i = 0; i < facets.size();) {
        size_t j = i;
        while (j < facets.size() && facets[j] == facets[i]) ++j;
        if (j - i == 1)
            for (int a = 0; a < d; ++a) {
                const int32_t l = facets[i][a];
                if (dist[l] < 0) { dist[l] = 0; queue.push_back(l); }
            }
        i = j;
    }
    // hop distance over the S_m graph (breadth-first from the boundary)
    const Csr& Sm = A.Sm;
    for (size_t q = 0; q < queue.size(); ++q) {
        const int64_t l = queue[q];
        for (int64_t p = Sm.ptr[l]; p < Sm.ptr[l + 1]; ++p) {
            const int32_t m = Sm.col[p];
            if (dist[m] < 0) { dist[m] = dist[l] + 1; queue.push_back(m); }
        }
    }
    int dmax = 1;
    for (int64_t l = 0; l < NH; ++l) dmax = std::max(dmax, dist[l]);
    for (int64_t l = 0; l < NH; ++l) hs.gnn_static[l * 15 + 2 * nent] = dist[l] < 0 ? 1.0 : (double)dist[l] / dmax;
    // row-normalised |off-diagonal| pattern of S_m
    Csr& G = hs.gnn_agg;
    G.n = NH;
    G.ptr.assign(NH + 1, 0);
    G.col.clear();
    G.val.clear();
    for (int64_t l = 0; l < NH; ++l) {
        double rs = 0.0;
        for (int64_t p = Sm.ptr[l]; p < Sm.ptr[l + 1]; ++p)
            if (Sm.col[p] != l) rs += std::fabs(Sm.val[p]);
        for (int64_t p = Sm.ptr[l]; p < Sm.ptr[l + 1]; ++p)
            if (Sm.col[p] != l && Sm.val[p] != 0.0) {
                G.col.push_back(Sm.col[p]);
                G.val.push_back(std::fabs(Sm.val[p]) / (rs > 0 ? rs : 1.0));
            }
        G.ptr[l + 1] = (int64_t)G.col.size();
    }
}

}  // namespace

bool build_host(const bido_mesh* mesh, const bido_tissue* tissue, const bido_params* params,
                HostSetup& hs, std::string& err) {
    auto t0 = std::chrono::steady_clock::now();
    if (!mesh || !tissue || !params) { err = "null argument"; return false; }
    const bido_params& P = *params;
    if (!(P.chi > 0) || !(P.cm > 0) || !(P.dt > 0)) { err = "chi, cm and dt must be > 0"; return false; }
    if (P.eps_h < 0 || P.leaf < 1 || P.max_iter < 1 || !(P.tol > 0)) { err = "bad solver parameters"; return false; }
    if (P.ionic != 0) { err = "only the Mitchell-Schaeffer model (ionic = 0) is built in"; return false; }
    if (P.precision != BIDO_PREC_FP64 && P.precision != BIDO_PREC_MIXED) { err = "bad precision"; return false; }
    if (P.precond != BIDO_PRECOND_PLAIN && P.precond != BIDO_PRECOND_LEARNED) { err = "bad precond"; return false; }
    if (!std::isfinite(tissue->stim_amp) || !std::isfinite(tissue->stim_t0) || !std::isfinite(tissue->stim_t1) ||
        tissue->stim_t1 < tissue->stim_t0) {
        err = "stimulus amplitude and window must be finite, with t0 <= t1";
        return false;
    }
    if (P.scheme != BIDO_SCHEME_EULER && P.scheme != BIDO_SCHEME_CN && P.scheme != BIDO_SCHEME_STRANG) {
        err = "bad time scheme";
        return false;
    }
    if (P.inner_p1 != BIDO_P1_CHOLESKY && P.inner_p1 != BIDO_P1_AMG) { err = "bad inner_p1"; return false; }
    if (P.amg_columns != 0 && P.amg_columns != 1) {
        err = "bad amg_columns";
        return false;
    }
    if (P.guess_states < 0 || P.guess_states > 16) {
        err = "bad guess_states (0 to 16)";
        return false;
    }
    if (P.inner_pk != BIDO_PK_CHOLESKY && P.inner_pk != BIDO_PK_CHEBYSHEV && P.inner_pk != BIDO_PK_AMG) {
        err = "bad inner_pk";
        return false;
    }
#ifdef _OPENMP
    if (P.n_threads > 0) omp_set_num_threads(P.n_threads);
#endif
    hs.params = P;
    MeshIn in;
    in.dim = mesh->dim;
    in.n_nodes = mesh->n_nodes;
    in.n_elems = mesh->n_elems;
    in.xyz = mesh->xyz;
    in.elems = mesh->elems;
    in.region = mesh->region;
    in.fibre = tissue->fibre;
    in.region_sigma = tissue->region_sigma;
    in.n_region_sigma = tissue->n_region_sigma;
    for (int i = 0; i < 3; ++i) { in.sigma_i[i] = tissue->sigma_i[i]; in.sigma_e[i] = tissue->sigma_e[i]; }
    if (!assemble(in, hs.A, err)) return false;
    hs.xyz.assign(mesh->xyz, mesh->xyz + mesh->n_nodes * mesh->dim);
    hs.elems.assign(mesh->elems, mesh->elems + mesh->n_elems * (mesh->dim + 1));
    const Assembled& A = hs.A;
    const int64_t N = A.N, NH = A.NH;
    const int d = A.dim;
    // the coefficient of M_H in Lambda and K_m: gamma = chi cm / dt for the
    // semi-implicit scheme, 2 gamma for Crank-Nicolson (the system times 2)
    hs.gamma = P.chi * P.cm / P.dt * (P.scheme == BIDO_SCHEME_EULER ? 1.0 : 2.0);

    // orderings: nested dissection of S_1 (u) and of K_m (v) for a factored
    // inner solve; otherwise reverse Cuthill-McKee (a narrow band of column
    // offsets), one order for u and v when the heart is the whole mesh
    std::vector<double> xyz_h((size_t)NH * d);
    for (int64_t k = 0; k < NH; ++k)
        for (int a = 0; a < d; ++a) xyz_h[k * d + a] = mesh->xyz[A.heart[k] * d + a];
    const bool p1_nd = P.inner_p1 == BIDO_P1_CHOLESKY, pk_nd = P.inner_pk == BIDO_PK_CHOLESKY;
    if (p1_nd) nested_dissection(A.S1, mesh->xyz, d, P.leaf, hs.p1.tree);
    else rcm_order(A.S1, hs.p1.tree);
    if (pk_nd) {
        nested_dissection(A.Si, xyz_h.data(), d, P.leaf, hs.pk.tree);
    } else if (!p1_nd && NH == N) {
        NdTree& t = hs.pk.tree;
        t = NdTree();
        t.perm.resize(NH);
        t.iperm.assign(NH, -1);
        for (int64_t l = 0; l < NH; ++l) {
            t.perm[l] = A.heart_loc[hs.p1.tree.perm[l]];
            t.iperm[t.perm[l]] = l;
        }
    } else {
        rcm_order(A.Si, hs.pk.tree);
    }
    const NdTree& t1 = hs.p1.tree;
    const NdTree& tk = hs.pk.tree;
    hs.u_pos = t1.iperm;
    hs.v_pos = tk.iperm;

    // inner-solve matrices: grounded S_1 and K_m = gamma M_H + S_m
    Csr S1p = permute(A.S1, t1.perm, t1.iperm);
    Csr Km = add_diag(A.Sm, A.mH, hs.gamma);
    if (Km.n < 0) { err = "missing diagonal in S_m"; return false; }
    Csr Kmp = permute(Km, tk.perm, tk.iperm);
    hs.km_int = Kmp;
    const int nth = P.n_threads;
    hs.p1_factored = P.inner_p1 == BIDO_P1_CHOLESKY;
    hs.pk_factored = P.inner_pk == BIDO_PK_CHOLESKY;
    if (hs.p1_factored) {
        if (!multifrontal(S1p, hs.p1, N - 1, nth, err)) { err = "P_1: " + err; return false; }
    } else {
        hs.p1.n = N;
        // the grounded vertex (held at zero, excluded from the hierarchy) is
        // the one nearest the centroid of the mesh: on the 128^3 slab 21.0
        // outer iterations per step against 22.7 with a corner vertex (the
        // last one of the reverse Cuthill-McKee order)
        const int64_t gnd = hs.p1.tree.iperm[central_vertex(mesh->xyz, N, d)];
        hs.p1.ground = gnd;
        hs.p1.grounds.assign(1, gnd);
        // S_1 is a pure Laplacian: a lower strength threshold gives larger
        // aggregates at the same outer iteration count (128^3 slab: 8 % fewer
        // bytes per V-cycle, 0.73 -> 0.69 ms); K_m keeps 0.08 (its mass term
        // makes the coarser levels of larger aggregates slower)
        AmgOptions o1;
        o1.theta = 0.04;
        if (!amg_build(S1p, gnd, o1, hs.amg1, err)) { err = "P_1: " + err; return false; }
    }
    if (hs.pk_factored) {
        if (!multifrontal(Kmp, hs.pk, -1, nth, err)) { err = "P_K: " + err; return false; }
    } else {
        hs.pk.n = NH;
        if (P.inner_pk == BIDO_PK_AMG) {
            std::vector<double> m0(NH);
            for (int64_t l = 0; l < NH; ++l) m0[l] = A.mH[tk.perm[l]];
            if (!amg_build(Kmp, -1, AmgOptions(), hs.amgk, err) || !amg_split_mass(hs.amgk, m0, hs.gamma, err)) {
                err = "P_K: " + err;
                return false;
            }
        }
    }
    {   // coordinates (tree order) and the accuracy of the hierarchical top
        std::vector<double> x1((size_t)N * d), xk((size_t)NH * d);
        for (int64_t p = 0; p < N; ++p)
            for (int a = 0; a < d; ++a) x1[p * d + a] = mesh->xyz[t1.perm[p] * d + a];
        for (int64_t p = 0; p < NH; ++p)
            for (int a = 0; a < d; ++a) xk[p * d + a] = xyz_h[tk.perm[p] * d + a];
        set_top_compression(hs.p1, x1.data(), d, P.eps_h);
        set_top_compression(hs.pk, xk.data(), d, P.eps_h);
    }

    // coupling blocks S_i Pi and Pi^T S_i in internal numbering
    const Csr& Si = A.Si;
    hs.avu.n = NH;
    hs.avu.ptr.assign(NH + 1, 0);
    for (int64_t l = 0; l < NH; ++l) {
        int64_t k = tk.perm[l];
        hs.avu.ptr[l + 1] = hs.avu.ptr[l] + (Si.ptr[k + 1] - Si.ptr[k]);
    }
    hs.avu.col.resize(hs.avu.ptr[NH]);
    hs.avu.val.resize(hs.avu.ptr[NH]);
    for (int64_t l = 0; l < NH; ++l) {
        int64_t k = tk.perm[l], base = hs.avu.ptr[l];
        std::vector<std::pair<int32_t, double>> row;
        for (int64_t p = Si.ptr[k]; p < Si.ptr[k + 1]; ++p)
            row.emplace_back((int32_t)hs.u_pos[A.heart[Si.col[p]]], Si.val[p]);
        std::sort(row.begin(), row.end());
        for (size_t q = 0; q < row.size(); ++q) { hs.avu.col[base + q] = row[q].first; hs.avu.val[base + q] = row[q].second; }
    }
    hs.auv.n = N;
    hs.auv.ptr.assign(N + 1, 0);
    for (int64_t p = 0; p < N; ++p) {
        int64_t g = t1.perm[p], k = A.heart_loc[g];
        hs.auv.ptr[p + 1] = hs.auv.ptr[p] + (k >= 0 ? Si.ptr[k + 1] - Si.ptr[k] : 0);
    }
    hs.auv.col.resize(hs.auv.ptr[N]);
    hs.auv.val.resize(hs.auv.ptr[N]);
    for (int64_t p = 0; p < N; ++p) {
        int64_t g = t1.perm[p], k = A.heart_loc[g];
        if (k < 0) continue;
        std::vector<std::pair<int32_t, double>> row;
        for (int64_t q = Si.ptr[k]; q < Si.ptr[k + 1]; ++q)
            row.emplace_back((int32_t)hs.v_pos[Si.col[q]], Si.val[q]);
        std::sort(row.begin(), row.end());
        int64_t base = hs.auv.ptr[p];
        for (size_t q = 0; q < row.size(); ++q) { hs.auv.col[base + q] = row[q].first; hs.auv.val[base + q] = row[q].second; }
    }

    // Lambda = [[S_1, Pi^T S_i], [S_i Pi, gamma M_H + S_i]] in internal order
    Csr Sip = permute(Si, tk.perm, tk.iperm);
    const int64_t n2 = N + NH;
    Csr& L = hs.lam;
    L.n = n2;
    L.ptr.assign(n2 + 1, 0);
    for (int64_t p = 0; p < N; ++p)
        L.ptr[p + 1] = L.ptr[p] + (S1p.ptr[p + 1] - S1p.ptr[p]) + (hs.auv.ptr[p + 1] - hs.auv.ptr[p]);
    for (int64_t l = 0; l < NH; ++l)
        L.ptr[N + l + 1] = L.ptr[N + l] + (hs.avu.ptr[l + 1] - hs.avu.ptr[l]) + (Sip.ptr[l + 1] - Sip.ptr[l]);
    L.col.resize(L.ptr[n2]);
    L.val.resize(L.ptr[n2]);
    for (int64_t p = 0; p < N; ++p) {
        int64_t o = L.ptr[p];
        for (int64_t q = S1p.ptr[p]; q < S1p.ptr[p + 1]; ++q) { L.col[o] = S1p.col[q]; L.val[o++] = S1p.val[q]; }
        for (int64_t q = hs.auv.ptr[p]; q < hs.auv.ptr[p + 1]; ++q) { L.col[o] = (int32_t)(N + hs.auv.col[q]); L.val[o++] = hs.auv.val[q]; }
    }
    for (int64_t l = 0; l < NH; ++l) {
        int64_t o = L.ptr[N + l];
        int64_t k = tk.perm[l];
        for (int64_t q = hs.avu.ptr[l]; q < hs.avu.ptr[l + 1]; ++q) { L.col[o] = hs.avu.col[q]; L.val[o++] = hs.avu.val[q]; }
        for (int64_t q = Sip.ptr[l]; q < Sip.ptr[l + 1]; ++q) {
            L.col[o] = (int32_t)(N + Sip.col[q]);
            L.val[o++] = Sip.val[q] + (Sip.col[q] == l ? hs.gamma * A.mH[k] : 0.0);
        }
    }

    hs.m_int.resize(N);
    for (int64_t p = 0; p < N; ++p) hs.m_int[p] = A.m[t1.perm[p]];
    hs.msum = 0.0;
    for (double v : A.m) hs.msum += v;
    hs.mh_loc = A.mH;
    hs.stim_loc.assign(NH, 0.0);
    if (tissue->stim_mask)
        for (int64_t k = 0; k < NH; ++k)
            if (tissue->stim_mask[A.heart[k]]) hs.stim_loc[k] = tissue->stim_amp;
    gnn_inputs(in, A, hs);
    hs.stim_n0 = std::llround(tissue->stim_t0 / P.dt);
    hs.stim_n1 = std::llround(tissue->stim_t1 / P.dt);
    hs.stim_t0 = tissue->stim_t0;
    hs.stim_t1 = tissue->stim_t1;
    build_lam_blocked(hs, hs.lamb);   // (none when the heart is not the whole mesh)
    hs.setup_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    return true;
}

}  // namespace bido

namespace bido {

// The blocked form of Lambda (see LamBlocked), built from its CSR when the heart
// is the whole mesh and the u and v orders agree: row k pairs u row k with v
// row N + k; positions are the union of the columns of S_1 and S_i in that
// row, S_i read from Pi^T S_i and checked against S_i Pi and the off-
// diagonal v-v entries; gm[k] = the v-v diagonal minus S_i's.  Returns false
// (CSR products only) when the structure does not match.
bool build_lam_blocked(const HostSetup& hs, LamBlocked& out) {
    out = LamBlocked();
    std::vector<int64_t>& ptr = out.ptr;
    std::vector<int32_t>& col = out.col;
    std::vector<double>& val = out.val;
    std::vector<double>& gm = out.gm;
    const int64_t N = hs.A.N;
    if (N != hs.A.NH || N == 0) return false;
    for (int64_t j = 0; j < N; ++j)
        if (hs.u_pos[hs.A.heart[j]] != hs.v_pos[j]) return false;
    const Csr& L = hs.lam;
    double big = 0.0;
    for (double v : L.val) big = std::max(big, std::fabs(v));
    const double tol = 1e-13 * big;
    ptr.assign(N + 1, 0);
    col.clear();
    val.clear();
    gm.assign(N, 0.0);
    struct E { int32_t c; double s1, si, vu, vv; bool has_si, has_vu, has_vv; };
    std::vector<E> row;
    std::vector<int64_t> tag(N, -1);     // row that last saw a column, and its slot
    std::vector<int32_t> slot(N, 0);
    for (int64_t k = 0; k < N; ++k) {
        row.clear();
        auto at = [&](int32_t c) -> E& {
            if (tag[c] != k) {
                tag[c] = k;
                slot[c] = (int32_t)row.size();
                row.push_back({c, 0.0, 0.0, 0.0, 0.0, false, false, false});
            }
            return row[slot[c]];
        };
        for (int64_t q = L.ptr[k]; q < L.ptr[k + 1]; ++q) {
            const int64_t c = L.col[q];
            if (c < N) at((int32_t)c).s1 += L.val[q];
            else { E& e = at((int32_t)(c - N)); e.si += L.val[q]; e.has_si = true; }
        }
        for (int64_t q = L.ptr[N + k]; q < L.ptr[N + k + 1]; ++q) {
            const int64_t c = L.col[q];
            if (c < N) { E& e = at((int32_t)c); e.vu += L.val[q]; e.has_vu = true; }
            else { E& e = at((int32_t)(c - N)); e.vv += L.val[q]; e.has_vv = true; }
        }
        std::sort(row.begin(), row.end(), [](const E& a, const E& b) { return a.c < b.c; });
        for (const E& e : row) {
            if (std::fabs(e.si - e.vu) > tol) return false;
            if (e.c == k) gm[k] = e.vv - e.si;
            else if (std::fabs(e.vv - e.si) > tol) return false;
            col.push_back(e.c);
            val.push_back(e.s1);
            val.push_back(e.si);
        }
        ptr[k + 1] = (int64_t)col.size();
    }
    out.n = N;
    return true;
}

bool host_set_dt(HostSetup& hs, double dt, bool refactor, std::string& err) {
    bido_params& P = hs.params;
    if (!(dt > 0.0) || !std::isfinite(dt)) { err = "dt must be > 0"; return false; }
    const Assembled& A = hs.A;
    const int64_t N = A.N, NH = A.NH;
    const double gamma = P.chi * P.cm / dt * (P.scheme == BIDO_SCHEME_EULER ? 1.0 : 2.0);
    const NdTree& tk = hs.pk.tree;
    // K_m = gamma M_H + S_m, as at set-up: only its diagonal moves, written
    // with the set-up's arithmetic (S_m's diagonal plus gamma m) into a copy
    Csr Kmp = hs.km_int;
    for (int64_t l = 0; l < NH; ++l) {
        const int64_t k = tk.perm[l];
        double sm = 0.0;
        bool f = false;
        for (int64_t q = A.Sm.ptr[k]; q < A.Sm.ptr[k + 1]; ++q)
            if (A.Sm.col[q] == k) { sm = A.Sm.val[q]; f = true; }
        if (!f) { err = "missing diagonal in S_m"; return false; }
        for (int64_t q = Kmp.ptr[l]; q < Kmp.ptr[l + 1]; ++q)
            if (Kmp.col[q] == l) Kmp.val[q] = sm + gamma * A.mH[k];
    }
    // the v-v diagonal of Lambda: S_i(k, k) + gamma m_k
    std::vector<double> sdiag(NH, 0.0);
    bool found = true;
    for (int64_t k = 0; k < NH; ++k) {
        bool f = false;
        for (int64_t q = A.Si.ptr[k]; q < A.Si.ptr[k + 1]; ++q)
            if (A.Si.col[q] == k) { sdiag[k] = A.Si.val[q]; f = true; }
        found = found && f;
    }
    if (!found) { err = "missing diagonal in S_i"; return false; }
    if (refactor && !hs.pk_factored) {
        // multigrid K_m: the same aggregation and transfers, each level's
        // matrix moved by (gamma' - gamma) times its Galerkin mass part
        if (P.inner_pk == BIDO_PK_AMG) {
            std::string e2;
            if (!amg_refresh_gamma(hs.amgk, gamma, e2)) { err = "P_K: " + e2; return false; }
        }
    } else if (refactor) {
        Factor nf;
        nf.tree = hs.pk.tree;
        std::string e2;
        if (!multifrontal(Kmp, nf, -1, P.n_threads, e2)) { err = "P_K: " + e2; return false; }
        set_top_compression(nf, hs.pk.xyz.data(), hs.pk.dim, hs.pk.eps);
        hs.pk = std::move(nf);
    }
    Csr& L = hs.lam;
    for (int64_t l = 0; l < NH; ++l) {
        const int64_t k = tk.perm[l], row = N + l;
        for (int64_t q = L.ptr[row]; q < L.ptr[row + 1]; ++q)
            if (L.col[q] == row) L.val[q] = sdiag[k] + gamma * A.mH[k];
    }
    hs.km_int = std::move(Kmp);
    hs.gamma = gamma;
    P.dt = dt;
    if (hs.lamb.n > 0) {     // only gm = the v-v diagonal minus S_i's moves
        LamBlocked& b = hs.lamb;
        for (int64_t k = 0; k < b.n; ++k) {
            double si = 0.0, vv = 0.0;
            for (int64_t q = b.ptr[k]; q < b.ptr[k + 1]; ++q)
                if (b.col[q] == k) si = b.val[2 * q + 1];
            for (int64_t q = L.ptr[N + k]; q < L.ptr[N + k + 1]; ++q)
                if (L.col[q] == N + k) vv = L.val[q];
            b.gm[k] = vv - si;
        }
    }
    hs.stim_n0 = std::llround(hs.stim_t0 / dt);
    hs.stim_n1 = std::llround(hs.stim_t1 / dt);
    return true;
}

}  // namespace bido
