// Smoothed-aggregation algebraic multigrid: an alternative inner
// preconditioner P_1 ~ S_1 (and P_K ~ K_m) inside the block-LU framework.
//
// Sec. 5.3 leaves P_1 and P_K free (any preconditioner of the elliptic or
// parabolic block that is cheap and parallel fits Def. 2) and names
// multigrid among the classical choices.  The hierarchy below needs no
// factorisation, so its set-up stays linear in the number of non-zeros.
//
// Construction (Vanek, Mandel, Brezina, "Algebraic multigrid by smoothed
// aggregation for second and fourth order elliptic problems", Computing 56,
// 1996), level by level from the fine matrix A_0:
//   * strength: j is a strong neighbour of i when
//     |a_ij| >= theta sqrt(a_ii a_jj);
//   * aggregation in three passes: (1) a vertex whose strong neighbours are
//     all free starts an aggregate with them; (2) a free vertex joins the
//     aggregate of its strongest neighbour from pass 1; (3) what is left
//     forms aggregates with its free strong neighbours.  The passes visit
//     the finest level in index order and a coarser level in the order its
//     aggregates were made (equal strengths in pass 2: the neighbour
//     visited first); aggregates are numbered by their first vertex, so a
//     banded fine order gives banded coarse matrices;
//   * tentative prolongation P^ (the constant vector, the kernel of the
//     Neumann Laplacian, restricted to each aggregate and normalised);
//   * smoothed prolongation P = (I - omega D^-1 A) P^ with
//     omega = 4 / (3 lambda_max(D^-1 A));
//   * Galerkin coarse matrix A_{l+1} = P^T A_l P,
// until the coarse matrix is small; the coarsest is inverted densely.
//
// The V-cycle is symmetric: the same Chebyshev smoother S (a fixed
// polynomial in D^-1 A times D^-1, on [hi / ratio, hi] with hi above the
// largest eigenvalue of D^-1 A) before and after the coarse correction, so
// the preconditioner is symmetric positive definite and plain CG stays valid.
// The finest level smooths with smooth_steps Chebyshev steps, the coarser
// ones with coarse_steps (one step is the damped Jacobi sweep, which reads no
// matrix: on the 128^3 slab it costs one outer iteration in 22 and saves
// two passes over each coarser level's matrix per smoothing).
//
// A vertex can be excluded (the grounded vertex of S_1, whose row and column
// are the unit vector): it joins no aggregate and its smoother weight is 0,
// so the V-cycle returns 0 there whatever the input, like the grounded
// factor.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <numeric>
#include <string>
#include <vector>

#ifdef _OPENMP
#include <omp.h>
#endif

#include "dense.h"
#include "host.h"

namespace bido {

namespace {

int n_threads_now() {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
int thread_id() {
#ifdef _OPENMP
    return omp_get_thread_num();
#else
    return 0;
#endif
}

// C = A B (Gustavson, two passes: row counts, then values), columns sorted.
Csr spgemm(const Csr& A, const Csr& B, int64_t ncols) {
    Csr C;
    C.n = A.n;
    C.ptr.assign(A.n + 1, 0);
    const int nt = n_threads_now();
    std::vector<std::vector<int64_t>> mark(nt);
#pragma omp parallel
    {
        std::vector<int64_t>& mk = mark[thread_id()];
        mk.assign(ncols, -1);
#pragma omp for schedule(dynamic, 1024)
        for (int64_t i = 0; i < A.n; ++i) {
            int64_t cnt = 0;
            for (int64_t p = A.ptr[i]; p < A.ptr[i + 1]; ++p) {
                const int64_t k = A.col[p];
                for (int64_t q = B.ptr[k]; q < B.ptr[k + 1]; ++q)
                    if (mk[B.col[q]] != i) {
                        mk[B.col[q]] = i;
                        ++cnt;
                    }
            }
            C.ptr[i + 1] = cnt;
        }
    }
    for (int64_t i = 0; i < A.n; ++i) C.ptr[i + 1] += C.ptr[i];
    C.col.resize(C.ptr[A.n]);
    C.val.resize(C.ptr[A.n]);
    std::vector<std::vector<double>> acc(nt);
#pragma omp parallel
    {
        std::vector<int64_t>& mk = mark[thread_id()];
        std::vector<double>& ac = acc[thread_id()];
        std::fill(mk.begin(), mk.end(), -1);
        ac.assign(ncols, 0.0);
        std::vector<int32_t> cols;
#pragma omp for schedule(dynamic, 1024)
        for (int64_t i = 0; i < A.n; ++i) {
            cols.clear();
            for (int64_t p = A.ptr[i]; p < A.ptr[i + 1]; ++p) {
                const int64_t k = A.col[p];
                const double a = A.val[p];
                for (int64_t q = B.ptr[k]; q < B.ptr[k + 1]; ++q) {
                    const int32_t j = B.col[q];
                    if (mk[j] != i) {
                        mk[j] = i;
                        ac[j] = 0.0;
                        cols.push_back(j);
                    }
                    ac[j] += a * B.val[q];
                }
            }
            std::sort(cols.begin(), cols.end());
            int64_t o = C.ptr[i];
            for (int32_t j : cols) {
                C.col[o] = j;
                C.val[o++] = ac[j];
            }
        }
    }
    return C;
}

Csr transpose(const Csr& A, int64_t ncols) {
    Csr T;
    T.n = ncols;
    T.ptr.assign(ncols + 1, 0);
    for (int64_t p = 0; p < A.nnz(); ++p) ++T.ptr[A.col[p] + 1];
    for (int64_t j = 0; j < ncols; ++j) T.ptr[j + 1] += T.ptr[j];
    T.col.resize(A.nnz());
    T.val.resize(A.nnz());
    std::vector<int64_t> next(T.ptr.begin(), T.ptr.end() - 1);
    for (int64_t i = 0; i < A.n; ++i)
        for (int64_t p = A.ptr[i]; p < A.ptr[i + 1]; ++p) {
            const int64_t o = next[A.col[p]]++;
            T.col[o] = (int32_t)i;
            T.val[o] = A.val[p];
        }
    return T;
}

void spmv(const Csr& A, const double* x, double* y) {
#pragma omp parallel for schedule(static) if (A.n > 20000)
    for (int64_t i = 0; i < A.n; ++i) {
        double s = 0.0;
        for (int64_t p = A.ptr[i]; p < A.ptr[i + 1]; ++p) s += A.val[p] * x[A.col[p]];
        y[i] = s;
    }
}

double diag_of(const Csr& A, int64_t i) {
    for (int64_t p = A.ptr[i]; p < A.ptr[i + 1]; ++p)
        if (A.col[p] == i) return A.val[p];
    return 0.0;
}

uint64_t mix64(uint64_t& s) {
    uint64_t z = (s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

}  // namespace

// The fixed pseudo-random start of the Lanczos estimates (zero on excluded
// rows), normalised; false when it is zero.
bool lanczos_start(const std::vector<double>& dinv, std::vector<double>& v) {
    const int64_t n = (int64_t)dinv.size();
    v.assign(n, 0.0);
    uint64_t seed = 0xa36ull;
    double nv = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        v[i] = dinv[i] > 0.0 ? (double)(mix64(seed) >> 11) * 0x1.0p-53 - 0.5 : 0.0;
        nv += v[i] * v[i];
    }
    if (!(nv > 0.0)) return false;
    nv = std::sqrt(nv);
    for (auto& x : v) x /= nv;
    return true;
}

// Largest eigenvalue of the symmetric tridiagonal matrix (diagonal al,
// off-diagonal be): bisection on the Sturm count.
double tridiag_largest(const std::vector<double>& al, const std::vector<double>& be) {
    double lo = al[0], hi = al[0];
    for (size_t i = 0; i < al.size(); ++i) {
        const double r = (i > 0 ? std::fabs(be[i - 1]) : 0.0) + (i + 1 < al.size() ? std::fabs(be[i]) : 0.0);
        lo = std::min(lo, al[i] - r);
        hi = std::max(hi, al[i] + r);
    }
    const int k = (int)al.size() - 1;
    for (int it = 0; it < 200 && hi - lo > 1e-14 * std::max(1.0, std::fabs(hi)); ++it) {
        const double mid = 0.5 * (lo + hi);
        int count = 0;
        double q = 1.0;
        for (size_t i = 0; i < al.size(); ++i) {
            const double b2 = i > 0 ? be[i - 1] * be[i - 1] : 0.0;
            q = al[i] - mid - (i > 0 ? b2 / q : 0.0);
            if (q == 0.0) q = -1e-300;
            if (q < 0.0) ++count;
        }
        if (count > k) hi = mid; else lo = mid;
    }
    return 0.5 * (lo + hi);
}

namespace {

// Dense inverse of a coarsest level (n <= 8192; an excluded vertex's row and
// column become the unit vector, and its row and column of the inverse 0):
// Cholesky, inverse of the factor, L^-T L^-1.
bool coarse_inverse(const Csr& A, int64_t excluded, std::vector<double>& inv, std::string& err) {
    const int64_t n = A.n;
    if (n > 8192) {
        err = "multigrid: coarsest level too large (" + std::to_string(n) + " > 8192)";
        return false;
    }
    std::vector<double> M((size_t)n * n, 0.0);
    for (int64_t i = 0; i < n; ++i)
        for (int64_t p = A.ptr[i]; p < A.ptr[i + 1]; ++p) M[(size_t)i * n + A.col[p]] = A.val[p];
    if (excluded >= 0) {         // ground the excluded vertex: unit row and column
        for (int64_t j = 0; j < n; ++j) {
            M[(size_t)excluded * n + j] = 0.0;
            M[(size_t)j * n + excluded] = 0.0;
        }
        M[(size_t)excluded * n + excluded] = 1.0;
    }
    if (dense::potrf_lower(n, M.data(), n, true) >= 0) {
        err = "multigrid: coarsest matrix is not positive definite";
        return false;
    }
    std::vector<double> Li((size_t)n * n);
    dense::trtri_lower(n, M.data(), n, Li.data(), true);
    inv.assign((size_t)n * n, 0.0);   // L^-T L^-1
#pragma omp parallel for schedule(dynamic, 8)
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = 0; j <= i; ++j) {
            double s = 0.0;
            for (int64_t k = i; k < n; ++k) s += Li[(size_t)k * n + i] * Li[(size_t)k * n + j];
            inv[(size_t)i * n + j] = s;
            inv[(size_t)j * n + i] = s;
        }
    if (excluded >= 0)
        for (int64_t j = 0; j < n; ++j) {
            inv[(size_t)excluded * n + j] = 0.0;
            inv[(size_t)j * n + excluded] = 0.0;
        }
    return true;
}

// Largest eigenvalue of D^-1 A (dinv = 0 on excluded rows) by Lanczos on
// D^-1/2 A D^-1/2 from the fixed start; Ritz values lie inside the
// spectrum, so the caller adds a margin.
double lambda_max_dinv(const Csr& A, const std::vector<double>& dinv, int steps) {
    const int64_t n = A.n;
    std::vector<double> s(n), v, vp(n, 0.0), w(n), t(n), al, be;
    for (int64_t i = 0; i < n; ++i) s[i] = std::sqrt(dinv[i]);
    if (!lanczos_start(dinv, v)) return 1.0;
    double beta = 0.0;
    steps = (int)std::min<int64_t>(steps, n);
    for (int j = 0; j < steps; ++j) {
        for (int64_t i = 0; i < n; ++i) t[i] = s[i] * v[i];
        spmv(A, t.data(), w.data());
        double a = 0.0;
        for (int64_t i = 0; i < n; ++i) {
            w[i] = s[i] * w[i] - beta * vp[i];
            a += w[i] * v[i];
        }
        double b = 0.0;
        for (int64_t i = 0; i < n; ++i) {
            w[i] -= a * v[i];
            b += w[i] * w[i];
        }
        al.push_back(a);
        b = std::sqrt(b);
        if (j + 1 == steps || b <= 1e-14 * std::fabs(a)) break;
        be.push_back(b);
        beta = b;
        for (int64_t i = 0; i < n; ++i) {
            vp[i] = v[i];
            v[i] = w[i] / b;
        }
    }
    return tridiag_largest(al, be);
}

}  // namespace

bool amg_build(const Csr& A0, int64_t excluded, const AmgOptions& opt, Amg& out, std::string& err) {
    auto t0 = std::chrono::steady_clock::now();
    out = Amg();
    out.excluded = excluded;
    out.smooth_steps = std::max(1, opt.smooth_steps);
    out.lanczos_steps = opt.lanczos_steps;
    out.smooth_ratio = opt.smooth_ratio;
    out.coarse_steps = opt.coarse_steps > 0 ? opt.coarse_steps : out.smooth_steps;
    Csr A = A0;
    // the order the aggregation visits a level's vertices: index order on
    // the finest level, the order the aggregates were made on the coarser
    std::vector<int64_t> visit(A0.n);
    std::iota(visit.begin(), visit.end(), 0);
    for (int lev = 0;; ++lev) {
        const int64_t n = A.n;
        AmgLevel L;
        L.dinv.assign(n, 0.0);
        std::vector<double> dg(n);
        for (int64_t i = 0; i < n; ++i) {
            dg[i] = diag_of(A, i);
            if (lev == 0 && i == excluded) continue;
            if (!(dg[i] > 0.0)) {
                err = "multigrid: non-positive diagonal at level " + std::to_string(lev);
                return false;
            }
            L.dinv[i] = 1.0 / dg[i];
        }
        const double lmax = lambda_max_dinv(A, L.dinv, opt.lanczos_steps);
        L.hi = 1.1 * lmax;
        L.lo = L.hi / opt.smooth_ratio;
        L.steps = lev == 0 ? out.smooth_steps : out.coarse_steps;
        const bool last = n <= opt.max_coarse || lev + 1 >= opt.max_levels;
        if (last) {
            if (!coarse_inverse(A, lev == 0 ? excluded : -1, out.coarse_inv, err)) return false;
            L.A = std::move(A);
            out.levels.push_back(std::move(L));
            break;
        }
        // strength of connection and aggregation; a level whose off-diagonal
        // couplings are weak against its diagonal (a mass-dominated K_m)
        // coarsens poorly at theta, so theta is lowered until it coarsens
        std::vector<int64_t> agg;
        int64_t na = 0;
        for (double th : {opt.theta, 0.25 * opt.theta, 0.0}) {
            std::vector<int64_t> sptr(n + 1, 0);
            std::vector<int32_t> scol;
            std::vector<double> sval;
            for (int64_t i = 0; i < n; ++i) {
                if (!(lev == 0 && i == excluded))
                    for (int64_t p = A.ptr[i]; p < A.ptr[i + 1]; ++p) {
                        const int64_t j = A.col[p];
                        if (j == i || (lev == 0 && j == excluded)) continue;
                        const double a = std::fabs(A.val[p]);
                        if (a > 0.0 && a >= th * std::sqrt(std::fabs(dg[i] * dg[j]))) {
                            scol.push_back((int32_t)j);
                            sval.push_back(a);
                        }
                    }
                sptr[i + 1] = (int64_t)scol.size();
            }
            agg.assign(n, -1);
            if (lev == 0 && excluded >= 0) agg[excluded] = -2;
            std::vector<int64_t> pos(n);
            for (int64_t k = 0; k < n; ++k) pos[visit[k]] = k;
            na = 0;
            for (int64_t k = 0; k < n; ++k) {              // pass 1
                const int64_t i = visit[k];
                if (agg[i] != -1 || sptr[i + 1] == sptr[i]) continue;
                bool free = true;
                for (int64_t p = sptr[i]; p < sptr[i + 1] && free; ++p) free = agg[scol[p]] == -1;
                if (!free) continue;
                agg[i] = na;
                for (int64_t p = sptr[i]; p < sptr[i + 1]; ++p) agg[scol[p]] = na;
                ++na;
            }
            const std::vector<int64_t> agg1 = agg;
            for (int64_t k = 0; k < n; ++k) {              // pass 2
                const int64_t i = visit[k];
                if (agg[i] != -1) continue;
                double best = -1.0;
                int64_t bpos = n;
                for (int64_t p = sptr[i]; p < sptr[i + 1]; ++p) {
                    const int64_t j = scol[p];
                    // equal strengths: the neighbour visited first
                    if (agg1[j] >= 0 && (sval[p] > best || (sval[p] == best && pos[j] < bpos))) {
                        best = sval[p];
                        bpos = pos[j];
                        agg[i] = agg1[j];
                    }
                }
            }
            for (int64_t k = 0; k < n; ++k) {              // pass 3
                const int64_t i = visit[k];
                if (agg[i] != -1) continue;
                agg[i] = na;
                for (int64_t p = sptr[i]; p < sptr[i + 1]; ++p)
                    if (agg[scol[p]] == -1) agg[scol[p]] = na;
                ++na;
            }
            if (na > 0 && (na <= n / 3 || th == 0.0)) break;
        }
        if (na == 0 || na > n - n / 8) {
            // no useful coarsening left: stop here and invert this level if it is small
            // enough, else give up
            if (n <= 8192) {
                AmgOptions o2 = opt;
                o2.max_coarse = (int)n;
                Amg tail;
                if (!amg_build(A, lev == 0 ? excluded : -1, o2, tail, err)) return false;
                L.A = std::move(A);
                L.P = Csr();
                L.R = Csr();
                out.coarse_inv = std::move(tail.coarse_inv);
                out.levels.push_back(std::move(L));
                break;
            }
            err = "multigrid: aggregation did not coarsen at level " + std::to_string(lev);
            return false;
        }
        // aggregates numbered by their first vertex; the next level is
        // visited in the order they were made
        {
            std::vector<int64_t> first(na, n), ord(na), id(na);
            for (int64_t i = 0; i < n; ++i)
                if (agg[i] >= 0) first[agg[i]] = std::min(first[agg[i]], i);
            std::iota(ord.begin(), ord.end(), 0);
            std::sort(ord.begin(), ord.end(), [&](int64_t a, int64_t b) { return first[a] < first[b]; });
            for (int64_t k = 0; k < na; ++k) id[ord[k]] = k;
            for (int64_t i = 0; i < n; ++i)
                if (agg[i] >= 0) agg[i] = id[agg[i]];
            visit = std::move(id);
        }
        // tentative prolongation (normalised constants per aggregate)
        std::vector<int64_t> asz(na, 0);
        for (int64_t i = 0; i < n; ++i)
            if (agg[i] >= 0) ++asz[agg[i]];
        Csr T;
        T.n = n;
        T.ptr.assign(n + 1, 0);
        for (int64_t i = 0; i < n; ++i) {
            if (agg[i] >= 0) {
                T.col.push_back((int32_t)agg[i]);
                T.val.push_back(1.0 / std::sqrt((double)asz[agg[i]]));
            }
            T.ptr[i + 1] = (int64_t)T.col.size();
        }
        // smoothed prolongation P = T - omega D^-1 A T
        const double omega = 4.0 / (3.0 * lmax);
        Csr AT = spgemm(A, T, na);
        Csr P;
        P.n = n;
        P.ptr.assign(n + 1, 0);
        {
            std::vector<int64_t> cnt(n, 0);
            std::vector<std::vector<std::pair<int32_t, double>>> rows(n);
#pragma omp parallel for schedule(dynamic, 1024)
            for (int64_t i = 0; i < n; ++i) {
                auto& r = rows[i];
                if (L.dinv[i] == 0.0) continue;        // excluded vertex: no coarse coupling
                const double f = omega * L.dinv[i];
                int64_t q = T.ptr[i];
                for (int64_t p = AT.ptr[i]; p < AT.ptr[i + 1]; ++p) {
                    double v = -f * AT.val[p];
                    if (q < T.ptr[i + 1] && T.col[q] == AT.col[p]) v += T.val[q++];
                    r.emplace_back(AT.col[p], v);
                }
                for (; q < T.ptr[i + 1]; ++q) r.emplace_back(T.col[q], T.val[q]);
                std::sort(r.begin(), r.end());
            }
            for (int64_t i = 0; i < n; ++i) P.ptr[i + 1] = P.ptr[i] + (int64_t)rows[i].size();
            P.col.resize(P.ptr[n]);
            P.val.resize(P.ptr[n]);
            for (int64_t i = 0; i < n; ++i) {
                int64_t o = P.ptr[i];
                for (auto& e : rows[i]) {
                    P.col[o] = e.first;
                    P.val[o++] = e.second;
                }
            }
        }
        Csr R = transpose(P, na);
        Csr AP = spgemm(A, P, na);
        Csr Ac = spgemm(R, AP, na);
        // exact symmetry of the coarse matrix (rounding of the two products)
        {
            Csr At = transpose(Ac, na);
            for (int64_t p = 0; p < Ac.nnz(); ++p) Ac.val[p] = 0.5 * (Ac.val[p] + At.val[p]);
        }
        L.A = std::move(A);
        L.P = std::move(P);
        L.R = std::move(R);
        out.levels.push_back(std::move(L));
        A = std::move(Ac);
    }
    int64_t nnz0 = out.levels[0].A.nnz(), nnz = 0;
    for (const auto& l : out.levels) nnz += l.A.nnz();
    out.op_complexity = nnz0 > 0 ? (double)nnz / (double)nnz0 : 1.0;
    out.setup_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    return true;
}

namespace {

// x = S b: `steps` Chebyshev steps on D^-1 A from x = 0 (the recurrence of
// chebyshev.cpp, with the level's interval).
void amg_smooth(const AmgLevel& L, int steps, const double* b, double* x) {
    const int64_t n = L.A.n;
    const ChebCoef cf = chebyshev_coefficients(L.lo, L.hi, steps);
    std::vector<double> r(b, b + n), d(n), q(n);
    for (int64_t i = 0; i < n; ++i) {
        d[i] = cf.inv_theta * L.dinv[i] * b[i];
        x[i] = d[i];
    }
    for (int k = 1; k < steps; ++k) {
        spmv(L.A, d.data(), q.data());
        for (int64_t i = 0; i < n; ++i) {
            r[i] -= q[i];
            d[i] = cf.c1[k - 1] * d[i] + cf.c2[k - 1] * L.dinv[i] * r[i];
            x[i] += d[i];
        }
    }
}

void vcycle(const Amg& M, size_t l, const double* b, double* x) {
    const AmgLevel& L = M.levels[l];
    const int64_t n = L.A.n;
    if (l + 1 == M.levels.size()) {
        for (int64_t i = 0; i < n; ++i) {
            double s = 0.0;
            for (int64_t j = 0; j < n; ++j) s += M.coarse_inv[(size_t)i * n + j] * b[j];
            x[i] = s;
        }
        return;
    }
    const int64_t nc = M.levels[l + 1].A.n;
    std::vector<double> r(n), t(n), rc(nc), ec(nc);
    amg_smooth(L, L.steps, b, x);
    spmv(L.A, x, r.data());
    for (int64_t i = 0; i < n; ++i) r[i] = b[i] - r[i];
    spmv(L.R, r.data(), rc.data());
    vcycle(M, l + 1, rc.data(), ec.data());
    spmv(L.P, ec.data(), t.data());
    for (int64_t i = 0; i < n; ++i) x[i] += t[i];
    spmv(L.A, x, r.data());
    for (int64_t i = 0; i < n; ++i) r[i] = b[i] - r[i];
    amg_smooth(L, L.steps, r.data(), t.data());
    for (int64_t i = 0; i < n; ++i) x[i] += t[i];
}

}  // namespace

bool amg_split_mass(Amg& M, const std::vector<double>& m0, double gamma, std::string& err) {
    M.mass.clear();
    if (M.levels.empty()) return true;
    Csr Ml = M.levels[0].A;
    if ((int64_t)m0.size() != Ml.n) { err = "mass vector size"; return false; }
    for (int64_t i = 0; i < Ml.n; ++i)
        for (int64_t p = Ml.ptr[i]; p < Ml.ptr[i + 1]; ++p) Ml.val[p] = Ml.col[p] == i ? m0[i] : 0.0;
    M.mass.push_back(Ml.val);
    for (size_t l = 0; l + 1 < M.levels.size(); ++l) {
        const AmgLevel& L = M.levels[l];
        const Csr& Ac = M.levels[l + 1].A;
        const int64_t nc = Ac.n;
        Csr Mc = spgemm(L.R, spgemm(Ml, L.P, nc), nc);
        Csr Mt = transpose(Mc, nc);
        for (int64_t p = 0; p < Mc.nnz(); ++p) Mc.val[p] = 0.5 * (Mc.val[p] + Mt.val[p]);
        if (Mc.ptr != Ac.ptr || Mc.col != Ac.col) {
            err = "multigrid: the mass part's pattern differs at level " + std::to_string(l + 1);
            return false;
        }
        M.mass.push_back(Mc.val);
        Ml = std::move(Mc);
    }
    M.gamma = gamma;
    return true;
}

bool amg_refresh_gamma(Amg& M, double gamma, std::string& err) {
    if (M.mass.size() != M.levels.size()) {
        err = "multigrid: no mass parts to refresh with";
        return false;
    }
    const double dg = gamma - M.gamma;
    for (size_t l = 0; l < M.levels.size(); ++l) {
        AmgLevel& L = M.levels[l];
        Csr& A = L.A;
        const int64_t n = A.n;
        for (int64_t p = 0; p < A.nnz(); ++p) A.val[p] += dg * M.mass[l][p];
        const bool last = l + 1 == M.levels.size();
        if (last) {
            if (!coarse_inverse(A, l == 0 ? M.excluded : -1, M.coarse_inv, err)) return false;
            break;
        }
        for (int64_t i = 0; i < n; ++i) {
            if (l == 0 && i == M.excluded) continue;
            const double d = diag_of(A, i);
            if (!(d > 0.0)) {
                err = "multigrid: non-positive diagonal at level " + std::to_string(l);
                return false;
            }
            L.dinv[i] = 1.0 / d;
        }
        L.hi = 1.1 * lambda_max_dinv(A, L.dinv, M.lanczos_steps);
        L.lo = L.hi / M.smooth_ratio;
    }
    M.gamma = gamma;
    return true;
}

void amg_apply(const Amg& M, const double* b, double* x) {
    if (M.levels.empty()) return;
    vcycle(M, 0, b, x);
    if (M.excluded >= 0) x[M.excluded] = 0.0;
}

}  // namespace bido
