// Host-side set-up of the bidomain solver: P1 assembly, nested-dissection
// ordering, multifrontal Cholesky and hierarchical (low-rank) compression of
// the inner-solve factors.  Pure C++ (no HIP); compiled into libbido.so.
#pragma once
#include <cstdint>
#include <map>
#include <memory>
#include <string>
#include <vector>

#include "kernels.h"

namespace bido {

// Compressed sparse rows with int64 row pointers and int32 columns.
struct Csr {
    int64_t n = 0;
    std::vector<int64_t> ptr;
    std::vector<int32_t> col;
    std::vector<double> val;
    int64_t nnz() const { return (int64_t)col.size(); }
};

struct MeshIn {
    int dim = 2;
    int64_t n_nodes = 0, n_elems = 0;
    const double* xyz = nullptr;
    const int32_t* elems = nullptr;
    const int8_t* region = nullptr;
    const double* fibre = nullptr;
    const double* region_sigma = nullptr;
    int n_region_sigma = 0;
    double sigma_i[3] = {0, 0, 0}, sigma_e[3] = {0, 0, 0};
};

// Matrices of Sec. 3.1 and Sec. 5.2 in the caller's numbering:
// S1 (N x N, sigma_1 on Omega), Si and Sm (N_H x N_H on heart elements,
// heart-local numbering = heart vertices in ascending global id),
// lumped masses m (N) and mH (N_H).
struct Assembled {
    int dim = 2;
    int64_t N = 0, NH = 0;
    std::vector<int64_t> heart;       // heart-local -> global id
    std::vector<int64_t> heart_loc;   // global -> heart-local or -1
    Csr S1, Si, Sm;
    std::vector<double> m, mH;
};

bool assemble(const MeshIn& in, Assembled& out, std::string& err);

// ---------------------------------------------------------------------
// Nested dissection (domain-decomposition clustering).
// ---------------------------------------------------------------------
struct NdNode {
    int64_t begin = 0, end = 0;     // own index range [begin, end) (new order)
    int64_t sub_begin = 0;          // first index of the subtree
    int parent = -1;
    int child[2] = {-1, -1};
    int height = 0;                 // 0 for leaves
    int depth = 0;                  // 0 for the root
    int nchild() const { return (child[0] >= 0) + (child[1] >= 0); }
};

struct NdTree {
    std::vector<NdNode> nodes;      // post-order (children before parents)
    std::vector<int64_t> perm;      // new -> old
    std::vector<int64_t> iperm;     // old -> new
    int root = -1;
    int height = 0;
};

// Build the tree for a symmetric pattern `g` (n x n) with coordinates
// xyz (n x dim).  Leaves hold at most `leaf` vertices.
void nested_dissection(const Csr& g, const double* xyz, int dim, int leaf,
                       NdTree& t);

// Reverse Cuthill-McKee order of a symmetric pattern: only t.perm and
// t.iperm are set (the order of the inner solves that need no factor).
void rcm_order(const Csr& g, NdTree& t);

// Symmetric permutation B = P A P^T with perm = new -> old.
Csr permute(const Csr& a, const std::vector<int64_t>& perm,
            const std::vector<int64_t>& iperm);

// ---------------------------------------------------------------------
// Multifrontal Cholesky on the nested-dissection tree.
//
// For every tree node t with own indices I_t and boundary B(t) (ancestor
// indices coupled to the subtree of t), the factor is stored as the panel
//     P_t = [ L_tt^{-1} ; L_Bt L_tt^{-1} ]     ((nI + nB) x nI)
// so that the forward solve of L y = b is  [y_t; c_t] = P_t w_t  (c_t is the
// contribution subtracted from the boundary) and the backward solve of
// L^T x = y is  x_t = P_t^T [y_t; -x_B].
// ---------------------------------------------------------------------
struct Front {
    int node = -1;
    int64_t off = 0;                 // first own index
    int nI = 0, nB = 0;
    std::vector<int64_t> B;          // boundary indices (sorted, new order)
    std::vector<double> P;           // dense panel, (nI+nB) x nI row-major
};

struct Hodlr {
    int64_t n = 0, t_size = 1;
    int max_rank = 0;
    std::vector<HodlrBlock> blocks;
    std::vector<HodlrLeaf> leaves;
    std::vector<int32_t> anc;
    std::vector<double> val;
};

// The top of a factor's execution plan for one cut height: its vertices
// (tree order), the bottom roots' update entries to gather, and S_top^-1,
// dense or in hierarchical form (then in bisection order, with the list of
// projection columns).
struct TopPart {
    double eps = 0.0;
    int64_t n_top = 0;
    std::vector<int64_t> pos;
    std::vector<int32_t> gptr;
    std::vector<int64_t> gsrc;
    std::vector<double> inv;
    bool hodlr = false;
    Hodlr hd;
    std::vector<int32_t> cols;
    double seconds = 0.0;
};

struct Factor {
    int64_t n = 0;
    int64_t ground = -1;             // grounded index (new order) or -1
    std::vector<int64_t> grounds;    // every grounded index (several in a merged forest)
    NdTree tree;
    std::vector<Front> fronts;       // indexed like tree.nodes
    // accuracy of the hierarchical top (eps = 0: exact); vertex coordinates in
    // tree order (the top's bisection order is built from them)
    double eps = 0.0;
    int dim = 0;
    std::vector<double> xyz;
    // tops of earlier plans, by cut height (plans built again while tuning
    // reuse them); clear_top_cache() frees them
    mutable std::map<int, std::shared_ptr<const TopPart>> top_cache;
    void clear_top_cache() const { top_cache.clear(); }
    // keep only the hierarchical top of cut `keep` (small; a merged forest
    // reuses it)
    void trim_top_cache(int keep) const {
        for (auto it = top_cache.begin(); it != top_cache.end();)
            it = (it->first == keep && it->second->hodlr) ? std::next(it) : top_cache.erase(it);
    }
    // merged forest: the factors it was built from (only read while they
    // live), their index offsets, first node ids and the top cut of each
    // (-1: the cost model's)
    std::vector<const Factor*> parts;
    std::vector<int64_t> part_off;
    std::vector<int> part_node0, part_top_h;
    int64_t dense_entries() const;   // panel entries (lower triangles + boundary blocks)
};

// Factor the SPD matrix a (already in tree order).  If ground >= 0 the
// row and column `ground` are replaced by the unit vector first.
bool multifrontal(const Csr& a, Factor& f, int64_t ground, int n_threads,
                  std::string& err);

// Record the accuracy eps and the vertex coordinates (tree order) of a
// factor; the execution plan then holds the inverse of the top separators'
// Schur complement in hierarchical low-rank form at eps (exact panels below).
void set_top_compression(Factor& f, const double* xyz, int dim, double eps);

// Rank-revealing QR truncation: B (m x n row-major, leading dimension ld)
// ~ U V^T, U (m x k) and V (n x k) column-major, stopping at the first pivot
// below eps times the first one or below abs_tol.
void rrqr_lowrank(const double* B, int64_t ld, int m, int n, double eps, std::vector<double>& U,
                  std::vector<double>& V, int& k, double abs_tol = 0.0);

// Recursive geometric bisection order of n points (leaves of <= leaf points).
void hodlr_order(int64_t n, const double* xyz, int dim, int leaf, std::vector<int64_t>& ord);
// Hierarchical form of the symmetric n x n row-major A (bisection order).
void hodlr_build(const std::vector<double>& A, int64_t n, double eps, int leaf, int n_threads, Hodlr& h);
// y = A w from the hierarchical form.
void hodlr_apply(const Hodlr& h, const double* w, double* y);

// Factor of a block-diagonal matrix from the factors of its blocks: block s
// at indices [offs[s], offs[s] + n_s) of n_total; the trees become a forest.
void merge_factors(const std::vector<const Factor*>& fs, const std::vector<int64_t>& offs, int64_t n_total,
                   Factor& out);

// Host application of the factor (test hook): x = (L L^T)^-1 b with the
// grounded entry fixed to zero.
void host_solve(const Factor& f, const double* b, double* x);

// Smoothed-aggregation multigrid (amg.cpp): level l holds its matrix A,
// the smoother's D^-1 (0 at an excluded vertex) and interval [lo, hi] of
// D^-1 A, and (all but the coarsest) the prolongation P (n_l x n_{l+1}) and
// R = P^T; the coarsest matrix is held as its dense inverse.
struct AmgLevel {
    Csr A, P, R;
    std::vector<double> dinv;
    double lo = 0.0, hi = 0.0;
    int steps = 2;                    // Chebyshev steps per smoothing on this level
};
struct Amg {
    std::vector<AmgLevel> levels;
    std::vector<double> coarse_inv;   // n_c x n_c row-major
    int64_t excluded = -1;            // fine vertex held at zero (grounded), or -1
    int smooth_steps = 2;             // Chebyshev steps per smoothing on the finest level
    int coarse_steps = 2;             // ... and on the coarser ones
    // K_m = gamma M_H + S_m: the Galerkin mass part of every level's matrix on
    // its pattern (amg_split_mass), so that a new gamma needs no new
    // aggregation: A_l(gamma') = A_l + (gamma' - gamma) M_l
    std::vector<std::vector<double>> mass;
    double gamma = 0.0;
    int lanczos_steps = 20;           // of the smoother bounds (as built)
    double smooth_ratio = 10.0;
    double op_complexity = 1.0;       // sum of nnz over levels / nnz of A_0
    double setup_seconds = 0.0;
};
struct AmgOptions {
    double theta = 0.08;        // strength threshold
    int max_coarse = 1024;      // coarsest size
    int max_levels = 16;
    int smooth_steps = 2;       // Chebyshev steps (degree of the smoother polynomial), finest level
    int coarse_steps = 1;       // the same on the coarser levels (0: smooth_steps)
    double smooth_ratio = 10.0; // smoother interval [hi / ratio, hi]
    int lanczos_steps = 20;     // estimate of lambda_max(D^-1 A) per level
};
bool amg_build(const Csr& A, int64_t excluded, const AmgOptions& opt, Amg& out, std::string& err);
// The mass part of every level (m0: the diagonal mass of the finest level,
// A_0 = gamma diag(m0) + S): M_0 = diag(m0) on A_0's pattern, M_{l+1} =
// P_l^T M_l P_l symmetrised as the levels are, checked to share A_{l+1}'s
// pattern.
bool amg_split_mass(Amg& M, const std::vector<double>& m0, double gamma, std::string& err);
// A new gamma on the same aggregation and transfer operators: A_l += (gamma
// - M.gamma) M_l on every level, new D_l^-1 and smoother bounds (the same
// Lanczos estimate as at build), the coarsest inverse again.
bool amg_refresh_gamma(Amg& M, double gamma, std::string& err);
// The fixed start vector of the Lanczos estimates (zero where dinv = 0),
// normalised, and the largest eigenvalue of a symmetric tridiagonal matrix.
bool lanczos_start(const std::vector<double>& dinv, std::vector<double>& v);
double tridiag_largest(const std::vector<double>& al, const std::vector<double>& be);
// Host V-cycle x = B b (the device apply in FP64 order-independent form; a
// check hook).
void amg_apply(const Amg& M, const double* b, double* x);

// Chebyshev-accelerated Jacobi iteration for P_K ~ K_m (chebyshev.cpp).
// Interval for the spectrum of D^-1 K (D = diag K): rigorous bounds
// [min gamma m_i / K_ii, Gershgorin] (gm = gamma M_H in the order of K),
// the extreme Ritz values of `lanczos_steps` Lanczos steps, and the interval
// used: [max(bound_lo, ritz_lo), min(bound_hi, 1.05 ritz_hi)].
struct ChebInterval { double lo = 0, hi = 0, ritz_lo = 0, ritz_hi = 0, bound_lo = 0, bound_hi = 0; };
bool chebyshev_interval(const Csr& K, const std::vector<double>& gm, int lanczos_steps, ChebInterval& out,
                        std::string& err);
// Step coefficients on [lo, hi]: d_0 = inv_theta D^-1 t, then for k >= 1
// d_k = c1[k-1] d_{k-1} + c2[k-1] D^-1 r_k (steps - 1 entries).
struct ChebCoef { double inv_theta = 0; std::vector<double> c1, c2; };
ChebCoef chebyshev_coefficients(double lo, double hi, int steps);

// Element and barycentric weights of each of np points (np x dim, row-major)
// in the mesh (xyz: vertices x dim, elems: elements x (dim+1)); a point on
// shared faces goes to the element it is deepest in.  False if a point lies
// outside every element.
bool locate_points(int dim, const std::vector<double>& xyz, const std::vector<int32_t>& elems, const double* pts,
                   int np, std::vector<int64_t>& ids, std::vector<double>& wts, std::string& err);

}  // namespace bido
