// Host-side launch wrappers of the HIP kernels (implemented in kernels.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

#include "kernels.h"

namespace bido {

struct CsrDev {
    int64_t n = 0;
    int64_t nnz = 0;
    int64_t* ptr = nullptr;
    int32_t* col = nullptr;
    double* val = nullptr;
    // compact columns (or null): col[q] = cb[row] + c16[q] for every entry
    // of a row, when each row spans fewer than 65536 columns
    uint16_t* c16 = nullptr;
    int32_t* cb = nullptr;
    // index bytes of the products that read it: per entry and per row
    double col_bytes() const { return c16 ? 2.0 : 4.0; }
    double row_bytes() const { return c16 ? 12.0 : 8.0; }
};

// partial-sum scratch of k_dot_reduce (the last block reduces)
struct Reduce {
    double* partials = nullptr;   // 2 * max_blocks doubles
    unsigned* counter = nullptr;
    unsigned max_blocks = 2048;
};

struct IonicConst {
    double gamma, chi, cm, dt;
    double dv, inv_dv, inv_tau_in, inv_tau_out, inv_tau_open, inv_tau_close, v_gate;
    double scale;   // 1 (semi-implicit), 2 (Crank-Nicolson: the system times 2)
    double reaction; // 1: Steps 1 + 3; 0: diffusion sub-step of a splitting (no ionic term, gates kept)
};

// Execution plan of one factor's sweeps: the subtrees below the cut height
// hc run in one launch (one workgroup walks a whole subtree), the levels
// above it run one launch each.
struct TriTopLevel {
    TriItem* fwd = nullptr;   // device
    int n_fwd = 0;
    BwdItem* bwd = nullptr;   // device
    int n_bwd = 0;
    size_t lds_f = 0;         // forward: max column chunk * 8
    size_t lds_b = 0;         // backward: max staged rows * 8
    TriItem* fcomb = nullptr; // device: split forward tiles (combine launch)
    int n_fcomb = 0;
    BwdItem* bcomb = nullptr; // device: split backward tiles
    int n_bcomb = 0;
    int bwd_nt = 256;         // threads of a backward item (256 or 1024)
};
struct TriPlan {
    int hc = -1;                  // subtree cut height (-1: no subtree phase)
    int n_sub = 0;                // subtrees (workgroups of the subtree phase)
    int32_t* sub_nodes = nullptr; // device: node ids grouped by subtree, by height
    TriNode* sub_tn = nullptr;    // device: the same nodes' records, in that order
    int32_t* sub_hoff = nullptr;  // device: n_sub x (hc+2) height offsets
    int sub_maxw = 0;             // max nI below the cut
    int bwd_group_max = 2;        // backward subtree heights with <= this many nodes use wave groups
    double* scratch = nullptr;    // partial sums of split tiles
    const uint8_t* skip = nullptr; // device, per tree of a merged forest: 1 = leave its nodes alone
    // dense top (n_top = 0: none): x[top_pos] = S_top^-1 w_top
    int64_t n_top = 0;
    const int64_t* top_pos = nullptr;
    const uint8_t* top_zero = nullptr;
    const int32_t* top_gptr = nullptr;
    const int64_t* top_gsrc = nullptr;
    double* top_w = nullptr;
    // hierarchical top (n_hblocks > 0 or n_hleaves > 0): S_top^-1 as low-rank blocks
    int n_hblocks = 0, n_hleaves = 0, n_hcols = 0;
    const HodlrBlock* hblocks = nullptr;
    const HodlrLeaf* hleaves = nullptr;
    const int32_t* hanc = nullptr;
    const int32_t* hcols = nullptr;
    double* ht = nullptr;         // projections, 2k per block
};

// Row ranges of a batch of independent slices held in one union vector:
// block b works on rows [r0, r1) of slice `slice`; slice s owns blocks
// [b0, b1), starts at union row `base` and has `nu` rows of its first part.
struct SegBlock {
    int64_t r0, r1;
    int32_t slice, pad;
};
struct SegSlice {
    int64_t base, nu;
    int32_t b0, b1;
};
struct SegTable {
    int nblocks = 0;
    const SegBlock* blk = nullptr;   // device
    const SegSlice* sl = nullptr;    // device
};

// Fixed workspace of the allocation-free entry points (noalloc.hip): 64 MiB
// per GPU, held until the process ends.  noalloc_scratch returns its device
// address on `device` (looked up once per device; the caller's current
// device is left unchanged).  Every call on a GPU shares that GPU's array.
constexpr int64_t NOALLOC_SCRATCH_DOUBLES = int64_t(8) << 20;
hipError_t noalloc_scratch(int device, double** ptr);

void launch_fill(hipStream_t s, int64_t n, double* x, double v);
// Projected initial guess (kernels.hip): the states W_k of the last steps,
// newest first, with their ring slots; out[k] = W_k . y (Reduce: partials
// of GUESS_MAX x max_blocks); the Gram row and the small solve; x = W c.
constexpr int GUESS_MAX = 16;
struct GuessList {
    const double* v[GUESS_MAX] = {};
    int slot[GUESS_MAX] = {};
    int m = 0;
};
void launch_multidot(hipStream_t s, int64_t n, const GuessList& W, const double* y, Reduce rd, double* out);
void launch_guess_solve(hipStream_t s, const GuessList& W, const double* d, double* G, const double* b, double* c);
void launch_guess_combine(hipStream_t s, int64_t n, const GuessList& W, const double* c, double* x);
void launch_axpy(hipStream_t s, int64_t n, double a, const double* x, double* y);   // y += a x
void launch_add2(hipStream_t s, int64_t n, const double* a, const double* b, double* out);   // out = a + b
// A CSR matrix of a multigrid level with FP64 or FP32 values, and the lanes
// per row its products use (amg.hip).
template <typename T>
struct AmgMat {
    int64_t n = 0, nnz = 0;
    const int64_t* ptr = nullptr;
    const int32_t* col = nullptr;
    const T* val = nullptr;
    int group = 4;
    const uint16_t* c16 = nullptr;   // compact columns (CsrDev), read instead of col when set
    const int32_t* cb = nullptr;
};
// y = b + sign A x (b may be null); vector types as instantiated in amg.hip
template <typename T, typename XV, typename BV, typename YV>
void launch_amg_spmv(hipStream_t s, const AmgMat<T>& A, const XV* x, const BV* b, double sign, YV* y);
// the first two Chebyshev smoothing steps from z = 0 in one pass (see amg.hip)
template <typename T, typename BV, typename VV, typename ZV>
void launch_amg_smooth2(hipStream_t s, const AmgMat<T>& A, const VV* dinv, const BV* b, double a0, double c1,
                        double c2, const VV* base, ZV* z, VV* r1, VV* d0, VV* d1, bool write_rd);
// A new gamma for a multigrid level (see amg.hip): A += dg M (FP64 and FP32
// copies), D^-1 (0 on the excluded row, < 0: none), A D^-1, the Lanczos
// steps of the smoother bound, and the dense inverse of the coarsest level
// (m: n x n output, f: n scratch; Gauss-Jordan, one pivot per launch)
void launch_amg_shift(hipStream_t s, int64_t nnz, double dg, const double* mass, double* a64, float* a32);
void launch_amg_dinv(hipStream_t s, int64_t n, const int64_t* ptr, const int32_t* col, const double* val,
                     int64_t excluded, double* dinv, float* dinv32);
void launch_amg_colscale(hipStream_t s, int64_t nnz, const int32_t* col, const double* val, const double* dinv,
                         double* s64, float* s32);
void launch_lz_in(hipStream_t s, int64_t n, const double* dinv, const double* v, double* t);
void launch_lz_w(hipStream_t s, int64_t n, const double* dinv, const double* y, double beta, const double* vp,
                 double* w);
void launch_lz_next(hipStream_t s, int64_t n, const double* w, double inv_b, double* v, double* vp);
void launch_amg_dense_inverse(hipStream_t s, int64_t n, const int64_t* ptr, const int32_t* col, const double* val,
                              int64_t excluded, double* m, double* f);
// z = base + a0 D^-1 b (base may be null): one Chebyshev step from zero
template <typename BV, typename VV, typename ZV>
void launch_amg_jacobi(hipStream_t s, int64_t n, const BV* b, const VV* dinv, double a0, const VV* base, ZV* z);
// one further Chebyshev step: r -= A dp, dn = c1 dp + c2 D^-1 r, z += dn
template <typename T>
void launch_amg_cheb(hipStream_t s, const AmgMat<T>& A, const double* dinv, double* r, const double* dp, double* dn,
                     double* z, double c1, double c2);
// per-slice stopping test of a fused batch after a PCG iteration (batch.hip):
// status 0 converged, 1 breakdown, 2 iteration cap (set together with done)
void launch_seg_stop(hipStream_t s, int S, const SegTable& T, const double* part_rr, const double* sc, int rho_slot,
                     const double* yy, const double* tol, const int* max_it, uint8_t* done, int* iters, int* status,
                     double* rel);
// y = A x, A dense n x n row-major (the coarsest level of a multigrid V-cycle)
template <typename V>
void launch_dense_gemv(hipStream_t s, int64_t n, const double* A, const V* x, V* y);
void launch_scatter_in(hipStream_t s, int64_t n, const int64_t* pos, const double* src, double* dst);
void launch_scatter_in_f(hipStream_t s, int64_t n, const int64_t* pos, const float* src, float* dst);
void launch_gather_f(hipStream_t s, int64_t n, const int64_t* pos, const float* src, float* dst);
void launch_gather_out(hipStream_t s, int64_t n, const int64_t* pos, const double* src, double* dst,
                       const double* sc, int shift_slot, double shift_den);
// Strang splitting: Heun half-steps tau of the reaction before (vs = V*,
// h <- h*) and after (v <- V^{n+1} from V** = x2[pos], h <- h^{n+1}; act:
// activation times as in launch_gather_v_act) the diffusion step
void launch_strang_in(hipStream_t s, int64_t nh, const double* v, double* h, const double* stim, double stim_on,
                      double tau, const IonicConst& c, double* vs);
void launch_strang_out(hipStream_t s, int64_t nh, const int64_t* pos, const double* x2, double* v, double* h,
                       const double* stim, double stim_on, double tau, const IonicConst& c, double* act, double v_act,
                       double t_n, double dt);
// v write-back with activation times (first time v reaches v_act, linear
// in time between t_n and t_n + dt; act < 0 = not reached)
void launch_gather_v_act(hipStream_t s, int64_t n, const int64_t* pos, const double* src, double* dst, double* act,
                         double v_act, double t_n, double dt);
// out[q] = sum_k wts[q nv + k] u[ids[q nv + k]]
void launch_probe(hipStream_t s, int np, int nv, const int64_t* ids, const double* wts, const double* u,
                  double* out);
void launch_dot_reduce(hipStream_t s, int64_t n, const double* a, const double* b, Reduce rd, double* out);
void launch_shift(hipStream_t s, int64_t n, double* x, const double* sc, int slot, double den);
// y2[pos] = scale M_H (gamma V - chi (I_ion - I_st)) - sub[pos] (sub may be
// null), x2[pos] = V, gates advanced
void launch_ionic(hipStream_t s, int64_t nh, const double* v, double* h, const double* stim,
                  double stim_on, const double* mh, const int64_t* pos, double* y2, double* x2,
                  const double* sub, const IonicConst& c);
// Each returns its grid size: the number of block partials it wrote.
// Lambda in blocked form when the heart is the whole mesh and u and v share
// one internal order (Pi = I): per row k one position list (column c,
// values {S_1[k,c], S_i[k,c]} interleaved) and gm[k] = gamma m_k, so that
//   (Lambda x)_u[k] = sum S_1 x_u[c] + S_i x_v[c]
//   (Lambda x)_v[k] = sum S_i (x_u[c] + x_v[c]) + gm[k] x_v[k]
// read 20 bytes per position instead of 48 for the four CSR blocks.
struct LamBlk {
    int64_t n = 0, npos = 0;           // rows (N = N_H) and positions
    int64_t* ptr = nullptr;             // n + 1
    int32_t* col = nullptr;             // npos
    double* val = nullptr;              // 2 npos: S_1, S_i per position
    double* gm = nullptr;               // n
    uint16_t* c16 = nullptr;            // compact columns (or null): col = cb[row] + c16
    int32_t* cb = nullptr;
    bool on() const { return n > 0; }
};
// the Lambda product on the blocked form (modes and partials of
// launch_spmv_lambda); returns the number of partials
unsigned launch_spmv_lam_blk(hipStream_t s, const LamBlk& A, int group, int mode, const double* x, const double* y,
                             double* out, double* pp);
unsigned launch_spmv_lambda(hipStream_t s, const CsrDev& A, int group, int mode, const double* x,
                            const double* y, double* out, double* pp);
void launch_spmv_csr(hipStream_t s, const CsrDev& A, int group, const double* x, const double* b,
                     double* y);
// P_K by Chebyshev-accelerated Jacobi on K_m: d = z = inv_theta D^-1 t, then
// per step r = r_in - K dp, dn = c1 dp + c2 D^-1 r, z += dn (r, dn not
// written on the last step; r_in may equal r; dp and dn must differ)
void launch_cheb_init(hipStream_t s, int64_t n, const double* t, const double* dinv, double inv_theta, double* d,
                      double* z);
void launch_cheb_step(hipStream_t s, const CsrDev& K, int group, const double* dinv, const double* r_in, double* r,
                      const double* dp, double* dn, double* z, double c1, double c2, bool last);
// dense top of a sweep: gather w_top from b and the bottom roots' updates,
// then x[top_pos] = S_top^-1 w_top (inv: n_top x n_top row-major, or the
// value array of the hierarchical form)
template <typename T>
void launch_tri_top(hipStream_t s, const TriPlan& P, const T* inv, const double* b, const double* upd,
                    double* x);
unsigned launch_pcg_update(hipStream_t s, int64_t n, double* x, double* r, double* r_old, const double* p,
                           const double* q, double* pp, unsigned nb_pq, int rho_slot);
unsigned launch_combine_dot(hipStream_t s, int64_t n1, int64_t n, double* z, const double* a, const double* b,
                            const double* r, const double* r_old, double* pp);
void launch_p_update(hipStream_t s, int64_t n, const double* z, double* p, double* pp, unsigned nb_rz, int first,
                     int flexible, int rho_old_slot, int rho_new_slot);

template <typename T>
void launch_tri_fwd_sub(hipStream_t s, const TriPlan& P, const TriNode* nodes, const T* panel,
                        const Ea* ea, const double* b, double* y, double* upd);
template <typename T>
void launch_tri_bwd_sub(hipStream_t s, const TriPlan& P, const TriNode* nodes, const T* panel,
                        const int64_t* bidx, const double* y, double* x);
template <typename T>
void launch_tri_fwd_lvl(hipStream_t s, const TriTopLevel& L, const TriPlan& P, const TriNode* nodes,
                        const T* panel_cm, const Ea* ea, const double* b, double* y, double* upd);
template <typename T>
void launch_tri_bwd_lvl(hipStream_t s, const TriTopLevel& L, const TriPlan& P, const TriNode* nodes,
                        const T* panel, const int64_t* bidx, const double* y, double* x);

// Segmented PCG kernels of a batch (batch.hip).  Scalars are per slice:
// rho[s], done[s] (1: frozen; its blocks do nothing, except in the residual
// SpMV of mode 1, which passes done = null), pq_out[s], rho_new[s]; partial
// regions have one entry per block of the table.
void launch_seg_spmv(hipStream_t s, const SegTable& T, const CsrDev& A, int group, int mode, const double* x,
                     const double* y, double* out, double* part0, double* part1, const uint8_t* done);
void launch_seg_csr(hipStream_t s, const SegTable& T, const CsrDev& A, int group, const double* x, const double* b,
                    double* y, const uint8_t* done);
// Chebyshev P_K per slice (coefficients indexed by slice; see launch_cheb_*)
void launch_seg_cheb_init(hipStream_t s, const SegTable& T, const double* t, const double* dinv,
                          const double* inv_theta, double* d, double* z, const uint8_t* done);
void launch_seg_cheb_step(hipStream_t s, const SegTable& T, const CsrDev& K, int group, const double* dinv,
                          const double* r_in, double* r, const double* dp, double* dn, double* z, const double* c1,
                          const double* c2, bool last, const uint8_t* done);
void launch_seg_pcg_update(hipStream_t s, const SegTable& T, double* x, double* r, double* r_old, const double* p,
                           const double* q, const double* part_pq, double* part_rr, const double* rho,
                           const uint8_t* done, double* pq_out);
void launch_seg_combine(hipStream_t s, const SegTable& T, double* z, const double* a, const double* b,
                        const double* r, const double* r_old, double* part_rz, double* part_zro,
                        const uint8_t* done);
void launch_seg_p_update(hipStream_t s, const SegTable& T, const double* z, double* p, const double* part_rz,
                         const double* part_zro, int first, int flexible, const double* rho_old, double* rho_new,
                         const uint8_t* done);

}  // namespace bido
