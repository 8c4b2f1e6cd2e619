// Host set-up of a solver context: everything bido_create computes before
// the upload to the device (also reachable without a GPU through the
// bido_host_* checks).
#pragma once
#include <string>
#include <vector>

#include "../../include/bido.h"
#include "host.h"

namespace bido {

// Lambda in blocked form when the heart is the whole mesh and u and v share
// one internal order (Pi = I): row k holds the columns c of S_1's row k and
// per column the pair {S_1[k,c], S_i[k,c]} (val, interleaved), and gm[k] =
// gamma m_k, so that
//   (Lambda x)_u[k] = sum_c S_1 x_u[c] + S_i x_v[c]
//   (Lambda x)_v[k] = sum_c S_i (x_u[c] + x_v[c]) + gm[k] x_v[k].
// n = 0: no blocked form.
struct LamBlocked {
    int64_t n = 0;
    std::vector<int64_t> ptr;
    std::vector<int32_t> col;
    std::vector<double> val, gm;
};

struct HostSetup {
    bido_params params{};
    Assembled A;
    Factor p1, pk;                 // factors of the grounded S_1 and of K_m (trees always;
                                   // fronts only when that block is factored)
    bool p1_factored = true, pk_factored = true;
    Amg amg1, amgk;                // multigrid hierarchies (inner_p1 / inner_pk = AMG)
    Csr lam;                       // Lambda, internal order [u (ND of S_1); v (ND of K_m)]
    LamBlocked lamb;               // its blocked form (heart = whole mesh), or n = 0
    Csr avu;                       // S_i Pi: N_H rows (v order), u columns
    Csr auv;                       // Pi^T S_i: N rows (u order), v columns
    std::vector<int64_t> u_pos;    // global id   -> internal u index
    std::vector<int64_t> v_pos;    // heart-local -> internal v index (0-based)
    std::vector<double> m_int;     // lumped M in internal u order
    std::vector<double> mh_loc;    // lumped M_H, heart-local order
    std::vector<double> stim_loc;  // stimulus amplitude per heart vertex (heart-local)
    int64_t stim_n0 = 0, stim_n1 = 0;
    double stim_t0 = 0.0, stim_t1 = 0.0;   // stimulus window [ms]
    double gamma = 0.0;
    double msum = 0.0;
    // learned correction: static vertex features (N_H x 15, heart-local order:
    // averaged conductivity entries / max diagonal value, then the hop distance
    // to the heart boundary / max) and the row-normalised |S_m| neighbour graph
    std::vector<double> gnn_static;
    Csr gnn_agg;
    Csr km_int;                    // K_m = gamma M_H + S_m in internal v order
    std::vector<double> xyz;       // the mesh (caller's numbering), for probe points
    std::vector<int32_t> elems;
    double setup_seconds = 0.0;
};

bool build_host(const bido_mesh* mesh, const bido_tissue* tissue, const bido_params* params,
                HostSetup& hs, std::string& err);

// New time step: gamma (the coefficient of M_H in Lambda and K_m, Sec. 3.2)
// and the stimulus step range follow dt; the v-v diagonal of Lambda and
// K_m are recomputed as at set-up (bit-identical to a set-up at dt).  With
// refactor, K_m is factored again in its elimination tree, or its multigrid
// hierarchy is moved to the new gamma on the same aggregation
// (amg_refresh_gamma); P_1 does not depend on dt.
bool host_set_dt(HostSetup& hs, double dt, bool refactor, std::string& err);

// The blocked form of hs.lam (LamBlocked); false when the heart is not the
// whole mesh, the u and v orders differ or the blocks do not match.
bool build_lam_blocked(const HostSetup& hs, LamBlocked& out);

}  // namespace bido
