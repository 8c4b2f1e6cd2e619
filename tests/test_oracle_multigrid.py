"""CPU pins of the multigrid inner preconditioner (an alternative P_1 ~ S_1
and P_K ~ K_m; Sec. 5.3 leaves both free).

The oracle V-cycle (oracle/multigrid.py) is pinned by properties that hold
for any hierarchy: with the identity as prolongation the cycle is the exact
solve; the cycle is a symmetric operator; for a symmetric positive definite
matrix and a convergent smoother the spectrum of B A lies in (0, 1]; the
excluded (grounded) vertex stays at zero.  The library's hierarchy is
checked for the Galerkin relation A_{l+1} = P_l^T A_l P_l, and its host
V-cycle against the oracle cycle on the same hierarchy."""
import numpy as np
import pytest
import scipy.sparse as sp

import workloads as w
from oracle import multigrid as mg


def _laplacian_2d(n, shift=0.0):
    """5-point Laplacian on an n x n grid with Dirichlet boundary, plus shift I."""
    e = np.ones(n)
    T = sp.diags([-e[:-1], 2 * e, -e[:-1]], [-1, 0, 1])
    I = sp.identity(n)
    return (sp.kron(I, T) + sp.kron(T, I) + shift * sp.identity(n * n)).tocsr()


def _pair_aggregation(n_fine):
    """Tentative prolongation of aggregates {2k, 2k+1} (plain, not smoothed)."""
    nc = (n_fine + 1) // 2
    rows = np.arange(n_fine)
    return sp.csr_matrix((np.full(n_fine, 1.0), (rows, rows // 2)), shape=(n_fine, nc))


def _level(A, P, hi_factor=1.1, ratio=10.0):
    d = A.diagonal()
    dinv = 1.0 / d
    lam = np.linalg.eigvalsh((sp.diags(np.sqrt(dinv)) @ A @ sp.diags(np.sqrt(dinv))).toarray()).max()
    return dict(A=A, P=P, dinv=dinv, lo=hi_factor * lam / ratio, hi=hi_factor * lam)


def test_identity_prolongation_gives_the_exact_solve():
    A = _laplacian_2d(6, 0.3)
    n = A.shape[0]
    levels = [_level(A, sp.identity(n, format="csr")), dict(A=A, P=None, dinv=A.diagonal() ** -1)]
    b = np.random.default_rng(0).normal(size=n)
    x = mg.vcycle(levels, 2, b)
    np.testing.assert_allclose(A @ x, b, rtol=0, atol=1e-12 * np.abs(b).max())


def test_single_level_is_the_exact_solve_with_excluded_vertex_at_zero():
    A = _laplacian_2d(5).tolil()
    n = A.shape[0]
    dinv = 1.0 / A.diagonal()
    dinv[-1] = 0.0
    b = np.random.default_rng(1).normal(size=n)
    x = mg.vcycle([dict(A=A.tocsr(), P=None, dinv=dinv)], 2, b)
    assert x[-1] == 0.0
    keep = np.arange(n - 1)
    Ad = A.toarray()[np.ix_(keep, keep)]
    np.testing.assert_allclose(Ad @ x[keep], b[keep], atol=1e-12 * np.abs(b).max())


@pytest.mark.parametrize("m", [1, 2, 3])
def test_vcycle_is_symmetric_and_contracting(m):
    """Three levels built by pair aggregation: B symmetric, spectrum of B A
    in (0, 1] (a symmetric V-cycle with Galerkin coarse matrices and a
    smoother with |1 - lambda q(lambda)| <= 1 on the spectrum)."""
    A0 = _laplacian_2d(8, 0.05)
    P0 = _pair_aggregation(A0.shape[0])
    A1 = (P0.T @ A0 @ P0).tocsr()
    P1 = _pair_aggregation(A1.shape[0])
    A2 = (P1.T @ A1 @ P1).tocsr()
    levels = [_level(A0, P0), _level(A1, P1), dict(A=A2, P=None, dinv=1.0 / A2.diagonal())]
    n = A0.shape[0]
    Bm = np.column_stack([mg.vcycle(levels, m, e) for e in np.eye(n)])
    assert np.abs(Bm - Bm.T).max() <= 1e-12 * np.abs(Bm).max()
    ev = np.linalg.eigvals(Bm @ A0.toarray()).real
    assert ev.min() > 0.0 and ev.max() <= 1.0 + 1e-10, (ev.min(), ev.max())
    # a missing post-smoothing or a wrong sign of the coarse correction breaks one of these
    assert ev.min() > 0.05


def test_two_grid_cycle_with_one_jacobi_step_is_the_written_out_propagator():
    """One smoothing step is the damped Jacobi sweep S = 2/(lo + hi) D^-1 (the
    degree-0 Chebyshev polynomial on [lo, hi]); a two-grid cycle with it has
    the error propagator I - B A = (I - S A)(I - P A_c^-1 P^T A)(I - S A).  The
    level's own step count (steps = 1) overrides the cycle's m = 3."""
    A = _laplacian_2d(6, 0.2)
    P = _pair_aggregation(A.shape[0])
    Ac = (P.T @ A @ P).tocsr()
    L0 = _level(A, P)
    L0["steps"] = 1
    levels = [L0, dict(A=Ac, P=None, dinv=1.0 / Ac.diagonal())]
    n = A.shape[0]
    Bm = np.column_stack([mg.vcycle(levels, 3, e) for e in np.eye(n)])
    Ad, Pd = A.toarray(), P.toarray()
    S = 2.0 / (L0["lo"] + L0["hi"]) * np.diag(L0["dinv"])
    I = np.eye(n)
    E = (I - S @ Ad) @ (I - Pd @ np.linalg.solve(Ac.toarray(), Pd.T @ Ad)) @ (I - S @ Ad)
    np.testing.assert_allclose(I - Bm @ Ad, E, atol=1e-12)


@pytest.mark.parametrize("mk", [lambda: w.slab3d(n=12), lambda: w.thorax2d(n_target=6000, seed=3),
                                lambda: w.square2d(n=20)], ids=["slab12", "thorax6000", "square20"])
def test_library_hierarchy_is_galerkin_and_its_cycle_is_the_oracle_cycle(mk):
    import paper_1711_08708_amd as B
    hs = B.HostSetup(mk(), eps_h=0.0, inner_p1=B.P1_AMG, inner_pk=B.PK_AMG)
    for which in (B.FACTOR_P1, B.FACTOR_PK):
        info = hs.amg_info(which)
        levels = [hs.amg_level(which, l) for l in range(info["levels"])]
        for a, b in zip(levels, levels[1:]):
            if a["P"] is None:
                continue
            G = (a["P"].T @ a["A"] @ a["P"]).toarray()
            np.testing.assert_allclose(b["A"].toarray(), G, atol=1e-12 * np.abs(G).max())
        # two Chebyshev steps on the finest level, the damped Jacobi sweep on
        # the coarser ones (the oracle cycle takes each level's count)
        assert levels[0]["steps"] == info["smooth_steps"] == 2
        assert all(l["steps"] == 1 for l in levels[1:])
        n = levels[0]["A"].shape[0]
        b = np.random.default_rng(5 + which).normal(size=n)
        xo = mg.vcycle(levels, info["smooth_steps"], b)
        xl = hs.amg_apply(which, b)
        err = np.linalg.norm(xl - xo) / np.linalg.norm(xo)
        print(which, info, "host vs oracle cycle", err)
        assert err <= 1e-11
        if which == B.FACTOR_P1:                                     # the grounded vertex
            g = np.flatnonzero(levels[0]["dinv"] == 0.0)
            assert len(g) == 1 and xl[g[0]] == 0.0 and xo[g[0]] == 0.0


def test_new_time_step_keeps_the_aggregation_and_moves_every_level():
    """A change of time step moves K_m = gamma M_H + S_m; the multigrid P_K
    keeps its prolongations and each level becomes the Galerkin product of
    the new K_m (checked level by level against P^T A P in NumPy), with new
    D^-1 and a smoother bound above the spectrum of D^-1 A; the library's
    host cycle is the oracle cycle on the moved hierarchy."""
    import paper_1711_08708_amd as B
    cfg = w.slab3d(n=10)
    hs = B.HostSetup(cfg, eps_h=0.0, inner_p1=B.P1_AMG, inner_pk=B.PK_AMG)
    info = hs.amg_info(B.FACTOR_PK)
    before = [hs.amg_level(B.FACTOR_PK, l) for l in range(info["levels"])]
    hs.set_dt(cfg["dt"] / 4)
    assert hs.amg_info(B.FACTOR_PK)["levels"] == info["levels"]
    after = [hs.amg_level(B.FACTOR_PK, l) for l in range(info["levels"])]
    K = hs.csr(B.MAT_KM)
    A = K
    for l, (b, a) in enumerate(zip(before, after)):
        np.testing.assert_allclose(a["A"].toarray(), A.toarray(), atol=1e-12 * abs(A).max())
        assert not np.allclose(a["A"].toarray(), b["A"].toarray())        # really moved
        if a["P"] is None:
            break
        assert (a["P"] != b["P"]).nnz == 0                                 # same transfer
        np.testing.assert_allclose(a["dinv"], 1.0 / a["A"].diagonal(), rtol=1e-14)
        lam = np.linalg.eigvalsh((sp.diags(np.sqrt(a["dinv"])) @ a["A"] @ sp.diags(np.sqrt(a["dinv"]))).toarray())
        assert lam.max() <= a["hi"] <= 1.2 * lam.max()
        G = (a["P"].T @ a["A"] @ a["P"])
        A = sp.csr_matrix(0.5 * (G + G.T))
    bvec = np.random.default_rng(9).normal(size=K.shape[0])
    xo = mg.vcycle(after, info["smooth_steps"], bvec)
    xl = hs.amg_apply(B.FACTOR_PK, bvec)
    assert np.linalg.norm(xl - xo) <= 1e-11 * np.linalg.norm(xo)


@pytest.mark.parametrize("n", [16, 24])
def test_multigrid_p1_converges_in_few_iterations(n):
    """CG on the grounded S_1 of a slab with the library's host V-cycle:
    the iteration count to 1e-10 stays small and nearly flat in the mesh
    size (a quality check of the hierarchy, not of the arithmetic)."""
    import paper_1711_08708_amd as B
    hs = B.HostSetup(w.slab3d(n=n), eps_h=0.0, inner_p1=B.P1_AMG)
    A = hs.amg_level(B.FACTOR_P1, 0)["A"]
    N = A.shape[0]
    g = np.flatnonzero(hs.amg_level(B.FACTOR_P1, 0)["dinv"] == 0.0)[0]    # the grounded vertex
    keep = np.arange(N) != g
    rng = np.random.default_rng(0)
    b = rng.normal(size=N)
    b[g] = 0.0
    b[keep] -= b[keep].mean()
    x = np.zeros(N)
    r = b.copy()
    z = hs.amg_apply(B.FACTOR_P1, r)
    p = z.copy()
    rz = r @ z
    for it in range(100):
        q = A @ p
        q[g] = 0.0
        a = rz / (p @ q)
        x += a * p
        r -= a * q
        if np.linalg.norm(r) <= 1e-10 * np.linalg.norm(b):
            break
        z = hs.amg_apply(B.FACTOR_P1, r)
        rz, rz_old = r @ z, rz
        p = z + (rz / rz_old) * p
    print("slab", n, "CG iterations with the multigrid P_1", it + 1, hs.amg_info(B.FACTOR_P1))
    assert it + 1 <= 25


def test_multigrid_blocks_take_a_banded_order():
    """A block that is not factored takes the reverse Cuthill-McKee order:
    the internal orders are permutations, u and v share one order when the
    heart is the whole mesh, and S_1 in that order has a band no wider than
    in the slab's own lexicographic numbering (about n^2 + n + 1 for an
    n^3 grid of cells); a factored block keeps nested dissection, whose
    separators couple far-apart indices."""
    import paper_1711_08708_amd as B
    n = 16
    cfg = w.slab3d(n=n)
    band = lambda M: np.abs(M.tocoo().row - M.tocoo().col).max()
    hs = B.HostSetup(cfg, eps_h=0.0, inner_p1=B.P1_AMG, inner_pk=B.PK_AMG)
    up, vp, heart = hs.index(B.IDX_UPOS), hs.index(B.IDX_VPOS), hs.index(B.IDX_HEART)
    N = len(up)
    assert sorted(up) == list(range(N)) and sorted(vp) == list(range(len(vp)))
    assert np.array_equal(up[heart], vp)
    S = hs.csr(B.MAT_S1)                        # caller's numbering
    perm = np.argsort(up)                       # internal -> caller
    Sint = S[perm][:, perm]
    print("band: caller order", band(S), "internal", band(Sint))
    assert band(Sint) <= band(S) <= (n + 1) ** 2 + (n + 1) + 1
    A0 = hs.amg_level(B.FACTOR_P1, 0)["A"]
    assert band(A0) == band(Sint)
    # the grounded vertex of the multigrid P_1: the one nearest the centroid
    g = np.flatnonzero(hs.amg_level(B.FACTOR_P1, 0)["dinv"] == 0.0)
    xyz = np.asarray(cfg["xyz"])
    dist = np.linalg.norm(xyz - xyz.mean(axis=0), axis=1)
    assert len(g) == 1 and dist[perm[g[0]]] == dist.min()
    hf = B.HostSetup(cfg, eps_h=0.0)
    upf = hf.index(B.IDX_UPOS)
    pf = np.argsort(upf)
    assert band(S[pf][:, pf]) > N // 2


def test_banded_orders_on_a_heart_torso_slice():
    """Heart and torso (the heart a part of the mesh): multigrid blocks take
    one reverse Cuthill-McKee order for u (over S_1's graph) and another for
    v (over S_i's graph on the heart); both are permutations and neither
    widens the band of its matrix against the generator's numbering."""
    import paper_1711_08708_amd as B
    cfg = w.thorax2d(n_target=3000, seed=4)
    band = lambda M: np.abs(M.tocoo().row - M.tocoo().col).max()
    hs = B.HostSetup(cfg, eps_h=0.0, inner_p1=B.P1_AMG, inner_pk=B.PK_AMG)
    up, vp = hs.index(B.IDX_UPOS), hs.index(B.IDX_VPOS)
    assert sorted(up) == list(range(len(up))) and sorted(vp) == list(range(len(vp)))
    assert len(vp) < len(up)
    S1, Si = hs.csr(B.MAT_S1), hs.csr(B.MAT_SI)
    pu, pv = np.argsort(up), np.argsort(vp)
    bu, bv = band(S1[pu][:, pu]), band(Si[pv][:, pv])
    print("bands: S_1", band(S1), "->", bu, " S_i", band(Si), "->", bv)
    assert bu <= band(S1) and bv <= band(Si)
    assert band(hs.amg_level(B.FACTOR_P1, 0)["A"]) == bu
