"""Pins for the block algebra of Sec. 4 and the preconditioner of Sec. 5."""
import numpy as np
import pytest

import workloads as w
from oracle import bidomain as bd
from oracle import blocklu as bl


@pytest.fixture(scope="module")
def blocks():
    s = bd.System(w.square2d(n=12))
    return s, bl.dense_blocks(s)


def test_pseudo_inverse_definition(blocks):
    """Def. 1: S^+ S = S S^+ = orthogonal projection on 1^perp."""
    _, b = blocks
    S = b["S1"]
    Sp = bl.pinv_kernel1(S)
    n = S.shape[0]
    P = np.eye(n) - np.ones((n, n)) / n
    np.testing.assert_allclose(Sp @ S, P, atol=1e-9)
    np.testing.assert_allclose(S @ Sp, P, atol=1e-9)
    np.testing.assert_allclose(Sp, np.linalg.pinv(S, rcond=1e-12), atol=1e-8)


def test_block_lu(blocks):
    """Prop. 2: Lambda = L U and the Schur complement K is SPD."""
    s, b = blocks
    L, U, Lp, Uinv, K = bl.LU_factors(b)
    Lam = s.Lam.toarray()
    np.testing.assert_allclose(L @ U, Lam, atol=1e-9 * np.abs(Lam).max())
    np.testing.assert_allclose(K, K.T, atol=1e-9)
    assert np.linalg.eigvalsh(K).min() > 0


def test_harmonic_mean_form(blocks):
    """Rem. 1 (and its proof): K_0 = K - gamma M_H inverts
    A = S_i^+ + Pi S_e^+ Pi^T on the orthogonal of 1_H."""
    _, b = blocks
    K = bl.schur_K(b)
    K0 = K - b["gamma"] * b["MH"]
    A = bl.pinv_kernel1(b["Si"]) + b["Pi"] @ bl.pinv_kernel1(b["Se"]) @ b["Pi"].T
    rng = np.random.default_rng(3)
    for _ in range(3):
        V = rng.normal(size=b["NH"])
        V -= V.mean()
        np.testing.assert_allclose(K0 @ (A @ V), V, atol=1e-8 * np.abs(V).max())
    # K_0 annihilates the constants
    np.testing.assert_allclose(K0 @ np.ones(b["NH"]), 0.0, atol=1e-9)


def test_pseudo_inverse_solution(blocks):
    """Prop. 3: L L^+ = diag(p_Omega, id) and X = U^-1 L^+ Y solves the
    system for Y in the range."""
    s, b = blocks
    L, U, Lp, Uinv, K = bl.LU_factors(b)
    N, NH = b["N"], b["NH"]
    D = np.zeros((N + NH, N + NH))
    D[:N, :N] = np.eye(N) - np.ones((N, N)) / N
    D[N:, N:] = np.eye(NH)
    np.testing.assert_allclose(L @ Lp, D, atol=1e-8)
    np.testing.assert_allclose(Uinv @ U, np.eye(N + NH), atol=1e-9)
    rng = np.random.default_rng(4)
    Y = s.rhs(rng.uniform(0, 100, NH), rng.uniform(0, 1, NH), 0)
    X = Uinv @ (Lp @ Y)
    Lam = s.Lam.toarray()
    assert np.linalg.norm(Lam @ X - Y) < 1e-10 * np.linalg.norm(Y)


def test_exact_inner_solves_converge_in_one_iteration(blocks):
    """Sec. 5.3: with exact inner solves the block-LU preconditioned CG
    converges in a single iteration.  P_1^-1 is the grounded inverse of S_1
    (a generalised inverse on the range), P_K the exact Schur complement."""
    s, b = blocks
    P1 = bl.grounded_solver(b["S1"])
    PK = bl.chol_solver(bl.schur_K(b))
    rng = np.random.default_rng(5)
    Y = s.rhs(rng.uniform(0, 100, b["NH"]), rng.uniform(0, 1, b["NH"]), 0)
    x, it, hist = bl.pcg(s.Lam, Y, bl.block_prec(b, P1, PK), tol=1e-10)
    assert it == 1
    assert bd.rel_err(s.normalise(x), s.solve_dense(Y)) < 1e-10


def test_monodomain_exact_for_equal_anisotropy():
    """Sec. 5.2 / Sec. 1: for an isolated heart with sigma_e = lambda
    sigma_i the monodomain matrix K_m equals K, so PCG takes one iteration."""
    cfg = w.slab3d(n=3)
    cfg["sigma_e"] = 0.7 * cfg["sigma_i"]
    s = bd.System(cfg)
    b = bl.dense_blocks(s)
    K, Km = bl.schur_K(b), bl.K_monodomain(b)
    np.testing.assert_allclose(Km, K, atol=1e-10 * np.abs(K).max())
    P1 = bl.grounded_solver(b["S1"])
    Y = s.rhs(np.linspace(0, 90, s.NH), np.ones(s.NH), 0)
    _, it, _ = bl.pcg(s.Lam, Y, bl.block_prec(b, P1, bl.chol_solver(Km)), tol=1e-10)
    assert it == 1


def test_monodomain_is_an_approximation(blocks):
    """For unequal anisotropy ratios K_m differs from K and PCG needs a few
    iterations, still converging to the same normalised solution."""
    s, b = blocks
    K, Km = bl.schur_K(b), bl.K_monodomain(b)
    assert np.abs(K - Km).max() > 1e-6 * np.abs(K).max()
    P1 = bl.grounded_solver(b["S1"])
    Y = s.rhs(np.linspace(0, 90, b["NH"]), np.ones(b["NH"]), 0)
    x, it, hist = bl.pcg(s.Lam, Y, bl.block_prec(b, P1, bl.chol_solver(Km)), tol=1e-10)
    assert 1 < it < 20
    assert bd.rel_err(s.normalise(x), s.solve_dense(Y)) < 1e-8


def test_iterations_stay_bounded_under_refinement():
    """Sec. 5 and 6: with exact P_1 and P_K = K_m the preconditioned
    spectrum does not depend on the mesh size, so the PCG iteration count of
    the block-LU / monodomain preconditioner stays flat (up to a log factor)
    while the mesh is refined 4x per direction."""
    its = []
    for n in (12, 24, 48):
        s = bd.System(w.square2d(n=n, seed=0))
        b = bl.dense_blocks(s)
        P1 = bl.grounded_solver(b["S1"])
        PK = bl.chol_solver(bl.K_monodomain(b))
        rng = np.random.default_rng(3)
        Y = s.rhs(rng.uniform(0, 100, b["NH"]), rng.uniform(0, 1, b["NH"]), 0)
        _, it, _ = bl.pcg(s.Lam, Y, bl.block_prec(b, P1, PK), tol=1e-10)
        its.append(it)
    print("iterations for n = 12, 24, 48:", its)
    lg = np.log([13 * 13, 25 * 25, 49 * 49])
    assert max(its) <= (lg[-1] / lg[0]) ** 2 * min(its)
    assert its[-1] <= its[0] + 3
