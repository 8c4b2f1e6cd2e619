"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

The bar is the relative error of Step 2's unique normalised solution
(Prop. 1): e_v = |V - V*| / |V*| <= 1e-8 and e_u = |U - U*| / |U*| <= 1e-8,
with the oracle solving the very right-hand side the GPU step used
(per-solve parity).  The oracle never sees GPU outputs except the state it
is asked to step from.
"""
import numpy as np
import pytest

import workloads as w

pytestmark = pytest.mark.gpu

TOL_PARITY = 1e-8


@pytest.fixture(scope="module")
def torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _errs(U, V, Uo, Vo):
    eu = np.linalg.norm(U - Uo) / max(np.linalg.norm(Uo), 1e-300)
    ev = np.linalg.norm(V - Vo) / max(np.linalg.norm(Vo), 1e-300)
    return eu, ev


def _oracle_solution_global(sysm, X):
    """Oracle X (heart-first order) -> (U in global order, V heart-local)."""
    return sysm.to_global_u(X[:sysm.N]), X[sysm.N:]


def _check_solve(torch, cfg, method="auto", **params):
    import paper_1711_08708_amd as B
    from oracle import bidomain as bd
    s = bd.System(cfg)
    rng = np.random.default_rng(7)
    V = rng.uniform(0, 100, s.NH)
    h = rng.uniform(0, 1, s.NH)
    Y = s.rhs(V, h, 0)
    Xo = s.solve(Y, method=method)
    Uo, Vo = _oracle_solution_global(s, Xo)
    solver = B.Solver(cfg, **params)
    assert np.array_equal(solver.heart_nodes, s.hn)
    rhs = np.concatenate([s.to_global_u(Y[:s.N]), Y[s.N:]])
    rhs_d = torch.tensor(rhs, dtype=torch.float64, device="cuda")
    x_d = torch.zeros_like(rhs_d)
    st = solver.solve(rhs_d, x_d, tol=params.get("tol", 1e-12))
    x = x_d.cpu().numpy()
    eu, ev = _errs(x[:s.N], x[s.N:], Uo, Vo)
    print(f"{cfg['name']}: iters={st['iterations']} rel_res={st['rel_residual']:.2e} "
          f"e_u={eu:.2e} e_v={ev:.2e}", flush=True)
    assert st["converged"] == 1
    assert eu <= TOL_PARITY and ev <= TOL_PARITY
    return st, solver


@pytest.mark.parametrize("mk", [
    lambda: w.square2d(n=5),            # 36 vertices: several single-node levels
    lambda: w.square2d(n=48),           # the 2,401-vertex square (ragged leaves)
    lambda: w.thorax2d(n_target=3000, seed=11),
    lambda: w.slab3d(n=6),
    lambda: w.slab3d(n=14),             # 3,375 vertices: oracle by Jacobi-CG
], ids=["square5", "square48", "thorax3000", "slab6", "slab14"])
def test_solve_parity_exact_factor(torch, mk):
    _check_solve(torch, mk(), eps_h=0.0, tol=1e-12)


@pytest.mark.parametrize("eps", [1e-8, 1e-4])
def test_solve_parity_hierarchical_top(torch, eps):
    """Inexact inner solves (hierarchical top at eps_h) change the iteration
    count, never the solution: parity at 1e-8 holds."""
    st, _ = _check_solve(torch, w.thorax2d(n_target=6000, seed=13), eps_h=eps, tol=1e-12)
    print("iterations at eps", eps, st["iterations"])


def test_exact_factor_iteration_count_matches_dense_block_lu(torch):
    """With exact inner factors the GPU preconditioner is the block-LU of
    Def. 2 with P_1 = grounded S_1 and P_K = K_m exactly, so its iteration
    count equals that of the dense oracle PCG with the same blocks."""
    from oracle import bidomain as bd, blocklu as bl
    import paper_1711_08708_amd as B
    cfg = w.square2d(n=24)
    s = bd.System(cfg)
    b = bl.dense_blocks(s)
    rng = np.random.default_rng(3)
    Y = s.rhs(rng.uniform(0, 100, s.NH), rng.uniform(0, 1, s.NH), 0)
    Pinv = bl.block_prec(b, bl.grounded_solver(b["S1"]), bl.chol_solver(bl.K_monodomain(b)))
    _, it_ref, _ = bl.pcg(s.Lam, Y, Pinv, tol=1e-10)
    solver = B.Solver(cfg, eps_h=0.0)
    rhs = torch.tensor(np.concatenate([s.to_global_u(Y[:s.N]), Y[s.N:]]), device="cuda")
    x = torch.zeros_like(rhs)
    st = solver.solve(rhs, x, tol=1e-10)
    print("iterations gpu", st["iterations"], "oracle", it_ref)
    assert st["iterations"] == it_ref


def test_step_trajectory_square48(torch):
    """20 steps of the 2,401-vertex square: every step's solve matches the
    oracle's solve of the same right-hand side, and the gating update is
    bit-for-bit the oracle's formula up to rounding."""
    import paper_1711_08708_amd as B
    from oracle import bidomain as bd
    cfg = w.make_config("square48")
    s = bd.System(cfg)
    solver = B.Solver(cfg, eps_h=0.0, tol=1e-12)
    v, h, u = solver.state()
    worst = 0.0
    for n in range(cfg["n_steps"]):
        Vn = v.cpu().numpy().copy()
        hn = h.cpu().numpy().copy()
        st = solver.step(v, h, u, n)
        Uo_p, Vo, ho = s.step(Vn, hn, n, method="dense")
        Uo = s.to_global_u(Uo_p)
        eu, ev = _errs(u.cpu().numpy(), v.cpu().numpy(), Uo, Vo)
        eh = np.abs(h.cpu().numpy() - ho).max()
        worst = max(worst, eu, ev)
        assert eu <= TOL_PARITY and ev <= TOL_PARITY, (n, eu, ev)
        assert eh <= 1e-14
    print("square48 worst per-step error", worst)


@pytest.mark.parametrize("name", ["square48", "thorax3000"])
def test_projected_initial_guess(torch, name):
    """The default initial guess, the Lambda-orthogonal projection of the
    solution onto the span of the states of the last 8 steps, with
    multigrid inner solves: steps match the oracle's step from the same
    state, a run takes fewer PCG iterations than with X0 = X^n
    (guess_states = 0) and ends in the same state; a change of dt restarts
    the span and the next steps still match the oracle."""
    import paper_1711_08708_amd as B
    from oracle import bidomain as bd
    cfg = w.make_config("square48") if name == "square48" else w.thorax2d(n_target=3000, seed=11)
    s = bd.System(cfg)
    n_steps = 16
    tot, final = {}, {}
    for k in (0, 8):
        solver = B.Solver(cfg, eps_h=0.0, tol=1e-12, inner_p1=B.P1_AMG, inner_pk=B.PK_AMG, guess_states=k)
        v, h, u = solver.state()
        tot[k] = 0
        for n in range(n_steps):
            Vn, hn = v.cpu().numpy().copy(), h.cpu().numpy().copy()
            tot[k] += solver.step(v, h, u, n)["iterations"]
            if k and n % 4 == 3:
                Uo_p, Vo, _ = s.step(Vn, hn, n, method="dense")
                eu, ev = _errs(u.cpu().numpy(), v.cpu().numpy(), s.to_global_u(Uo_p), Vo)
                assert eu <= TOL_PARITY and ev <= TOL_PARITY, (n, eu, ev)
        final[k] = (u.cpu().numpy(), v.cpu().numpy())
        if k:
            solver.set_dt(cfg["dt"] / 2)
            s2 = bd.System(cfg, dt=cfg["dt"] / 2)
            for n in range(n_steps, n_steps + 3):
                Vn, hn = v.cpu().numpy().copy(), h.cpu().numpy().copy()
                solver.step(v, h, u, n)
                Uo_p, Vo, _ = s2.step(Vn, hn, n, method="dense")
                eu, ev = _errs(u.cpu().numpy(), v.cpu().numpy(), s2.to_global_u(Uo_p), Vo)
                assert eu <= TOL_PARITY and ev <= TOL_PARITY, ("after set_dt", n, eu, ev)
    print(f"{name}: PCG iterations over {n_steps} steps, X0 = X^n {tot[0]}, projected {tot[8]}", flush=True)
    assert tot[8] < tot[0]
    eu, ev = _errs(final[8][0], final[8][1], final[0][0], final[0][1])
    assert eu <= TOL_PARITY and ev <= TOL_PARITY


def test_reset_guess_matches_a_fresh_context(torch):
    """After bido_reset_guess the next steps start a new span of states:
    from the same state they are bit-identical to those of a fresh context
    (stale states in the ring are never read); a context that keeps its
    states starts from another guess and reaches other iterates."""
    import paper_1711_08708_amd as B
    cfg = w.slab3d(n=10)
    kw = dict(eps_h=0.0, tol=1e-12, inner_p1=B.P1_AMG, inner_pk=B.PK_AMG)
    runs = {}
    for name in ("reset", "kept", "fresh"):
        sv = B.Solver(cfg, **kw)
        v, h, u = sv.state()
        if name != "fresh":
            for n in range(6):
                sv.step(v, h, u, n)
            st0 = [t.clone() for t in (v, h, u)]
            if name == "reset":
                sv.reset_guess()
        st = [t.clone() for t in st0]
        its = [sv.step(st[0], st[1], st[2], n)["iterations"] for n in range(6, 10)]
        runs[name] = (its, [t.cpu().numpy() for t in st])
        sv.close()
    print("iterations after reset / kept / fresh", runs["reset"][0], runs["kept"][0], runs["fresh"][0], flush=True)
    assert runs["reset"][0] == runs["fresh"][0]
    assert all(np.array_equal(x, y) for x, y in zip(runs["reset"][1], runs["fresh"][1]))
    assert not all(np.array_equal(x, y) for x, y in zip(runs["kept"][1], runs["fresh"][1]))


@pytest.mark.parametrize("mk,eps,n_steps", [(lambda: w.make_config("square48"), 0.0, 20),
                                             (lambda: w.thorax2d(n_target=3000, seed=11), 1e-8, 12)],
                         ids=["square48", "thorax3000"])
def test_crank_nicolson_trajectory(torch, mk, eps, n_steps):
    """Crank-Nicolson steps (Lambda and K_m with 2 gamma; Step 1 reads U^n
    through the v rows of Lambda): every step's U^{n+1}, V^{n+1} match the
    oracle's Crank-Nicolson step from the same U^n, V^n, h^n."""
    import paper_1711_08708_amd as B
    from oracle import bidomain as bd
    cfg = mk()
    s = bd.System(cfg, scheme="cn")
    solver = B.Solver(cfg, eps_h=eps, tol=1e-12, scheme=B.SCHEME_CN)
    v, h, u = solver.state()
    worst = 0.0
    for n in range(n_steps):
        Vn = v.cpu().numpy().copy()
        hn = h.cpu().numpy().copy()
        Un = s.from_global_u(u.cpu().numpy())
        st = solver.step(v, h, u, n)
        assert st["converged"] == 1
        Uo_p, Vo, ho = s.step(Vn, hn, n, U0=Un)
        eu, ev = _errs(u.cpu().numpy(), v.cpu().numpy(), s.to_global_u(Uo_p), Vo)
        worst = max(worst, eu, ev)
        assert eu <= TOL_PARITY and ev <= TOL_PARITY, (n, eu, ev)
        assert np.abs(h.cpu().numpy() - ho).max() <= 1e-14
    print(cfg["name"], "Crank-Nicolson worst per-step error", worst, "iterations", st["iterations"])


def test_thorax200k_solve_parity(torch):
    """Full-size thorax slice (about 200k vertices): the normalised solution
    of one step's system matches the oracle's sparse direct solve."""
    _check_solve(torch, w.make_config("thorax200k"), eps_h=0.0, tol=1e-12)


def _check_solve_cg(torch, cfg, solver, label):
    """One solve of a random state's system against the oracle's Jacobi-CG
    (augmented SPD matrix, condition-aware stop): per-solve parity."""
    from oracle import bidomain as bd
    s = bd.System(cfg)
    rng = np.random.default_rng(5)
    V = rng.uniform(0, 100, s.NH)
    h = rng.uniform(0, 1, s.NH)
    Y = s.rhs(V, h, 0)
    rhs = torch.tensor(np.concatenate([s.to_global_u(Y[:s.N]), Y[s.N:]]), device="cuda")
    x = torch.zeros_like(rhs)
    st = solver.solve(rhs, x, tol=1e-12)
    Xo = s.solve_cg(Y)
    Uo, Vo = _oracle_solution_global(s, Xo)
    xh = x.cpu().numpy()
    eu, ev = _errs(xh[:s.N], xh[s.N:], Uo, Vo)
    print(f"{label}: iters={st['iterations']} rel_res={st['rel_residual']:.2e} oracle CG {s.last_cg} "
          f"e_u={eu:.2e} e_v={ev:.2e}", flush=True)
    assert st["converged"] == 1
    assert eu <= TOL_PARITY and ev <= TOL_PARITY


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("wide,rows", [(1, 128), (0, 64)], ids=["wide128", "narrow64"])
def test_split_backward_items_parity(torch, precision, wide, rows):
    """Backward level items forced onto row ranges (the split tiles of tall
    3D separators, summed by the combine launch) on every level up to the
    root (no top), on a slab small enough for the oracle: the plan really
    splits tiles, and the solve matches the oracle."""
    import paper_1711_08708_amd as B
    cfg = w.slab3d(n=20)
    hs = B.HostSetup(cfg, eps_h=0.0)
    solver = B.Solver(cfg, eps_h=0.0, precision=precision)
    for which in (0, 1):
        H = hs.factor_stats(which)["height"]
        hs.set_plan(which, bwd_wide=wide, bwd_rows=rows, top_h=H + 1)
        plan = hs.factor_plan(which)
        print(f"slab20 factor {which} plan {plan}", flush=True)
        assert plan["n_bwd_split"] > 0
        solver.set_plan(which, bwd_wide=wide, bwd_rows=rows, top_h=H + 1)
    _check_solve_cg(torch, cfg, solver, f"slab20 split {wide}/{rows} precision {precision}")


def test_slab40_default_plan_splits_and_matches_oracle(torch):
    """A 41^3-vertex slab: its default plan cuts the tall backward tiles of
    its separators into row ranges (asserted), and the mixed-precision
    solve matches the oracle."""
    import paper_1711_08708_amd as B
    cfg = w.slab3d(n=40)
    hs = B.HostSetup(cfg, eps_h=0.0)
    plan = hs.factor_plan(0)
    print("slab40 P1 plan", plan, flush=True)
    assert plan["n_bwd_split"] > 0
    solver = B.Solver(cfg, eps_h=0.0, precision=B.PREC_MIXED)
    _check_solve_cg(torch, cfg, solver, "slab40 mixed")


@pytest.mark.timeout(900)
def test_slab64_full_size_parity(torch):
    """Full-size 3D slab (274,625 vertices, mixed precision as in its
    configuration): the default plan splits tall backward tiles (asserted)
    and one solve matches the oracle's Jacobi-CG to 1e-8 in U and V."""
    import paper_1711_08708_amd as B
    cfg = w.make_config("slab64")
    hs = B.HostSetup(cfg, eps_h=0.0)
    plan = hs.factor_plan(0)
    print("slab64 P1 plan", plan, flush=True)
    assert plan["n_bwd_split"] > 0
    del hs
    solver = B.Solver(cfg, eps_h=0.0, precision=B.PREC_MIXED)
    _check_solve_cg(torch, cfg, solver, "slab64 mixed")


def test_lambda_blocked_form(torch):
    """A slab (heart = whole mesh, one internal order for u and v) runs the
    Lambda product on the blocked form (20 bytes per position instead of 12
    per entry of the four CSR blocks) and a solve still matches the oracle to
    1e-8; a thorax slice (torso rows) keeps the CSR product.  With multigrid
    blocks (a banded order) the positions hold 16-bit column offsets (18
    bytes per position) and the solve matches the oracle too."""
    import paper_1711_08708_amd as B
    cfg = w.slab3d(n=12)
    solver = B.Solver(cfg, eps_h=0.0)
    info = solver.info
    print("slab12 Lambda bytes", info["bytes_lambda"], "nnz", info["nnz_lambda"], flush=True)
    assert info["bytes_lambda"] < 12 * info["nnz_lambda"]
    _check_solve_cg(torch, cfg, solver, "slab12 blocked Lambda")
    th = B.Solver(w.thorax2d(n_target=3000, seed=7), eps_h=0.0)
    assert th.info["bytes_lambda"] > 12 * th.info["nnz_lambda"]
    kw = dict(eps_h=0.0, inner_p1=B.P1_AMG, inner_pk=B.PK_AMG)
    s16 = B.Solver(cfg, amg_columns=0, **kw)
    s32 = B.Solver(cfg, amg_columns=1, **kw)
    assert s16.info["nnz_lambda"] % 4 == 0
    npos = s16.info["nnz_lambda"] // 4                     # Lambda = four blocks of one pattern
    print("slab12 multigrid Lambda bytes, 16-bit / 32-bit columns", s16.info["bytes_lambda"],
          s32.info["bytes_lambda"], flush=True)
    assert s32.info["bytes_lambda"] - s16.info["bytes_lambda"] == 2 * npos - 4 * s16.N
    _check_solve_cg(torch, cfg, s16, "slab12 blocked Lambda, 16-bit columns")


def test_range_and_dt_errors(torch):
    import paper_1711_08708_amd as B
    cfg = w.square2d(n=8)
    solver = B.Solver(cfg, eps_h=0.0)
    n2 = solver.N + solver.NH
    rhs = torch.zeros(n2, dtype=torch.float64, device="cuda")
    rhs[: solver.N] = 1.0      # not in Ran(Lambda)
    x = torch.zeros_like(rhs)
    with pytest.raises(B.BidoError) as e:
        solver.solve(rhs, x)
    assert e.value.code == -6
    v, h, u = solver.state()
    with pytest.raises(B.BidoError) as e:
        B._check(B.lib.bido_step(solver.ctx, solver._dev(v, solver.NH), solver._dev(h, solver.NH),
                                 solver._dev(u, solver.N), 0.05, 0, None))
    assert e.value.code == -5


def test_zero_rhs_and_not_converged(torch):
    import paper_1711_08708_amd as B
    cfg = w.square2d(n=12)
    solver = B.Solver(cfg, eps_h=0.0)
    n2 = solver.N + solver.NH
    rhs = torch.zeros(n2, dtype=torch.float64, device="cuda")
    x = torch.ones_like(rhs)
    st = solver.solve(rhs, x)
    assert st["iterations"] == 0 and float(x.abs().max()) == 0.0
    rhs[solver.N:] = 1.0
    x.zero_()
    solver.set_solver(tol=1e-14, max_iter=1)
    with pytest.raises(B.BidoError) as e:
        solver.solve(rhs, x)
    assert e.value.code == -4


@pytest.mark.parametrize("mk,n_steps", [(lambda: w.make_config("square48"), 20),
                                        (lambda: w.thorax2d(n_target=3000, seed=11), 12)],
                         ids=["square48", "thorax3000"])
@pytest.mark.parametrize("eps_h", [0.0, 1e-4])
def test_strang_splitting_trajectory(torch, mk, n_steps, eps_h):
    """Strang splitting (Heun reaction half-steps around the Crank-Nicolson
    diffusion step started from the elliptic potential of V*): every step's
    U^{n+1}, V^{n+1}, w^{n+1} match the oracle's splitting step from the
    same state.  With eps_h > 0 the P_1 apply alone misses the elliptic
    potential by O(eps_h); the library refines it to the solver tolerance,
    so the bar is the same."""
    import paper_1711_08708_amd as B
    from oracle import bidomain as bd
    cfg = mk()
    s = bd.System(cfg, scheme="strang")
    solver = B.Solver(cfg, eps_h=eps_h, tol=1e-12, scheme=B.SCHEME_STRANG)
    v, h, u = solver.state()
    worst = 0.0
    for n in range(n_steps):
        Vn = v.cpu().numpy().copy()
        hn = h.cpu().numpy().copy()
        Un = s.from_global_u(u.cpu().numpy())
        st = solver.step(v, h, u, n)
        assert st["converged"] == 1
        Uo_p, Vo, ho = s.step(Vn, hn, n, U0=Un)
        eu, ev = _errs(u.cpu().numpy(), v.cpu().numpy(), s.to_global_u(Uo_p), Vo)
        worst = max(worst, eu, ev)
        assert eu <= TOL_PARITY and ev <= TOL_PARITY, (n, eu, ev)
        assert np.abs(h.cpu().numpy() - ho).max() <= 1e-12
    print(cfg["name"], "Strang worst per-step error", worst, "iterations", st["iterations"])
