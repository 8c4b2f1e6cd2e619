"""GPU: the multigrid inner preconditioner (a symmetric smoothed-aggregation
V-cycle for P_1 ~ S_1 and P_K ~ K_m; Sec. 5.3 leaves both inner solves
free and names multigrid among the classical choices).

The device V-cycle is compared element by element with the host cycle of
the same hierarchy (itself pinned to the oracle's cycle on the CPU), and
solves and step trajectories with it against the oracle's unique
normalised solution: the inner preconditioner changes the iteration
count, never X*."""
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


CASES = {
    "square48": lambda: w.square2d(n=48),
    "thorax3000": lambda: w.thorax2d(n_target=3000, seed=11),
    "slab16": lambda: w.slab3d(n=16),
    "slab32": lambda: w.slab3d(n=32),
    "thorax40k": lambda: w.thorax2d(n_target=40000, seed=12),
}


def _errs(U, V, Uo, Vo):
    return (np.linalg.norm(U - Uo) / max(np.linalg.norm(Uo), 1e-300),
            np.linalg.norm(V - Vo) / max(np.linalg.norm(Vo), 1e-300))


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("name", list(CASES))
def test_device_vcycle_matches_host_cycle(torch, name, precision):
    """One device V-cycle against the host cycle of the same hierarchy: to
    1e-12 in FP64; in mixed precision (FP32 level values and level vectors,
    FP64 input, output and accumulation) to 1e-5."""
    import paper_1711_08708_amd as B
    cfg = CASES[name]()
    hs = B.HostSetup(cfg, eps_h=0.0, inner_p1=B.P1_AMG, inner_pk=B.PK_AMG)
    solver = B.Solver(cfg, eps_h=0.0, inner_p1=B.P1_AMG, inner_pk=B.PK_AMG,
                      precision=B.PREC_MIXED if precision == "mixed" else B.PREC_FP64)
    tol = 1e-5 if precision == "mixed" else 1e-12
    for which in (0, 1):
        n = solver.N if which == 0 else solver.NH
        b = np.random.default_rng(3 + which).normal(size=n)
        ref = hs.amg_apply(which, b)
        xd = torch.full((n,), float("nan"), dtype=torch.float64, device="cuda")
        solver.inner_solve(which, torch.tensor(b, device="cuda"), xd)
        x = xd.cpu().numpy()
        err = np.abs(x - ref).max() / np.abs(ref).max()
        print(f"{name} {precision} block {which}: {hs.amg_info(which)} max rel diff {err:.2e}", flush=True)
        assert np.isfinite(x).all() and err < tol
        if which == 0:
            g = solver.info["ground_index"]
            assert x[g] == 0.0             # the grounded vertex, the one nearest the centroid


@pytest.mark.parametrize("name", ["slab16", "thorax3000"])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_compact_columns_give_the_same_cycle(torch, name, precision):
    """The level matrices of a banded order hold 16-bit column offsets from
    a per-row base (amg_columns = 0); the cycle reads fewer bytes and is
    bit-identical to the one on 32-bit columns (amg_columns = 1)."""
    import paper_1711_08708_amd as B
    cfg = CASES[name]()
    prec = B.PREC_MIXED if precision == "mixed" else B.PREC_FP64
    kw = dict(eps_h=0.0, inner_p1=B.P1_AMG, inner_pk=B.PK_AMG, precision=prec)
    s16 = B.Solver(cfg, amg_columns=0, **kw)
    s32 = B.Solver(cfg, amg_columns=1, **kw)
    i16, i32 = s16.info, s32.info
    print(name, precision, "V-cycle bytes 16-bit / 32-bit columns:", i16["bytes_p1"], i32["bytes_p1"],
          i16["bytes_pk"], i32["bytes_pk"], flush=True)
    assert i16["bytes_p1"] < i32["bytes_p1"]
    # a one-level hierarchy (the dense inverse alone) has no level products
    assert i16["bytes_pk"] < i32["bytes_pk"] if i16["levels_pk"] > 1 else i16["bytes_pk"] == i32["bytes_pk"]
    for which in (0, 1):
        n = s16.N if which == 0 else s16.NH
        b = torch.tensor(np.random.default_rng(11 + which).normal(size=n), device="cuda")
        x16 = torch.full((n,), float("nan"), dtype=torch.float64, device="cuda")
        x32 = torch.full((n,), float("nan"), dtype=torch.float64, device="cuda")
        s16.inner_solve(which, b, x16)
        s32.inner_solve(which, b, x32)
        assert torch.isfinite(x16).all()
        assert torch.equal(x16, x32)


def _solve_vs_oracle(torch, cfg, label, **params):
    import paper_1711_08708_amd as B
    from oracle import bidomain as bd
    s = bd.System(cfg)
    rng = np.random.default_rng(7)
    V = rng.uniform(0, 100, s.NH)
    h = rng.uniform(0, 1, s.NH)
    Y = s.rhs(V, h, 0)
    Xo = s.solve(Y)
    solver = B.Solver(cfg, **params)
    rhs = torch.tensor(np.concatenate([s.to_global_u(Y[:s.N]), Y[s.N:]]), device="cuda")
    x = torch.zeros_like(rhs)
    st = solver.solve(rhs, x, tol=1e-12)
    xh = x.cpu().numpy()
    eu, ev = _errs(xh[:s.N], xh[s.N:], s.to_global_u(Xo[:s.N]), Xo[s.N:])
    print(f"{label}: iters={st['iterations']} rel_res={st['rel_residual']:.2e} e_u={eu:.2e} e_v={ev:.2e}",
          flush=True)
    assert st["converged"] == 1
    assert eu <= TOL_PARITY and ev <= TOL_PARITY
    return st


@pytest.mark.parametrize("name", ["square48", "thorax3000", "slab16", "slab32"])
@pytest.mark.parametrize("pk", ["amg", "chebyshev", "cholesky"])
def test_solve_parity_with_multigrid_p1(torch, name, pk):
    import paper_1711_08708_amd as B
    kind = {"amg": B.PK_AMG, "chebyshev": B.PK_CHEBYSHEV, "cholesky": B.PK_CHOLESKY}[pk]
    _solve_vs_oracle(torch, CASES[name](), f"{name} P1 amg, PK {pk}", eps_h=0.0,
                     inner_p1=B.P1_AMG, inner_pk=kind)


def test_solve_parity_multigrid_mixed_precision(torch):
    """Mixed precision with multigrid inner solves (the cycles stay FP64;
    flexible CG in FP64 outside): same parity."""
    import paper_1711_08708_amd as B
    _solve_vs_oracle(torch, CASES["slab32"](), "slab32 amg/amg mixed", eps_h=0.0, precision=B.PREC_MIXED,
                     inner_p1=B.P1_AMG, inner_pk=B.PK_AMG)


@pytest.mark.parametrize("scheme", ["euler", "strang"])
def test_trajectory_with_multigrid(torch, scheme):
    """Eight steps with multigrid P_1 and Chebyshev P_K: every step matches
    the oracle's step from the same state (Strang: the elliptic potential
    of V* is refined to the tolerance with the inexact P_1)."""
    import paper_1711_08708_amd as B
    from oracle import bidomain as bd
    cfg = CASES["thorax3000"]()
    s = bd.System(cfg, scheme=scheme)
    sch = B.SCHEME_EULER if scheme == "euler" else B.SCHEME_STRANG
    solver = B.Solver(cfg, eps_h=0.0, tol=1e-11, scheme=sch, inner_p1=B.P1_AMG, inner_pk=B.PK_CHEBYSHEV)
    v, h, u = solver.state()
    worst = 0.0
    for n in range(8):
        Vn, hn = v.cpu().numpy().copy(), h.cpu().numpy().copy()
        Un = s.from_global_u(u.cpu().numpy())
        st = solver.step(v, h, u, n)
        assert st["converged"] == 1
        Uo, Vo, ho = s.step(Vn, hn, n, U0=Un)
        eu, ev = _errs(u.cpu().numpy(), v.cpu().numpy(), s.to_global_u(Uo), Vo)
        worst = max(worst, eu, ev)
        assert eu <= TOL_PARITY and ev <= TOL_PARITY, (n, eu, ev)
    print(scheme, "multigrid trajectory worst", worst, "iterations", st["iterations"])


def test_learned_stencil_with_multigrid_pk(torch):
    """The learned stencil with a multigrid P_K: K_m + C gets its own
    hierarchy (no factorisation) and flexible CG with it keeps parity."""
    import paper_1711_08708_amd as B
    from oracle import bidomain as bd
    cfg = w.slab3d(n=10)
    s = bd.System(cfg)
    solver = B.Solver(cfg, eps_h=0.0, tol=1e-11, inner_p1=B.P1_AMG, inner_pk=B.PK_AMG)
    v, h, u = solver.state()
    info = solver.learn_collect(v, h, u, 0, 6, max_samples=128)
    ts = solver.learn_train(kind=B.LEARN_STENCIL, epochs=20, batch=4, lr=2e-3, seed=1, n_val=2)
    print("collected", info, "trained", ts)
    assert ts["spd"] == 1
    solver.set_precond(B.PRECOND_LEARNED)
    for n in range(6, 9):
        Vn, hn = v.cpu().numpy().copy(), h.cpu().numpy().copy()
        st = solver.step(v, h, u, n)
        Uo, Vo, _ = s.step(Vn, hn, n)
        eu, ev = _errs(u.cpu().numpy(), v.cpu().numpy(), s.to_global_u(Uo), Vo)
        print(n, st["iterations"], eu, ev)
        assert eu <= TOL_PARITY and ev <= TOL_PARITY


def test_set_dt_with_multigrid_pk(torch):
    """A time-step change moves the hierarchy to the new K_m; steps after it
    match the oracle at the new step."""
    import paper_1711_08708_amd as B
    from oracle import bidomain as bd
    cfg = CASES["slab16"]()
    solver = B.Solver(cfg, eps_h=0.0, tol=1e-11, inner_p1=B.P1_AMG, inner_pk=B.PK_AMG)
    solver.set_dt(0.05)
    s = bd.System(cfg, dt=0.05)
    v, h, u = solver.state()
    for n in range(3):
        Vn, hn = v.cpu().numpy().copy(), h.cpu().numpy().copy()
        st = solver.step(v, h, u, n)
        Uo, Vo, _ = s.step(Vn, hn, n)
        eu, ev = _errs(u.cpu().numpy(), v.cpu().numpy(), s.to_global_u(Uo), Vo)
        assert eu <= TOL_PARITY and ev <= TOL_PARITY, (n, eu, ev)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_new_time_step_moves_the_hierarchy_on_the_device(torch, precision):
    """bido_set_dt with a multigrid P_K moves every level to the new gamma on
    the device (mass parts, D^-1, the smoother copy, the Lanczos bound, the
    coarsest inverse by Gauss-Jordan): one device V-cycle equals the host
    cycle of a set-up moved the same way (the host's refresh is pinned to the
    Galerkin products and the oracle cycle on the CPU), twice in a row; and
    it takes a fraction of a fresh set-up."""
    import paper_1711_08708_amd as B
    cfg = CASES["slab16"]()
    solver = B.Solver(cfg, eps_h=0.0, tol=1e-11, inner_p1=B.P1_AMG, inner_pk=B.PK_AMG,
                      precision=B.PREC_MIXED if precision == "mixed" else B.PREC_FP64)
    hs = B.HostSetup(cfg, eps_h=0.0, inner_p1=B.P1_AMG, inner_pk=B.PK_AMG)
    rng = np.random.default_rng(2)
    for dt in (cfg["dt"] / 3, cfg["dt"] * 2):
        sec = solver.set_dt(dt)
        hs.set_dt(dt)
        b = rng.normal(size=solver.NH)
        x = torch.zeros(solver.NH, dtype=torch.float64, device="cuda")
        solver.inner_solve(B.FACTOR_PK, torch.tensor(b, device="cuda"), x)
        xh = hs.amg_apply(B.FACTOR_PK, b)
        err = np.linalg.norm(x.cpu().numpy() - xh) / np.linalg.norm(xh)
        print(f"dt {dt}: set_dt {sec * 1e3:.1f} ms, device vs host cycle {err:.2e}", flush=True)
        assert err <= (1e-5 if precision == "mixed" else 1e-11)


def test_factor_only_calls_refuse_multigrid_blocks(torch):
    import paper_1711_08708_amd as B
    cfg = w.square2d(n=12)
    solver = B.Solver(cfg, eps_h=0.0, inner_p1=B.P1_AMG, inner_pk=B.PK_AMG)
    with pytest.raises(B.BidoError) as e:
        solver.set_plan(0, top_h=1)
    assert e.value.code == -7
    with pytest.raises(B.BidoError) as e:
        solver.set_pk(B.PK_CHOLESKY)
    assert e.value.code == -7
    with pytest.raises(B.BidoError) as e:
        B.Batch([solver], fused=True)
    assert e.value.code == -7
    b = torch.zeros(solver.N, dtype=torch.float64, device="cuda")
    with pytest.raises(B.BidoError) as e:
        solver.inner_solve_noalloc(0, b, b.clone())
    assert e.value.code == -7
