"""GPU: the polynomial P_K (Chebyshev acceleration of the Jacobi iteration on
K_m, an alternative inner solve inside the block-LU preconditioner; Sec. 5.3
leaves P_K free).

The device apply (three-term recurrence, one fused product-and-update launch
per step) is compared element by element with the oracle's closed-form
polynomial on the same interval; solves and step trajectories with it are
compared with the oracle's unique normalised solution."""
import numpy as np
import pytest
import scipy.sparse as sp

import workloads as w

pytestmark = pytest.mark.gpu

TOL_PARITY = 1e-8


@pytest.fixture(scope="module")
def torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _oracle_km(cfg):
    from oracle import bidomain as bd
    s = bd.System(cfg)
    return s, (s.gamma_eff * sp.diags(s.mH) + s.Sm).tocsr()


def _extremes(K):
    """Extreme eigenvalues of D^-1/2 K D^-1/2 (oracle side, dense or Lanczos)."""
    import scipy.sparse.linalg as spl
    d = K.diagonal()
    Ds = sp.diags(1.0 / np.sqrt(d))
    B = (Ds @ K @ Ds).tocsc()
    if B.shape[0] <= 3000:
        ev = np.linalg.eigvalsh(B.toarray())
        return ev[0], ev[-1]
    hi = spl.eigsh(B, k=1, which="LA", return_eigenvectors=False, tol=1e-10)[0]
    lo = spl.eigsh(B, k=1, sigma=0.0, which="LM", return_eigenvectors=False, tol=1e-10)[0]
    return lo, hi


CASES = {
    "square48": lambda: w.square2d(n=48),
    "thorax3000": lambda: w.thorax2d(n_target=3000, seed=11),
    "slab8": lambda: w.slab3d(n=8),
    "thorax40k": lambda: w.thorax2d(n_target=40000, seed=12),
}


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("m", [1, 2, 3, 5])
def test_chebyshev_apply_matches_oracle_polynomial(torch, name, m):
    import paper_1711_08708_amd as B
    from oracle import chebyshev as ch
    cfg = CASES[name]()
    s, K = _oracle_km(cfg)
    lo, hi = _extremes(K)
    hi *= 1.05
    solver = B.Solver(cfg, eps_h=0.0)
    vpos = B.HostSetup(cfg).index(B.IDX_VPOS)
    rng = np.random.default_rng(m)
    t = rng.normal(size=s.NH)                       # heart-local order
    ref = ch.chebyshev_jacobi(K, t, lo, hi, m)
    solver.set_pk(B.PK_CHEBYSHEV, m, lo, hi)
    assert solver.pk() == dict(kind=B.PK_CHEBYSHEV, steps=m, lo=lo, hi=hi)
    t_int = np.empty(s.NH)
    t_int[vpos] = t
    bd_ = torch.tensor(t_int, device="cuda")
    xd = torch.full((s.NH,), float("nan"), dtype=torch.float64, device="cuda")
    print(f"{name} m={m}: N_H={s.NH} interval [{lo:.4f}, {hi:.4f}]", flush=True)
    solver.inner_solve(B.FACTOR_PK, bd_, xd)
    x = xd.cpu().numpy()[vpos]
    err = np.abs(x - ref).max() / np.abs(ref).max()
    print(f"  max rel diff {err:.2e}", flush=True)
    assert np.isfinite(x).all()
    assert err < 1e-12


def _solve_case(torch, cfg, steps, precision=0):
    import paper_1711_08708_amd as B
    from oracle import bidomain as bd
    s = bd.System(cfg)
    rng = np.random.default_rng(7)
    V = rng.uniform(0, 100, s.NH)
    h = rng.uniform(0, 1, s.NH)
    Y = s.rhs(V, h, 0)
    Xo = s.solve(Y)
    Uo, Vo = s.to_global_u(Xo[:s.N]), Xo[s.N:]       # the normalised solution (Prop. 1)
    rhs = np.concatenate([s.to_global_u(Y[:s.N]), Y[s.N:]])
    out = {}
    for kind in (B.PK_CHOLESKY, B.PK_CHEBYSHEV):
        solver = B.Solver(cfg, eps_h=0.0, tol=1e-12, precision=precision)
        if kind == B.PK_CHEBYSHEV:
            solver.set_pk(kind, steps)
        rhs_d = torch.tensor(rhs, dtype=torch.float64, device="cuda")
        x_d = torch.zeros_like(rhs_d)
        st = solver.solve(rhs_d, x_d, tol=1e-12)
        x = x_d.cpu().numpy()
        eu = np.linalg.norm(x[:s.N] - Uo) / np.linalg.norm(Uo)
        ev = np.linalg.norm(x[s.N:] - Vo) / np.linalg.norm(Vo)
        print(f"{cfg['name']} pk={kind} steps={steps}: iters={st['iterations']} e_u={eu:.2e} e_v={ev:.2e}",
              flush=True)
        assert st["converged"] == 1
        assert eu <= TOL_PARITY and ev <= TOL_PARITY
        out[kind] = st["iterations"]
    return out


@pytest.mark.parametrize("mk", [lambda: w.square2d(n=48), lambda: w.thorax2d(n_target=3000, seed=11),
                                lambda: w.slab3d(n=6), lambda: w.thorax2d(n_target=20000, seed=3)],
                         ids=["square48", "thorax3000", "slab6", "thorax20k"])
def test_solve_parity_with_chebyshev_pk(torch, mk):
    """The normalised solution is unique: with the polynomial P_K (library
    interval, 3 steps) the solve matches the oracle at 1e-8; in 2D the
    iteration count stays within two of the factored P_K."""
    import paper_1711_08708_amd as B
    cfg = mk()
    its = _solve_case(torch, cfg, 3)
    if cfg["dim"] == 2:
        assert its[B.PK_CHEBYSHEV] <= its[B.PK_CHOLESKY] + 2, its


def test_solve_parity_chebyshev_pk_mixed(torch):
    import paper_1711_08708_amd as B
    _solve_case(torch, w.thorax2d(n_target=3000, seed=11), 3, precision=B.PREC_MIXED)


def test_trajectory_with_chebyshev_pk(torch):
    """Ten steps of a thorax slice with the polynomial P_K: each step's
    state matches the oracle's step from the same state."""
    import paper_1711_08708_amd as B
    from oracle import bidomain as bd
    cfg = w.thorax2d(n_target=3000, seed=11)
    s = bd.System(cfg)
    solver = B.Solver(cfg, eps_h=0.0, tol=1e-12)
    solver.set_pk(B.PK_CHEBYSHEV, 3)
    v, h, u = solver.state()
    worst = 0.0
    for n in range(10):
        Vn = v.cpu().numpy().copy()
        hn = h.cpu().numpy().copy()
        st = solver.step(v, h, u, n)
        assert st["converged"] == 1
        Uo_p, Vo, ho = s.step(Vn, hn, n)
        Uo = s.to_global_u(Uo_p)
        U = u.cpu().numpy()
        eu = np.linalg.norm(U - Uo) / max(np.linalg.norm(Uo), 1e-300)
        ev = np.linalg.norm(v.cpu().numpy() - Vo) / np.linalg.norm(Vo)
        worst = max(worst, eu, ev)
        assert eu <= TOL_PARITY and ev <= TOL_PARITY, (n, eu, ev)
    print("thorax3000 Chebyshev P_K worst per-step error", worst, "iterations", st["iterations"])


def test_chebyshev_graph_replay_matches_eager(torch):
    """Captured iteration graphs (with the Chebyshev launches inside) give
    bit-identical states to eager launches, over several steps."""
    import paper_1711_08708_amd as B
    cfg = w.thorax2d(n_target=3000, seed=11)
    states = []
    for graphs in (0, 1):
        solver = B.Solver(cfg, eps_h=1e-8, tol=1e-10)
        solver.set_pk(B.PK_CHEBYSHEV, 3)
        solver.set_graphs(graphs)
        v, h, u = solver.state()
        for n in range(5):
            solver.step(v, h, u, n)
            torch.cuda.synchronize()
        states.append((v.cpu().numpy(), u.cpu().numpy()))
    assert np.array_equal(states[0][0], states[1][0]) and np.array_equal(states[0][1], states[1][1])


def test_set_pk_arguments_and_switching(torch):
    import paper_1711_08708_amd as B
    cfg = w.thorax2d(n_target=3000, seed=11)
    solver = B.Solver(cfg, eps_h=0.0)
    for args in [(7, 3, 0.0, 0.0), (B.PK_CHEBYSHEV, 0, 0.0, 0.0),
                 (B.PK_CHEBYSHEV, B.PK_MAX_STEPS + 1, 0.0, 0.0), (B.PK_CHEBYSHEV, 3, 1.0, 0.5),
                 (B.PK_CHEBYSHEV, 3, -1.0, 1.0), (B.PK_CHEBYSHEV, 3, 0.5, 0.0)]:
        with pytest.raises(RuntimeError, match="BIDO_ERR_ARG"):
            solver.set_pk(*args)
    assert solver.pk()["kind"] == B.PK_CHOLESKY
    solver.set_pk(B.PK_CHEBYSHEV, 4)
    got = solver.pk()
    iv = B.HostSetup(cfg).pk_interval()
    assert got["steps"] == 4 and got["lo"] == iv["lo"] and got["hi"] == iv["hi"]
    # a fused batch needs one P_K choice for all its slices
    other = B.Solver(w.thorax2d(n_target=2000, seed=5), eps_h=0.0)
    with pytest.raises(RuntimeError, match="BIDO_ERR_STATE"):
        B.Batch([solver, other], fused=True)
    # back to the factor: the same iterations as a fresh context
    solver.set_pk(B.PK_CHOLESKY)
    assert solver.pk() == dict(kind=B.PK_CHOLESKY, steps=0, lo=0.0, hi=0.0)
    fresh = B.Solver(cfg, eps_h=0.0)
    res = []
    for sv in (solver, fresh):
        v, h, u = sv.state()
        res.append(sv.step(v, h, u, 0)["iterations"])
    assert res[0] == res[1]


def test_thorax200k_solve_parity_with_chebyshev_pk(torch):
    """Full-size thorax slice (200,656 vertices, 25,768 heart vertices) with
    the polynomial P_K at its default three steps: the normalised solution
    of one step's system matches the oracle's sparse direct solve."""
    import paper_1711_08708_amd as B
    from oracle import bidomain as bd
    cfg = w.make_config("thorax200k")
    s = bd.System(cfg)
    rng = np.random.default_rng(7)
    Y = s.rhs(rng.uniform(0, 100, s.NH), rng.uniform(0, 1, s.NH), 0)
    Xo = s.solve(Y)
    Uo, Vo = s.to_global_u(Xo[:s.N]), Xo[s.N:]
    sv = B.Solver(cfg, tol=1e-12)
    sv.set_pk(B.PK_CHEBYSHEV, 3)
    rhs = torch.tensor(np.concatenate([s.to_global_u(Y[:s.N]), Y[s.N:]]), dtype=torch.float64, device="cuda")
    x = torch.zeros_like(rhs)
    st = sv.solve(rhs, x, tol=1e-12)
    x = x.cpu().numpy()
    eu = np.linalg.norm(x[:s.N] - Uo) / np.linalg.norm(Uo)
    ev = np.linalg.norm(x[s.N:] - Vo) / np.linalg.norm(Vo)
    print(f"thorax200k Chebyshev P_K: iterations {st['iterations']} e_u {eu:.2e} e_v {ev:.2e}", flush=True)
    assert st["converged"] == 1
    assert eu <= TOL_PARITY and ev <= TOL_PARITY


def test_streams_batch_with_chebyshev_pk(torch):
    """A batch on streams runs each slice's own steps, Chebyshev P_K included:
    bit-identical to the slices run alone."""
    import paper_1711_08708_amd as B
    cfgs = [w.thorax2d(n_target=3000, seed=11), w.thorax2d(n_target=2000, seed=5), w.square2d(n=24, seed=3)]
    alone = []
    for cfg in cfgs:
        sv = B.Solver(cfg, tol=1e-12)
        sv.set_pk(B.PK_CHEBYSHEV, 3)
        v, h, u = sv.state()
        for n in range(6):
            sv.step(v, h, u, n)
        alone.append([t.cpu().numpy() for t in (v, h, u)])
        sv.close()
    solvers = [B.Solver(cfg, tol=1e-12) for cfg in cfgs]
    for sv in solvers:
        sv.set_pk(B.PK_CHEBYSHEV, 3)
    batch = B.Batch(solvers, n_streams=2)
    states = [sv.state() for sv in solvers]
    tot, _ = batch.run(states, 0, 6)
    assert tot["converged"] == 1
    batch.close()
    for st, ref in zip(states, alone):
        for a, b in zip([t.cpu().numpy() for t in st], ref):
            assert np.array_equal(a, b)
    for sv in solvers:
        sv.close()
