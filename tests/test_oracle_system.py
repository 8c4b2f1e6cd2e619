"""Pins for the oracle's system matrix, normalised solve and time step
(Sec. 3.2, Prop. 1) and for the Mitchell-Schaeffer reaction terms."""
import numpy as np
import pytest

import workloads as w
from oracle import bidomain as bd
from oracle import ionic


@pytest.fixture(scope="module")
def small():
    return bd.System(w.square2d(n=12))


def test_lambda_symmetric_psd_kernel(small):
    """Prop. 1: symmetric PSD, kernel 1_Omega x {0}."""
    L = small.Lam.toarray()
    assert np.abs(L - L.T).max() <= 1e-14 * np.abs(L).max()
    ev, vec = np.linalg.eigh(L)
    scale = np.abs(ev).max()
    assert ev.min() >= -1e-12 * scale
    assert (np.abs(ev) <= 1e-11 * scale).sum() == 1
    k = vec[:, np.argmin(np.abs(ev))]
    ref = np.concatenate([np.ones(small.N), np.zeros(small.NH)])
    ref /= np.linalg.norm(ref)
    assert abs(abs(k @ ref) - 1.0) < 1e-10


def test_range_and_restriction(small):
    """Ran Lambda = 1^perp x R^NH; Pi Pi^T = id; Pi^T S_i Pi = S_1 - S_e."""
    rng = np.random.default_rng(1)
    X = rng.normal(size=small.N + small.NH)
    assert abs((small.Lam @ X)[:small.N].sum()) < 1e-11 * np.abs(small.Lam @ X).max()
    PiT = small.PiT.toarray()
    np.testing.assert_allclose(PiT.T @ PiT, np.eye(small.NH))
    lhs = PiT @ small.Si.toarray() @ PiT.T
    np.testing.assert_allclose(lhs, (small.S1 - small.Se).toarray(), atol=1e-13)


@pytest.mark.parametrize("mk", [lambda: w.square2d(n=12),
                                lambda: w.slab3d(n=4),
                                lambda: w.thorax2d(n_target=1500, seed=2)])
def test_three_solvers_agree(mk):
    """Dense augmented Cholesky, grounded sparse LU and Jacobi-CG reach the
    same normalised solution; it satisfies Lambda X = Y and (M U, 1) = 0."""
    s = bd.System(mk())
    rng = np.random.default_rng(2)
    V = rng.uniform(0, 100, s.NH)
    h = rng.uniform(0, 1, s.NH)
    Y = s.rhs(V, h, 0)
    Xd = s.solve_dense(Y)
    Xs = s.solve_sparse(Y)
    Xc = s.solve_cg(Y)
    assert np.linalg.norm(s.Lam @ Xd - Y) <= 1e-12 * np.linalg.norm(Y)
    assert abs(s.m @ Xd[:s.N]) <= 1e-12 * np.abs(Xd).max()
    assert bd.rel_err(Xs, Xd) < 1e-11
    assert bd.rel_err(Xc, Xd) < 1e-9


@pytest.mark.parametrize("n", [12, 16])
def test_cg_meets_sparse_lu_in_3d(n):
    """At 3D sizes where the stopping test's condition estimate matters
    (12^3 and 16^3 cubes, Jacobi condition numbers in the hundreds to
    thousands), the Jacobi-CG solution agrees with the grounded sparse LU
    solution to 1e-11, from rest and from a warm start, and its estimate
    settles (the augmented matrix has no kernel)."""
    s = bd.System(w.slab3d(n=n))
    rng = np.random.default_rng(4)
    V = rng.uniform(0, 100, s.NH)
    h = rng.uniform(0, 1, s.NH)
    Y = s.rhs(V, h, 0)
    Xs = s.solve_sparse(Y)
    Xc = s.solve_cg(Y)
    kappa = s.last_cg["kappa"]
    assert 10.0 < kappa < 1e6, s.last_cg
    assert bd.rel_err(Xc[:s.N], Xs[:s.N]) < 1e-11 and bd.rel_err(Xc[s.N:], Xs[s.N:]) < 1e-11
    x0 = Xs + rng.normal(0, 1.0, Xs.shape)
    Xw = s.solve_cg(Y, x0=x0)
    assert bd.rel_err(Xw[:s.N], Xs[:s.N]) < 1e-11 and bd.rel_err(Xw[s.N:], Xs[s.N:]) < 1e-11


def test_constant_potential_is_stationary(small):
    """With Y = [0; gamma M_H c 1] the normalised solution is U = 0, V = c 1
    (S_i 1 = 0 and Pi^T S_i 1 = 0)."""
    c = 37.5
    Y = np.concatenate([np.zeros(small.N), small.gamma * small.mH * c])
    X = small.solve_dense(Y)
    np.testing.assert_allclose(X[:small.N], 0.0, atol=1e-10)
    np.testing.assert_allclose(X[small.N:], c, rtol=1e-12)


def test_rest_state_stays_at_rest(small):
    """At rest (V = 0, h = 1, no stimulus) every step returns exactly rest."""
    V = np.zeros(small.NH)
    h = np.ones(small.NH)
    U, V1, h1 = small.step(V, h, n=10**6)   # far outside the stimulus window
    assert np.abs(U).max() < 1e-13 and np.abs(V1).max() < 1e-13
    np.testing.assert_allclose(h1, 1.0)


def test_stimulus_window():
    s = bd.System(w.square2d(n=12))
    assert s.n0 == 0 and s.n1 == 20
    assert s.i_stim(19).max() == 50.0 and s.i_stim(20).max() == 0.0


def test_ms_fixed_points():
    """With h = 1 frozen the MS model has equilibria at vt = 0 and at the two
    roots of vt (1 - vt) = tau_in / tau_out; between the lower two roots
    the current is depolarising (negative I_ion)."""
    r = ionic.TAU_IN / ionic.TAU_OUT
    lo = (1 - np.sqrt(1 - 4 * r)) / 2
    hi = (1 + np.sqrt(1 - 4 * r)) / 2
    assert abs(lo - 0.0528) < 1e-4 and abs(hi - 0.9472) < 1e-4
    for vt in (0.0, lo, hi):
        assert abs(ionic.i_ion(vt * ionic.DV, 1.0, 1.0)) < 1e-12
    assert ionic.i_ion(0.5 * lo * ionic.DV, 1.0, 1.0) > 0
    assert ionic.i_ion(0.5 * ionic.DV, 1.0, 1.0) < 0
    assert ionic.i_ion(1.2 * ionic.DV, 1.0, 1.0) > 0


def test_gate_relaxation():
    """Forward Euler on dh/dt converges to the exponential relaxation
    h(t) = 1 - (1 - h0) exp(-t / tau_open) below the gate threshold, and
    h(t) = h0 exp(-t / tau_close) above it."""
    for V, h0, exact in ((0.0, 0.2, lambda t: 1 - 0.8 * np.exp(-t / 120.0)),
                         (50.0, 0.9, lambda t: 0.9 * np.exp(-t / 150.0))):
        T = 30.0
        errs = []
        for n in (100, 200):
            h = np.array([h0])
            dt = T / n
            for _ in range(n):
                h = h + dt * ionic.gate_rate(np.array([V]), h)
            errs.append(abs(h[0] - exact(T)))
        assert errs[1] < 0.6 * errs[0] and errs[1] < 1e-3


def _bump_state(s):
    """A smooth transmembrane bump on the heart and the potential U that the
    elliptic row (S_1 U + Pi^T S_i V = 0) gives it, normalised."""
    xy = s.cfg["xyz"][s.hn]
    c = xy.mean(axis=0)
    V = 60.0 * np.exp(-np.sum((xy - c) ** 2, axis=1) / 4.0)
    rhs = -(s.PiT @ (s.Si @ V))
    U = np.linalg.lstsq(s.S1.toarray(), rhs, rcond=None)[0]
    U -= (s.m @ U) / s.m.sum()
    return U, V


@pytest.mark.parametrize("scheme,order", [("euler", 1.0), ("cn", 2.0)])
def test_time_scheme_orders(scheme, order):
    """Without the reaction terms the problem is linear; from a smooth state
    the backward-Euler scheme of Sec. 3.2 converges at order 1 in dt and the
    Crank-Nicolson reading at order 2 (errors against a CN run at dt/16)."""
    cfg = w.square2d(n=8)
    T = 2.0

    def run(dt, sch):
        s = bd.System(cfg, dt=dt, scheme=sch, reaction=False)
        U, V = _bump_state(s)
        h = np.ones(s.NH)
        for n in range(int(round(T / dt))):
            U, V, h = s.step(V, h, n, method="dense", U0=U)
        return V

    ref = run(0.2 / 16, "cn")
    errs = [np.linalg.norm(run(dt, scheme) - ref) for dt in (0.2, 0.1, 0.05)]
    rates = [np.log2(errs[k] / errs[k + 1]) for k in range(2)]
    print(scheme, "errors", errs, "rates", rates)
    assert all(abs(r - order) < 0.25 for r in rates), rates


def test_cn_rest_and_constants():
    """Crank-Nicolson keeps rest at rest, and a constant V with U = 0 (a
    state the elliptic row admits) is stationary without reaction."""
    cfg = w.square2d(n=12)
    s = bd.System(cfg, scheme="cn")
    U, V1, h1 = s.step(np.zeros(s.NH), np.ones(s.NH), n=10**6, U0=np.zeros(s.N))
    assert np.abs(U).max() < 1e-13 and np.abs(V1).max() < 1e-13
    lin = bd.System(cfg, scheme="cn", reaction=False)
    c = 12.5
    U, V1, _ = lin.step(np.full(lin.NH, c), np.ones(lin.NH), 0, U0=np.zeros(lin.N))
    np.testing.assert_allclose(V1, c, rtol=1e-12)
    assert np.abs(U).max() < 1e-10
    assert abs(lin.gamma_eff - 2.0 * lin.gamma) < 1e-12 * lin.gamma


def test_strang_without_reaction_is_crank_nicolson():
    """With the reaction switched off the reaction half-steps are the
    identity, so the splitting is exactly the Crank-Nicolson step."""
    cfg = w.square2d(n=8)
    a = bd.System(cfg, scheme="strang", reaction=False)
    b = bd.System(cfg, scheme="cn", reaction=False)
    U, V = _bump_state(a)
    h = np.ones(a.NH)
    Ua, Va, ha = a.step(V, h, 0, method="dense", U0=U)
    Ub, Vb, hb = b.step(V, h, 0, method="dense", U0=U)
    assert np.abs(Va - Vb).max() <= 1e-12 * np.abs(Vb).max()
    assert np.abs(Ua - Ub).max() <= 1e-12 * np.abs(Ub).max() and np.array_equal(ha, h)


def test_reaction_half_step_is_heun():
    """One half-step of a single uniform vertex state against Heun's method
    written out for the scalar ODE system (no diffusion involved)."""
    from oracle import ionic
    cfg = w.square2d(n=4)
    s = bd.System(cfg, scheme="strang")
    V = np.full(s.NH, 7.0)
    h = np.full(s.NH, 0.8)
    Vs, hs = s.reaction_half(V, h, 10 ** 6)       # no stimulus
    tau = s.dt / 2

    def f(v, w):
        return -ionic.i_ion(np.array([v]), np.array([w]), s.cm)[0] / s.cm, ionic.gate_rate(np.array([v]), np.array([w]))[0]
    a1, b1 = f(7.0, 0.8)
    a2, b2 = f(7.0 + tau * a1, 0.8 + tau * b1)
    assert np.allclose(Vs, 7.0 + tau / 2 * (a1 + a2), rtol=1e-15, atol=0)
    assert np.allclose(hs, 0.8 + tau / 2 * (b1 + b2), rtol=1e-15, atol=0)


@pytest.mark.parametrize("scheme,order", [("euler", 1.0), ("strang", 2.0)])
def test_orders_with_reaction(scheme, order):
    """With the reaction on, in a smooth regime (potentials below the gate
    threshold, no stimulus), the semi-implicit scheme converges at order 1
    and the Strang splitting at order 2 (errors against a Strang run at
    dt/16)."""
    cfg = dict(w.square2d(n=8))
    cfg["stim_amp"] = 0.0
    T = 2.0

    def run(dt, sch):
        s = bd.System(cfg, dt=dt, scheme=sch)
        U, V = _bump_state(s)
        V = V * (8.0 / 60.0)                      # peak 8 mV: below the 13 mV gate threshold
        U = U * (8.0 / 60.0)
        h = np.full(s.NH, 0.9)
        for n in range(int(round(T / dt))):
            U, V, h = s.step(V, h, n, method="dense", U0=U)
        return V

    ref = run(0.2 / 16, "strang")
    errs = [np.linalg.norm(run(dt, scheme) - ref) for dt in (0.2, 0.1, 0.05)]
    rates = [np.log2(errs[k] / errs[k + 1]) for k in range(2)]
    print(scheme, "errors", errs, "rates", rates)
    assert all(abs(r - order) < 0.3 for r in rates), rates


@pytest.mark.parametrize("mk", [lambda: w.thorax2d(n_target=3000, seed=5), lambda: w.slab3d(n=6)],
                         ids=["thorax3000", "slab6"])
def test_sampled_residual_rows_equal_the_assembled_system(mk):
    """The row-by-row residual used for full-size checks (each row assembled
    from the elements of its vertex) equals the rows of Lambda X - Y of the
    fully assembled system, for an arbitrary X (torso and heart rows)."""
    cfg = mk()
    s = bd.System(cfg)
    rng = np.random.default_rng(8)
    Vn = rng.uniform(0, 100, s.NH)
    hn = rng.uniform(0, 1, s.NH)
    U1 = rng.normal(size=s.N)
    V1 = rng.normal(size=s.NH)
    n = 0
    Y = s.rhs(Vn, hn, n)
    X = np.concatenate([s.from_global_u(U1), V1])
    R = s.Lam @ X - Y
    Ru = s.to_global_u(R[:s.N])
    verts = rng.choice(s.N, size=min(200, s.N), replace=False)
    ru, rv, yv = bd.sampled_residual(cfg, verts, Vn, hn, n, U1, V1)
    np.testing.assert_allclose(ru, Ru[verts], rtol=1e-12, atol=1e-12 * np.abs(Ru).max())
    loc = -np.ones(s.N, dtype=np.int64)
    loc[s.hn] = np.arange(s.NH)
    hv = verts[loc[verts] >= 0]
    assert len(hv) > 0
    np.testing.assert_allclose(rv, R[s.N + loc[hv]], rtol=1e-12, atol=1e-12 * np.abs(R[s.N:]).max())
    np.testing.assert_allclose(yv, Y[s.N + loc[hv]], rtol=1e-13, atol=0)
