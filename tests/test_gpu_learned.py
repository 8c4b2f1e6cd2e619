"""GPU learned corrections against the FP64 oracle network (oracle.mpnn).

The device network runs in BF16 (weights and activations) with FP32
accumulation, so forward values, stencil values and gradients are compared
at BF16 tolerance after rounding the oracle's weights to BF16.  The
corrected flexible CG (learned stencil or additive correction) must still
reach the oracle's normalised solution at 1e-8."""
import numpy as np
import pytest

import workloads as w

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _bf16(x):
    """Round FP64 values to the nearest BF16 (ties to even), as FP64."""
    f = np.asarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    f = (f + 0x7FFF + ((f >> 16) & 1)) >> 16
    return (f.astype(np.uint32) << 16).view(np.float32).astype(np.float64)


@pytest.fixture(scope="module")
def setup(torch):
    import paper_1711_08708_amd as B
    from oracle import bidomain as bd, mpnn
    cfg = w.thorax2d(n_target=6000, seed=21)
    s = bd.System(cfg)
    A = mpnn.aggregation_matrix(s.Sm)
    st = mpnn.static_features(cfg, s.Sm)
    solver = B.Solver(cfg, eps_h=0.0, tol=1e-12)
    rng = np.random.default_rng(5)
    theta = _bf16(mpnn.init_params(7) + np.concatenate(
        [np.zeros(mpnn.N_PARAMS - 33), rng.normal(0, 0.2, 33)]))
    return B, mpnn, s, A, st, solver, theta


def test_forward_matches_oracle(torch, setup):
    B, mpnn, s, A, st, solver, theta = setup
    solver.set_weights(theta)
    rng = np.random.default_rng(11)
    t = rng.normal(size=s.NH)
    d_gpu = solver.gnn_eval(torch.tensor(t, device="cuda")).cpu().numpy()
    f, nt = mpnn.features(t, st)
    o, _ = mpnn.forward(theta, A, f)
    d_ref = nt * o
    err = np.linalg.norm(d_gpu - d_ref) / np.linalg.norm(d_ref)
    print(f"forward rel err {err:.2e}")
    assert err < 3e-2


def test_gradient_matches_oracle(torch, setup):
    B, mpnn, s, A, st, solver, theta = setup
    solver.set_weights(theta)
    rng = np.random.default_rng(12)
    t = rng.normal(size=s.NH)
    that = (t / (np.linalg.norm(t) / np.sqrt(s.NH))).astype(np.float32)
    y = (rng.normal(size=s.NH) * 0.5).astype(np.float32)
    loss_g, grad_g = solver.gnn_loss_grad(torch.tensor(that, device="cuda"),
                                          torch.tensor(y, device="cuda"))
    f, _ = mpnn.features(t, st)
    f[:, 0] = that
    W = mpnn.energy_weight(s.gamma * np.diag(s.mH) + s.Sm.toarray())
    loss_r, grad_r = mpnn.loss_and_grad(theta, A, f, y.astype(np.float64), W)
    el = abs(loss_g - loss_r) / abs(loss_r)
    eg = np.linalg.norm(grad_g - grad_r) / np.linalg.norm(grad_r)
    print(f"loss rel err {el:.2e}, gradient rel err {eg:.2e}")
    assert el < 3e-2 and eg < 6e-2


def test_stencil_matches_oracle(torch, setup):
    """C^ zh - bh, its squared norm and the weight gradient against the
    oracle's stencil regression (static-feature embedding, f0 = 1)."""
    B, mpnn, s, A, st, solver, theta = setup
    solver.set_weights(theta)
    rng = np.random.default_rng(13)
    zh = rng.normal(size=s.NH).astype(np.float32)
    bh = (rng.normal(size=s.NH) * 0.3).astype(np.float32)
    r_g, loss_g, grad_g = solver.stencil_check(torch.tensor(zh, device="cuda"), torch.tensor(bh, device="cuda"))
    f = mpnn.static_input(st)
    C = mpnn.stencil_matrix(theta, A, f, s.Sm)
    r_o = C @ zh.astype(np.float64) - bh
    loss_o, grad_o = mpnn.stencil_loss_and_grad(theta, A, f, s.Sm, zh[None, :].astype(np.float64),
                                                bh[None, :].astype(np.float64))
    er = np.linalg.norm(r_g.cpu().numpy() - r_o) / np.linalg.norm(r_o)
    el = abs(loss_g - loss_o) / loss_o
    eg = np.linalg.norm(grad_g - grad_o) / np.linalg.norm(grad_o)
    print(f"stencil residual rel err {er:.2e}, loss {el:.2e}, gradient {eg:.2e}")
    assert er < 3e-2 and el < 3e-2 and eg < 6e-2


def _solve_steps(torch, solver, s, state, n0, n_steps, learned):
    import paper_1711_08708_amd as B
    v, h, u = [x.clone() for x in state]
    solver.set_precond(learned if learned else B.PRECOND_PLAIN)
    solver.reset_guess()                # runs compared from equal starting points
    iters, worst, fb = [], 0.0, 0
    for n in range(n0, n0 + n_steps):
        Vn, hn = v.cpu().numpy().copy(), h.cpu().numpy().copy()
        st = solver.step(v, h, u, n)
        iters.append(st["iterations"])
        fb += st["fallbacks"]
        Uo, Vo, _ = s.step(Vn, hn, n)
        Uo = s.to_global_u(Uo)
        eu = np.linalg.norm(u.cpu().numpy() - Uo) / np.linalg.norm(Uo)
        ev = np.linalg.norm(v.cpu().numpy() - Vo) / np.linalg.norm(Vo)
        worst = max(worst, eu, ev)
    return iters, worst, fb, (v, h, u)


@pytest.fixture(scope="module")
def collected(torch, setup):
    B, mpnn, s, A, st, solver, theta = setup
    solver.set_weights(mpnn.init_params(3) * np.concatenate([np.ones(mpnn.N_PARAMS - 33), np.zeros(33)]))
    solver.set_precond(B.PRECOND_PLAIN)
    v, h, u = solver.state()
    info = solver.learn_collect(v, h, u, 0, 12, max_samples=256)
    print("collected", info["samples"], "pairs over 12 steps")
    assert info["samples"] >= 24
    return (v, h, u)


def test_learned_stencil_and_flexible_cg(torch, setup, collected):
    """The stencil regression goes below the loss of C = 0; K_m + C stays
    SPD and is factored; flexible CG with it keeps 1e-8 parity."""
    B, mpnn, s, A, st, solver, theta = setup
    with pytest.raises(B.BidoError):
        solver.set_precond(B.PRECOND_LEARNED)      # not trained yet
    ts = solver.learn_train(kind=B.LEARN_STENCIL, epochs=30, batch=4, lr=2e-3, seed=1, n_val=4)
    print("train stencil", ts)
    assert ts["loss_last"] < ts["loss_first"] and ts["loss_last"] < ts["loss_zero"]
    # the kept weights are those of the lowest held-out loss, the untrained
    # ones (C = 0 here) included
    assert ts["best_epoch"] > 0 and ts["loss_val"] <= ts["loss_zero_val"]
    assert ts["spd"] == 1
    it_p, wp, _, _ = _solve_steps(torch, solver, s, collected, 12, 6, learned=0)
    it_l, wl, fb, _ = _solve_steps(torch, solver, s, collected, 12, 6, learned=B.PRECOND_LEARNED)
    print("iterations plain", it_p, "stencil", it_l, "worst err", wp, wl)
    assert wp <= 1e-8 and wl <= 1e-8
    assert fb == 0


def test_learned_additive_and_flexible_cg(torch, setup, collected):
    """Additive correction: training goes below the zero correction's loss;
    corrected flexible CG keeps 1e-8 parity."""
    B, mpnn, s, A, st, solver, theta = setup
    solver.set_weights(mpnn.init_params(3) * np.concatenate([np.ones(mpnn.N_PARAMS - 33), np.zeros(33)]))
    ts = solver.learn_train(kind=B.LEARN_ADDITIVE, epochs=40, batch=4, lr=2e-3, seed=1, n_val=4)
    print("train additive", ts)
    assert ts["loss_last"] < ts["loss_first"]
    assert ts["loss_last"] < ts["loss_zero"]
    it_p, wp, _, _ = _solve_steps(torch, solver, s, collected, 12, 6, learned=0)
    it_l, wl, fb, _ = _solve_steps(torch, solver, s, collected, 12, 6, learned=B.PRECOND_LEARNED_ADDITIVE)
    print("iterations plain", it_p, "additive", it_l, "fallbacks", fb, "worst err", wp, wl)
    assert wp <= 1e-8 and wl <= 1e-8


def _gain(torch, setup, collected, kind):
    """Iterations of the plain block-LU preconditioner and of the trained
    correction on the 6 held-out steps after the 12 collected ones, each run
    from the same state and a fresh span of initial-guess states, both at
    1e-8 parity."""
    B, mpnn, s, A, st, solver, theta = setup
    solver.set_weights(mpnn.init_params(3) * np.concatenate([np.ones(mpnn.N_PARAMS - 33), np.zeros(33)]))
    if kind == "stencil":
        ts = solver.learn_train(kind=B.LEARN_STENCIL, epochs=30, batch=4, lr=2e-3, seed=1, n_val=4)
        mode = B.PRECOND_LEARNED
    else:
        ts = solver.learn_train(kind=B.LEARN_ADDITIVE, epochs=40, batch=4, lr=2e-3, seed=1, n_val=4)
        mode = B.PRECOND_LEARNED_ADDITIVE
    it_p, wp, _, _ = _solve_steps(torch, solver, s, collected, 12, 6, learned=0)
    it_l, wl, _, _ = _solve_steps(torch, solver, s, collected, 12, 6, learned=mode)
    print(f"gain {kind}: plain {sum(it_p)} ({it_p}) learned {sum(it_l)} ({it_l}), kept epoch {ts['best_epoch']}",
          flush=True)
    assert wp <= 1e-8 and wl <= 1e-8
    return it_p, it_l


def test_learned_stencil_gain(torch, setup, collected):
    """What the trained stencil gains over the plain block-LU preconditioner
    on held-out steps (thorax6000 with exact inner factors: 23 -> 21
    iterations over 6 steps): fewer iterations in total."""
    it_p, it_l = _gain(torch, setup, collected, "stencil")
    assert sum(it_l) < sum(it_p)


@pytest.mark.xfail(reason="the trained additive correction does not lower the iteration count: "
                          "measured thorax6000 23 plain vs 25 additive over 6 held-out steps", strict=False)
def test_learned_additive_gain(torch, setup, collected):
    """The same for the additive correction of the Schur-complement solve."""
    it_p, it_l = _gain(torch, setup, collected, "additive")
    assert sum(it_l) < sum(it_p)


def test_fallback_keeps_parity(torch, setup):
    """A network with large random weights gives non-descent directions; the
    solve falls back to the plain apply there and still converges."""
    B, mpnn, s, A, st, solver, theta = setup
    rng = np.random.default_rng(9)
    solver.set_weights(rng.normal(0, 30.0, mpnn.N_PARAMS))
    v, h, u = solver.state()
    it, worst, fb, _ = _solve_steps(torch, solver, s, (v, h, u), 0, 3, learned=B.PRECOND_LEARNED_ADDITIVE)
    print("iterations", it, "fallbacks", fb, "worst err", worst)
    assert worst <= 1e-8
