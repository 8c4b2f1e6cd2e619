"""GPU: changing the time step of a context (bido_set_dt), with the factored
P_K (host refactorisation of K_m) and with the Chebyshev P_K (device update
only), against the oracle at the new step."""
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


@pytest.mark.parametrize("scheme", ["euler", "cn", "strang"])
@pytest.mark.parametrize("pk", ["cholesky", "chebyshev"])
def test_steps_after_set_dt_match_oracle(torch, pk, scheme):
    """Three steps at dt, the step changed to 0.4 dt, three more steps: each
    later step matches the oracle's step at the new dt from the same state,
    and a context created at the new dt takes the same steps."""
    import paper_1711_08708_amd as B
    from oracle import bidomain as bd
    cfg = w.thorax2d(n_target=3000, seed=11)
    sch = {"euler": B.SCHEME_EULER, "cn": B.SCHEME_CN, "strang": B.SCHEME_STRANG}[scheme]
    dt2 = 0.4 * cfg["dt"]
    sv = B.Solver(cfg, eps_h=0.0, tol=1e-12, scheme=sch)
    if pk == "chebyshev":
        sv.set_pk(B.PK_CHEBYSHEV, 3)
    v, h, u = sv.state()
    for n in range(3):
        sv.step(v, h, u, n)
    sec = sv.set_dt(dt2)
    print(f"{pk} {scheme}: set_dt took {sec * 1e3:.2f} ms", flush=True)
    if pk == "chebyshev":
        iv = B.HostSetup(cfg, scheme=sch, dt=dt2).pk_interval()
        got = sv.pk()
        assert got["lo"] == iv["lo"] and got["hi"] == iv["hi"]
    fresh = B.Solver(cfg, eps_h=0.0, tol=1e-12, scheme=sch, dt=dt2)
    if pk == "chebyshev":
        fresh.set_pk(B.PK_CHEBYSHEV, 3)
    fv, fh, fu = [t.clone() for t in (v, h, u)]
    s = bd.System(cfg, dt=dt2, scheme=scheme)
    for n in range(3, 6):
        Vn, hn = v.cpu().numpy().copy(), h.cpu().numpy().copy()
        Un = s.from_global_u(u.cpu().numpy())
        st = sv.step(v, h, u, n)
        stf = fresh.step(fv, fh, fu, n)
        assert st["converged"] == 1 and st["iterations"] == stf["iterations"]
        Uo_p, Vo, _ = s.step(Vn, hn, n, U0=Un)
        Uo = s.to_global_u(Uo_p)
        U, V = u.cpu().numpy(), v.cpu().numpy()
        eu = np.linalg.norm(U - Uo) / np.linalg.norm(Uo)
        ev = np.linalg.norm(V - Vo) / np.linalg.norm(Vo)
        assert eu <= 1e-8 and ev <= 1e-8, (n, eu, ev)
        for a, b in ((u, fu), (v, fv), (h, fh)):
            a_, b_ = a.cpu().numpy(), b.cpu().numpy()
            assert np.linalg.norm(a_ - b_) <= 1e-12 * np.linalg.norm(b_)
    # the old step is refused now
    with pytest.raises(B.BidoError, match="BIDO_ERR_DT_MISMATCH"):
        B._check(B.lib.bido_step(sv.ctx, sv._dev(v, sv.NH), sv._dev(h, sv.NH), sv._dev(u, sv.N), cfg["dt"], 6,
                                 None))
    sv.close()
    fresh.close()


def test_set_dt_arguments_and_batch(torch):
    import paper_1711_08708_amd as B
    cfgs = [w.thorax2d(n_target=2000, seed=5), w.thorax2d(n_target=1500, seed=6)]
    svs = [B.Solver(c) for c in cfgs]
    for dt in (0.0, -0.1, float("nan")):
        with pytest.raises(B.BidoError, match="BIDO_ERR_ARG"):
            svs[0].set_dt(dt)
    assert svs[0].set_dt(cfgs[0]["dt"]) == 0.0          # same step: nothing to do
    batch = B.Batch(svs, fused=True)
    with pytest.raises(B.BidoError, match="BIDO_ERR_STATE"):
        svs[0].set_dt(0.05)
    batch.close()
    for s in svs:
        s.set_dt(0.05)
    batch = B.Batch(svs, fused=True)                    # a batch at the new step
    states = [s.state() for s in svs]
    tot, _ = batch.run(states, 0, 2)
    assert tot["converged"] == 1
    batch.close()
    for s in svs:
        s.close()


def test_set_dt_resets_the_learned_correction(torch):
    """Pairs and a trained stencil belong to K_m at the old step: after the
    change the sample store is empty, the learned stencil cannot be selected
    until trained again, and training at the new step works."""
    import ctypes
    import paper_1711_08708_amd as B
    cfg = w.thorax2d(n_target=3000, seed=11)
    sv = B.Solver(cfg, tol=1e-10)
    w0 = sv.weights()
    v, h, u = sv.state()
    col = sv.learn_collect(v, h, u, 0, 6, max_samples=64)
    assert col["samples"] > 0
    ts = sv.learn_train(kind=B.LEARN_STENCIL, epochs=2, batch=8, lr=2e-3, seed=0, n_val=1)
    if ts["spd"]:
        sv.set_precond(B.PRECOND_LEARNED)
    # training keeps its best held-out epoch, which may be the initial one:
    # move the weights off the initial ones in any case
    sv.set_weights(sv.weights() + 0.01)
    assert not np.array_equal(sv.weights(), w0)
    sv.set_dt(0.05)
    assert np.array_equal(sv.weights(), w0)          # the weights start again
    n = ctypes.c_int()
    B._check(B.lib.bido_learn_samples(sv.ctx, ctypes.byref(n)))
    assert n.value == 0
    with pytest.raises(B.BidoError, match="BIDO_ERR_STATE"):
        sv.set_precond(B.PRECOND_LEARNED)
    assert sv.step(v, h, u, 6)["converged"] == 1
    col = sv.learn_collect(v, h, u, 7, 6, max_samples=64)
    assert col["samples"] > 0
    ts = sv.learn_train(kind=B.LEARN_STENCIL, epochs=2, batch=8, lr=2e-3, seed=0, n_val=1)
    assert np.isfinite(ts["loss_last"])
    sv.close()
