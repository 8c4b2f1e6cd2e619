"""Batched execution of independent slices (bido_batch_*).

Each slice of a batch runs the same kernels in the same order as on its
own, with its own PCG scalars, so a batch must reproduce the per-slice runs
bit for bit; the last step of every slice is also checked against the FP64
oracle at 1e-8."""
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


def _slices():
    return [w.thorax2d(n_target=3000, seed=31), w.thorax2d(n_target=6000, seed=32, sigma_scale=0.8),
            w.square2d(n=24, seed=3), w.thorax2d(n_target=1500, seed=33, sigma_scale=1.2)]


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_batch_matches_single_slices_and_oracle(torch, precision):
    import paper_1711_08708_amd as B
    from oracle import bidomain as bd
    prec = B.PREC_MIXED if precision == "mixed" else B.PREC_FP64
    cfgs = _slices()
    n_steps = 12
    # reference: each slice alone, every kernel launched eagerly (the batch
    # replays captured graphs)
    ref = []
    for cfg in cfgs:
        s = B.Solver(cfg, tol=1e-12, precision=prec)
        s.set_graphs(False)
        v, h, u = s.state()
        s.run(v, h, u, 0, n_steps)
        ref.append((v.cpu().numpy(), h.cpu().numpy(), u.cpu().numpy()))
        s.close()
    solvers = [B.Solver(cfg, tol=1e-12, precision=prec) for cfg in cfgs]
    batch = B.Batch(solvers, n_streams=3)
    states = [s.state() for s in solvers]
    tot, per = batch.run(states, 0, n_steps - 1)
    before = [(st[0].cpu().numpy().copy(), st[1].cpu().numpy().copy()) for st in states]
    tot2, per2 = batch.run(states, n_steps - 1, 1)
    print(precision, "iterations per slice (last step)", [p["iterations"] for p in per2],
          "batch max", tot["iterations"], "total", tot["total_iterations"] + tot2["total_iterations"])
    assert tot["converged"] == 1 and tot2["converged"] == 1
    for k, (cfg, st) in enumerate(zip(cfgs, states)):
        v, h, u = [t.cpu().numpy() for t in st]
        # bit-identical to the slice run on its own
        assert np.array_equal(v, ref[k][0]) and np.array_equal(h, ref[k][1]) and np.array_equal(u, ref[k][2]), k
        # last step against the oracle
        sy = bd.System(cfg)
        Uo, Vo, _ = sy.step(before[k][0], before[k][1], n_steps - 1)
        Uo = sy.to_global_u(Uo)
        eu = np.linalg.norm(u - Uo) / np.linalg.norm(Uo)
        ev = np.linalg.norm(v - Vo) / np.linalg.norm(Vo)
        print(f"  slice {k} ({cfg['name']}): e_u {eu:.2e} e_v {ev:.2e}")
        assert eu <= 1e-8 and ev <= 1e-8
    batch.close()
    for s in solvers:
        s.close()


def test_batch_refusals(torch):
    import paper_1711_08708_amd as B
    cfgs = _slices()[:2]
    a, b = [B.Solver(cfg, tol=1e-10) for cfg in cfgs]
    with pytest.raises(B.BidoError):
        B.Batch([a, a])                      # listed twice
    bt = B.Batch([a, b])
    with pytest.raises(B.BidoError):
        B.Batch([b])                         # already in a batch
    a.set_precond(B.PRECOND_LEARNED_ADDITIVE)
    states = [a.state(), b.state()]
    with pytest.raises(B.BidoError):
        bt.run(states, 0, 1)                 # additive learned mode needs host checks
    bt.close()
    a.set_precond(B.PRECOND_PLAIN)
    v, h, u = a.state()
    a.run(v, h, u, 0, 2)                     # usable on its own again
    # a context destroyed while in a batch leaves it: the batch refuses to
    # run, closes cleanly, and the other context works on its own
    bt = B.Batch([a, b])
    a.close()
    with pytest.raises(B.BidoError):
        bt.run([states[0], states[1]], 0, 1)
    bt.close()
    v, h, u = b.state()
    assert b.step(v, h, u, 0)["converged"] == 1
    b.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_graph_replays_match_eager_launches(torch, precision):
    """The captured per-iteration graphs, replayed many times with eager
    work (Steps 1 and 3, normalisation) and host waits in between, give the
    same trajectory bit for bit as launching every kernel eagerly."""
    import paper_1711_08708_amd as B
    prec = B.PREC_MIXED if precision == "mixed" else B.PREC_FP64
    cfg = w.thorax2d(n_target=6000, seed=41)
    out = []
    for graphs in (False, True):
        s = B.Solver(cfg, tol=1e-12, precision=prec)
        s.set_graphs(graphs)
        v, h, u = s.state()
        its = [s.step(v, h, u, n)["iterations"] for n in range(15)]
        out.append(([t.cpu().numpy() for t in (v, h, u)], its))
        s.close()
    print(precision, "iterations", out[1][1])
    assert out[0][1] == out[1][1]
    for a, b in zip(out[0][0], out[1][0]):
        assert np.array_equal(a, b)


def _single_runs(B, cfgs, prec, n_steps, pk_steps=0, **kw):
    out = []
    for cfg in cfgs:
        s = B.Solver(cfg, tol=1e-12, precision=prec, **kw)
        if pk_steps:
            s.set_pk(B.PK_CHEBYSHEV, pk_steps)
        s.set_graphs(False)
        v, h, u = s.state()
        its = [s.step(v, h, u, n)["iterations"] for n in range(n_steps)]
        out.append(((v.cpu().numpy(), h.cpu().numpy(), u.cpu().numpy()), its))
        s.close()
    return out


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_fused_batch_matches_single_slices_and_oracle(torch, precision):
    """One union PCG over all slices (segmented vector kernels with per-slice
    scalars, merged forests of the factors) follows each slice's own solve:
    same iteration counts within one, states within 1e-9 of the slice run
    alone (only the rounding order of the reductions differs), last step
    against the FP64 oracle at 1e-8."""
    import paper_1711_08708_amd as B
    from oracle import bidomain as bd
    prec = B.PREC_MIXED if precision == "mixed" else B.PREC_FP64
    cfgs = _slices() + [w.square2d(n=6, seed=4)]        # plus a one-block slice
    n_steps = 12
    ref = _single_runs(B, cfgs, prec, n_steps)
    solvers = [B.Solver(cfg, tol=1e-12, precision=prec) for cfg in cfgs]
    batch = B.Batch(solvers, fused=True)
    info = batch.info()
    print(precision, "fused union", info)
    assert info["fused"] and info["n_union"] == sum(s.N + s.NH for s in solvers)
    states = [s.state() for s in solvers]
    its = []
    for n in range(n_steps - 1):
        tot, per = batch.run(states, n, 1)
        assert tot["converged"] == 1
        its.append([p["iterations"] for p in per])
    before = [(st[0].cpu().numpy().copy(), st[1].cpu().numpy().copy()) for st in states]
    tot, per = batch.run(states, n_steps - 1, 1)
    its.append([p["iterations"] for p in per])
    # the stopping test runs on the device: the host waits about twice per
    # step (one less than the previous step's count, then one at a time),
    # not once per iteration
    cnt = batch.counters()
    per_step = max(max(row) for row in its[1:])
    print(precision, "counters", cnt, "iterations per step up to", per_step)
    assert cnt["steps"] == n_steps
    assert cnt["host_waits"] <= 3 * cnt["steps"] < cnt["iterations"]
    for k, (cfg, st) in enumerate(zip(cfgs, states)):
        v, h, u = [t.cpu().numpy() for t in st]
        fused_its = [row[k] for row in its]
        print(f"  slice {k} ({cfg['name']}): iterations fused {fused_its} alone {ref[k][1]}")
        assert all(abs(a - b) <= 1 for a, b in zip(fused_its, ref[k][1]))
        for a, b in zip((v, h, u), ref[k][0]):
            assert np.linalg.norm(a - b) <= 1e-9 * np.linalg.norm(b), k
        sy = bd.System(cfg)
        Uo, Vo, _ = sy.step(before[k][0], before[k][1], n_steps - 1)
        Uo = sy.to_global_u(Uo)
        eu = np.linalg.norm(u - Uo) / np.linalg.norm(Uo)
        ev = np.linalg.norm(v - Vo) / np.linalg.norm(Vo)
        print(f"    e_u {eu:.2e} e_v {ev:.2e}")
        assert eu <= 1e-8 and ev <= 1e-8
    batch.close()
    # the contexts work on their own again, on their own vectors
    v, h, u = solvers[0].state()
    assert solvers[0].step(v, h, u, 0)["converged"] == 1
    for s in solvers:
        s.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_fused_batch_learned_stencil(torch, precision):
    """Slices with a trained stencil (P_K = (K_m + C)^-1, C on the pattern of
    S_m) next to a plain slice in one fused batch: the learned slices bring
    their factor of K_m + C into the merged forest and the union PCG takes the
    flexible direction update, as each slice run alone does.  Iteration counts
    within one of the slices run alone, states within 1e-9, the last step
    against the FP64 oracle at 1e-8."""
    import paper_1711_08708_amd as B
    from oracle import bidomain as bd, mpnn
    prec = B.PREC_MIXED if precision == "mixed" else B.PREC_FP64
    cfgs = _slices()[:3]
    learned = [True, False, True]
    # the network starts with a zero last layer (C = 0)
    theta = mpnn.init_params(3) * np.concatenate([np.ones(mpnn.N_PARAMS - 33), np.zeros(33)])
    solvers = [B.Solver(cfg, tol=1e-12, precision=prec) for cfg in cfgs]
    for s, ln in zip(solvers, learned):
        if not ln:
            continue
        s.set_weights(theta)
        v, h, u = s.state()
        info = s.learn_collect(v, h, u, 0, 8, max_samples=64)
        ts = s.learn_train(kind=B.LEARN_STENCIL, epochs=10, batch=4, lr=2e-3, seed=1, n_val=2)
        print("collected", info["samples"], "train", ts)
        assert ts["spd"] == 1
        s.set_precond(B.PRECOND_LEARNED)
    n_steps = 8
    ref = []
    for s in solvers:
        v, h, u = s.state()
        its = [s.step(v, h, u, n)["iterations"] for n in range(n_steps)]
        ref.append(((v.cpu().numpy(), h.cpu().numpy(), u.cpu().numpy()), its))
    batch = B.Batch(solvers, fused=True)
    states = [s.state() for s in solvers]
    its = [[p["iterations"] for p in batch.run(states, n, 1)[1]] for n in range(n_steps - 1)]
    before = [(st[0].cpu().numpy().copy(), st[1].cpu().numpy().copy()) for st in states]
    its.append([p["iterations"] for p in batch.run(states, n_steps - 1, 1)[1]])
    with pytest.raises(B.BidoError):
        solvers[0].set_precond(B.PRECOND_PLAIN)     # fixed while batched
    for k, (cfg, st) in enumerate(zip(cfgs, states)):
        v, h, u = [t.cpu().numpy() for t in st]
        fused_its = [row[k] for row in its]
        print(f"  slice {k} learned={learned[k]}: iterations fused {fused_its} alone {ref[k][1]}")
        assert all(abs(a - b) <= 1 for a, b in zip(fused_its, ref[k][1]))
        for a, b in zip((v, h, u), ref[k][0]):
            assert np.linalg.norm(a - b) <= 1e-9 * np.linalg.norm(b), k
        sy = bd.System(cfg)
        Uo, Vo, _ = sy.step(before[k][0], before[k][1], n_steps - 1)
        Uo = sy.to_global_u(Uo)
        eu = np.linalg.norm(u - Uo) / np.linalg.norm(Uo)
        ev = np.linalg.norm(v - Vo) / np.linalg.norm(Vo)
        assert eu <= 1e-8 and ev <= 1e-8
    batch.close()
    for s in solvers:
        s.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_fused_graph_replays_match_eager(torch, precision):
    """The fused batch's captured iteration graphs, replayed with the per-slice
    step kernels and host checks between them, give the eager trajectory bit
    for bit."""
    import paper_1711_08708_amd as B
    prec = B.PREC_MIXED if precision == "mixed" else B.PREC_FP64
    cfgs = _slices()[:3]
    out = []
    for graphs in (False, True):
        solvers = [B.Solver(cfg, tol=1e-12, precision=prec) for cfg in cfgs]
        batch = B.Batch(solvers, fused=True)
        batch.set_graphs(graphs)
        states = [s.state() for s in solvers]
        its = [[p["iterations"] for p in batch.run(states, n, 1)[1]] for n in range(8)]
        out.append(([[t.cpu().numpy() for t in st] for st in states], its))
        batch.close()
        for s in solvers:
            s.close()
    assert out[0][1] == out[1][1]
    for a, b in zip(out[0][0], out[1][0]):
        for x, y in zip(a, b):
            assert np.array_equal(x, y)


def test_fused_batch_refusals(torch):
    import paper_1711_08708_amd as B
    cfgs = _slices()[:2]
    a = B.Solver(cfgs[0], tol=1e-10)
    b = B.Solver(cfgs[1], tol=1e-10, precision=B.PREC_MIXED)
    with pytest.raises(B.BidoError):
        B.Batch([a, b], fused=True)          # two precisions
    b.close()
    b = B.Solver(cfgs[1], tol=1e-10)
    with pytest.raises(B.BidoError):
        B.Batch([a, a], fused=True)          # listed twice
    a.set_precond(B.PRECOND_LEARNED_ADDITIVE)
    with pytest.raises(B.BidoError):
        B.Batch([a, b], fused=True)          # no additive network correction
    a.set_precond(B.PRECOND_PLAIN)
    bt = B.Batch([a, b], fused=True)
    with pytest.raises(B.BidoError):
        B.Batch([b], fused=True)             # already in a batch
    a.set_precision(B.PREC_MIXED)
    with pytest.raises(B.BidoError):
        bt.run([a.state(), b.state()], 0, 1)  # precision changed inside the batch
    bt.close()
    a.set_precision(B.PREC_FP64)
    v, h, u = a.state()
    a.run(v, h, u, 0, 2)
    # destroying a context of a fused batch gives it back its own vectors first
    bt = B.Batch([a, b], fused=True)
    st2 = [a.state(), b.state()]
    b.close()
    with pytest.raises(B.BidoError):
        bt.run(st2, 0, 1)
    bt.close()
    v, h, u = a.state()
    assert a.step(v, h, u, 0)["converged"] == 1
    a.close()


def test_fused_batch_crank_nicolson(torch):
    """A fused batch of Crank-Nicolson slices follows each slice run alone."""
    import paper_1711_08708_amd as B
    cfgs = _slices()[:3]
    n_steps = 8
    ref = _single_runs(B, cfgs, B.PREC_FP64, n_steps, scheme=B.SCHEME_CN)
    solvers = [B.Solver(cfg, tol=1e-12, scheme=B.SCHEME_CN) for cfg in cfgs]
    batch = B.Batch(solvers, fused=True)
    states = [s.state() for s in solvers]
    its = [[p["iterations"] for p in batch.run(states, n, 1)[1]] for n in range(n_steps)]
    for k, st in enumerate(states):
        print(k, "iterations fused", [row[k] for row in its], "alone", ref[k][1])
        for a, b in zip([t.cpu().numpy() for t in st], ref[k][0]):
            assert np.linalg.norm(a - b) <= 1e-9 * np.linalg.norm(b), k
    batch.close()
    for s in solvers:
        s.close()


def test_fused_batch_chebyshev_pk(torch):
    """Slices with the polynomial P_K (Chebyshev-accelerated Jacobi on K_m,
    each slice with its own interval) in one fused batch: segmented
    Chebyshev launches over the union follow each slice run alone, graph
    replays match eager launches bit for bit, the last step matches the
    oracle, and slices with different step counts are refused."""
    import paper_1711_08708_amd as B
    from oracle import bidomain as bd
    cfgs = _slices()
    n_steps = 8
    ref = _single_runs(B, cfgs, B.PREC_FP64, n_steps, pk_steps=3)
    out = []
    for graphs in (False, True):
        solvers = [B.Solver(cfg, tol=1e-12) for cfg in cfgs]
        for sv in solvers:
            sv.set_pk(B.PK_CHEBYSHEV, 3)
        batch = B.Batch(solvers, fused=True)
        batch.set_graphs(graphs)
        states = [sv.state() for sv in solvers]
        its = [[p["iterations"] for p in batch.run(states, n, 1)[1]] for n in range(n_steps - 1)]
        before = [(st[0].cpu().numpy().copy(), st[1].cpu().numpy().copy()) for st in states]
        its.append([p["iterations"] for p in batch.run(states, n_steps - 1, 1)[1]])
        out.append(([[t.cpu().numpy() for t in st] for st in states], its, before))
        batch.close()
        for sv in solvers:
            sv.close()
    assert out[0][1] == out[1][1]
    for a, b in zip(out[0][0], out[1][0]):
        for x, y in zip(a, b):
            assert np.array_equal(x, y)
    states, its, before = out[1]
    for k, cfg in enumerate(cfgs):
        fused_its = [row[k] for row in its]
        print(f"  slice {k} ({cfg['name']}): iterations fused {fused_its} alone {ref[k][1]}")
        assert all(abs(a - b) <= 1 for a, b in zip(fused_its, ref[k][1]))
        for a, b in zip(states[k], ref[k][0]):
            assert np.linalg.norm(a - b) <= 1e-9 * np.linalg.norm(b), k
        sy = bd.System(cfg)
        Uo, Vo, _ = sy.step(before[k][0], before[k][1], n_steps - 1)
        Uo = sy.to_global_u(Uo)
        v, _, u = states[k]
        assert np.linalg.norm(u - Uo) <= 1e-8 * np.linalg.norm(Uo)
        assert np.linalg.norm(v - Vo) <= 1e-8 * np.linalg.norm(Vo)
    solvers = [B.Solver(cfg, tol=1e-12) for cfg in cfgs[:2]]
    solvers[0].set_pk(B.PK_CHEBYSHEV, 3)
    solvers[1].set_pk(B.PK_CHEBYSHEV, 4)
    with pytest.raises(B.BidoError, match="BIDO_ERR_STATE"):
        B.Batch(solvers, fused=True)
    for sv in solvers:
        sv.close()


@pytest.mark.timeout(900)
@pytest.mark.parametrize("mode", ["fp64", "mixed_learned"])
def test_fused_batch64_sampled_slices_full_size(torch, mode):
    """batch64 at full size, in the fused configuration the bench times (FP64
    plain, and mixed precision with every slice's learned stencil, trained
    on pairs of its first steps): the smallest, the median and the largest
    of its 64 slices plus two others (one of them with a heart in two
    parts), 3 steps in one fused batch, each slice's last step against the
    FP64 oracle at 1e-8."""
    import paper_1711_08708_amd as B
    from oracle import bidomain as bd, mpnn
    kws = w.make_config("batch64")
    sizes = [kw["n_target"] for kw in kws]
    pick = sorted({int(np.argmin(sizes)), int(np.argsort(sizes)[len(sizes) // 2]), int(np.argmax(sizes)), 7, 20})
    cfgs = [w.thorax2d(**kws[k]) for k in pick]
    prec = B.PREC_MIXED if mode == "mixed_learned" else B.PREC_FP64
    solvers = [B.Solver(cfg, tol=1e-10, eps_h=1e-8, precision=prec) for cfg in cfgs]
    if mode == "mixed_learned":
        theta = mpnn.init_params(3) * np.concatenate([np.ones(mpnn.N_PARAMS - 33), np.zeros(33)])
        for sv in solvers:
            sv.set_weights(theta)
            v, h, u = sv.state()
            sv.learn_collect(v, h, u, 0, 6, max_samples=48)
            ts = sv.learn_train(kind=B.LEARN_STENCIL, epochs=10, batch=8, lr=2e-3, seed=0, n_val=2)
            assert ts["spd"] == 1
            sv.set_precond(B.PRECOND_LEARNED)
    batch = B.Batch(solvers, fused=True)
    states = [s.state() for s in solvers]
    batch.run(states, 0, 2)
    before = [(st[0].cpu().numpy().copy(), st[1].cpu().numpy().copy()) for st in states]
    tot, per = batch.run(states, 2, 1)
    assert tot["converged"] == 1
    for k, (cfg, st) in enumerate(zip(cfgs, states)):
        sy = bd.System(cfg)
        Uo, Vo, _ = sy.step(before[k][0], before[k][1], 2)
        Uo = sy.to_global_u(Uo)
        u, v = st[2].cpu().numpy(), st[0].cpu().numpy()
        eu = np.linalg.norm(u - Uo) / np.linalg.norm(Uo)
        ev = np.linalg.norm(v - Vo) / np.linalg.norm(Vo)
        print(f"  batch64 slice {pick[k]} ({cfg['name']}): iterations {per[k]['iterations']} "
              f"e_u {eu:.2e} e_v {ev:.2e}")
        assert eu <= 1e-8 and ev <= 1e-8
    batch.close()
    for s in solvers:
        s.close()


def test_fused_batch_profiler(torch):
    """bido_batch_profile brackets the union's sweeps with events: records
    for the triangular classes with their algorithmic bytes, no change of
    the trajectory (the profiled steps launch eagerly), and a batch on
    streams is refused."""
    import paper_1711_08708_amd as B
    cfgs = _slices()[:3]
    out = []
    for prof in (False, True):
        solvers = [B.Solver(cfg, tol=1e-12) for cfg in cfgs]
        batch = B.Batch(solvers, fused=True)
        states = [sv.state() for sv in solvers]
        batch.run(states, 0, 2)
        if prof:
            batch.profile(True)
        batch.run(states, 2, 2)
        if prof:
            rec = batch.profile_read()
            batch.profile(False)
            print("fused batch profile", {k: (v["launches"], round(v["ms"], 3)) for k, v in rec.items()})
            for cls in ("tri_fwd_sub", "tri_bwd_sub", "tri_top"):
                assert rec[cls]["launches"] > 0 and rec[cls]["bytes"] > 0 and rec[cls]["ms"] > 0
        out.append([[t.cpu().numpy() for t in st] for st in states])
        batch.close()
        for sv in solvers:
            sv.close()
    for a, b in zip(out[0], out[1]):
        for x, y in zip(a, b):
            assert np.array_equal(x, y)
    solvers = [B.Solver(cfg) for cfg in cfgs[:2]]
    batch = B.Batch(solvers, n_streams=2)
    with pytest.raises(B.BidoError, match="BIDO_ERR_STATE"):
        batch.profile(True)
    batch.close()
    for sv in solvers:
        sv.close()


def test_fused_batch_strang(torch):
    """A fused batch of Strang-splitting slices follows each slice run alone."""
    import paper_1711_08708_amd as B
    cfgs = _slices()[:3]
    n_steps = 8
    ref = _single_runs(B, cfgs, B.PREC_FP64, n_steps, scheme=B.SCHEME_STRANG)
    solvers = [B.Solver(cfg, tol=1e-12, scheme=B.SCHEME_STRANG) for cfg in cfgs]
    batch = B.Batch(solvers, fused=True)
    states = [s.state() for s in solvers]
    for n in range(n_steps):
        batch.run(states, n, 1)
    for k, st in enumerate(states):
        for a, b in zip([t.cpu().numpy() for t in st], ref[k][0]):
            assert np.linalg.norm(a - b) <= 1e-9 * np.linalg.norm(b), k
    batch.close()
    for s in solvers:
        s.close()
