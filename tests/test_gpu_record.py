"""GPU recordings of a run (the activation maps and ECG of the test cases of
Sec. 6): activation times fused into the write-back of V^{n+1} and the
potential u at probe points after every step, against the oracle."""
import numpy as np
import pytest

import workloads as w

pytestmark = pytest.mark.gpu

V_ACT = 64.0          # mV above rest


@pytest.fixture(scope="module")
def torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _probe_points(cfg):
    rng = np.random.default_rng(9)
    el = cfg["elems"][rng.integers(0, len(cfg["elems"]), size=4)]
    inner = cfg["xyz"][el].mean(axis=1)
    return np.vstack([cfg["electrodes"], inner])


@pytest.mark.parametrize("v_act", [V_ACT, 0.5])
def test_activation_and_ecg_against_oracle(torch, v_act):
    """40 steps of a thorax slice (2 ms stimulus, dt 0.1 ms) recording
    activation at v_act mV above rest (64: the upstroke, reached by the
    stimulated vertices; 0.5: the foot of the wave, reached by many) and u
    at the six electrodes plus four interior points:
      - the probe rows equal the oracle's P1 interpolant of each step's u,
        and match the oracle's own step from the same state within 1e-8;
      - the activation times equal the oracle's activation of the recorded
        potentials, and some vertices are reached, others not."""
    import paper_1711_08708_amd as B
    from oracle import bidomain as bd
    from oracle import record as rc
    cfg = w.thorax2d(n_target=3000, seed=11)
    s = bd.System(cfg)
    pts = _probe_points(cfg)
    K = 40
    solver = B.Solver(cfg, eps_h=0.0, tol=1e-12)
    solver.record(v_act, pts, max_steps=K)
    v, h, u = solver.state()
    Vs = [v.cpu().numpy().copy()]
    Us = []
    worst = 0.0
    for n in range(K):
        Vn, hn = v.cpu().numpy().copy(), h.cpu().numpy().copy()
        assert solver.step(v, h, u, n)["converged"] == 1
        Vs.append(v.cpu().numpy().copy())
        Us.append(u.cpu().numpy().copy())
        if n % 10 == 9:
            Uo_p, _, _ = s.step(Vn, hn, n)
            Uo = s.to_global_u(Uo_p)
            po = rc.probe_values(cfg["xyz"], cfg["elems"], Uo, pts)
            pg = rc.probe_values(cfg["xyz"], cfg["elems"], Us[-1], pts)
            err = np.abs(po - pg).max() / np.abs(Uo).max()
            worst = max(worst, err)
            assert err <= 1e-8, (n, err)
    act, rows = solver.record_read()
    assert rows.shape == (K, len(pts))
    ref_rows = np.array([rc.probe_values(cfg["xyz"], cfg["elems"], uk, pts) for uk in Us])
    scale = np.abs(ref_rows).max()
    assert np.abs(rows - ref_rows).max() <= 1e-12 * scale
    ref_act = rc.activation_times(Vs, 0.0, cfg["dt"], v_act)
    reached = ref_act >= 0
    print(f"activated {reached.sum()} of {len(ref_act)} heart vertices by t = {K * cfg['dt']} ms; "
          f"ECG worst vs oracle step {worst:.2e}; electrode u at the end {rows[-1, :6]}")
    assert 0 < reached.sum() < len(ref_act)
    if v_act < 1.0:
        assert reached.sum() > 10
    assert np.array_equal(act >= 0, reached)
    assert np.abs(act[reached] - ref_act[reached]).max() <= 1e-12 * K * cfg["dt"]
    assert (act[reached] <= K * cfg["dt"]).all()
    # rows stop at max_steps; a new recording starts over
    solver.step(v, h, u, K)
    assert solver.record_read()[1].shape == (K, len(pts))
    solver.record(float("nan"), pts[:2], max_steps=3)
    solver.step(v, h, u, K + 1)
    act2, rows2 = solver.record_read()
    assert act2 is None and rows2.shape == (1, 2)
    solver.close()


def test_recording_in_a_fused_batch(torch):
    """Recordings started before a fused batch keep running inside it and
    follow each slice run alone (up to the batch's rounding order)."""
    import paper_1711_08708_amd as B
    cfgs = [w.thorax2d(n_target=3000, seed=11), w.thorax2d(n_target=2000, seed=5)]
    K = 12
    alone = []
    for cfg in cfgs:
        sv = B.Solver(cfg, tol=1e-12)
        sv.record(V_ACT, cfg["electrodes"], max_steps=K)
        v, h, u = sv.state()
        for n in range(K):
            sv.step(v, h, u, n)
        alone.append(sv.record_read())
        sv.close()
    solvers = [B.Solver(cfg, tol=1e-12) for cfg in cfgs]
    for sv, cfg in zip(solvers, cfgs):
        sv.record(V_ACT, cfg["electrodes"], max_steps=K)
    batch = B.Batch(solvers, fused=True)
    with pytest.raises(B.BidoError, match="BIDO_ERR_STATE"):
        solvers[0].record(V_ACT, cfgs[0]["electrodes"], max_steps=K)
    states = [sv.state() for sv in solvers]
    for n in range(K):
        batch.run(states, n, 1)
    batch.close()
    for sv, (act_a, rows_a) in zip(solvers, alone):
        act, rows = sv.record_read()
        assert rows.shape == rows_a.shape
        assert np.abs(rows - rows_a).max() <= 1e-9 * np.abs(rows_a).max()
        both = (act >= 0) & (act_a >= 0)
        assert np.array_equal(act >= 0, act_a >= 0)
        assert np.abs(act[both] - act_a[both]).max() <= 1e-6
        sv.close()


def test_record_arguments(torch):
    import paper_1711_08708_amd as B
    cfg = w.thorax2d(n_target=2000, seed=5)
    sv = B.Solver(cfg)
    with pytest.raises(B.BidoError, match="BIDO_ERR_ARG"):
        sv.record(V_ACT, np.array([[1e3, 0.0]]), max_steps=4)
    with pytest.raises(B.BidoError, match="BIDO_ERR_ARG"):
        sv.record(float("inf"), None, 0)
    with pytest.raises(B.BidoError, match="BIDO_ERR_ARG"):
        sv.record(V_ACT, cfg["electrodes"], max_steps=0)
    sv.record(float("nan"), cfg["electrodes"], max_steps=2)
    import ctypes
    buf = (ctypes.c_double * sv.NH)()
    with pytest.raises(B.BidoError, match="BIDO_ERR_STATE"):
        B._check(B.lib.bido_record_read(sv.ctx, buf, None, None))
    sv.close()
