"""Pins for the FP64 reference of the learned correction (oracle.mpnn)."""
import numpy as np
import pytest

import workloads as w
from oracle import bidomain as bd
from oracle import mpnn


@pytest.fixture(scope="module")
def graph():
    s = bd.System(w.square2d(n=12))
    A = mpnn.aggregation_matrix(s.Sm)
    st = mpnn.static_features(s.cfg, s.Sm)
    return s, A, st


def test_aggregation_rows_are_normalised(graph):
    s, A, _ = graph
    rs = np.asarray(A.sum(axis=1)).ravel()
    np.testing.assert_allclose(rs, 1.0, rtol=1e-14)
    assert (A.diagonal() == 0).all()
    assert (A.data > 0).all()


def test_gradient_matches_central_differences(graph):
    """Backward pass of the oracle against central differences in FP64."""
    s, A, st = graph
    rng = np.random.default_rng(0)
    theta = mpnn.init_params(1)
    f, nt = mpnn.features(rng.normal(size=s.NH), st)
    y = rng.normal(size=s.NH) * 0.1
    loss, g = mpnn.loss_and_grad(theta, A, f, y)
    idx = rng.choice(mpnn.N_PARAMS, size=60, replace=False)
    h = 1e-6
    for k in idx:
        e = np.zeros_like(theta)
        e[k] = h
        lp, _ = mpnn.loss_and_grad(theta + e, A, f, y)
        lm, _ = mpnn.loss_and_grad(theta - e, A, f, y)
        fd = (lp - lm) / (2 * h)
        assert abs(fd - g[k]) <= 1e-6 * max(1.0, abs(fd)), (k, fd, g[k])


def test_energy_loss_gradient_matches_central_differences(graph):
    """Same check with the energy-norm loss r^T W r, W = K_m / mean diag."""
    s, A, st = graph
    W = mpnn.energy_weight(s.gamma * np.diag(s.mH) + s.Sm.toarray())
    rng = np.random.default_rng(4)
    theta = mpnn.init_params(2)
    f, _ = mpnn.features(rng.normal(size=s.NH), st)
    y = rng.normal(size=s.NH)
    loss, g = mpnn.loss_and_grad(theta, A, f, y, W)
    assert loss > 0
    for k in rng.choice(mpnn.N_PARAMS, size=40, replace=False):
        e = np.zeros_like(theta)
        e[k] = 1e-6
        fd = (mpnn.loss_and_grad(theta + e, A, f, y, W)[0] - mpnn.loss_and_grad(theta - e, A, f, y, W)[0]) / 2e-6
        assert abs(fd - g[k]) <= 1e-6 * max(1.0, abs(fd)), (k, fd, g[k])


def test_linear_regime_equals_composed_map(graph):
    """With non-negative weights and inputs every ReLU is active, so the
    network is the affine map o = w3.(W2s h1 + W2n A h1 + b2) + b3 with
    h1 = W1s f + W1n A f + b1, written here with Kronecker products."""
    s, A, st = graph
    rng = np.random.default_rng(2)
    p = {name: rng.uniform(0.0, 0.2, size=shape) for name, shape in mpnn.PARAM_SHAPES}
    theta = mpnn.pack(p)
    f = rng.uniform(0.0, 1.0, size=(s.NH, mpnn.F))
    o, _ = mpnn.forward(theta, A, f)
    I = np.eye(s.NH)
    Ad = A.toarray()
    L1 = np.kron(I, p["W1s"]) + np.kron(Ad, p["W1n"])          # acts on vec(f) row-major
    h1 = L1 @ f.ravel() + np.tile(p["b1"], s.NH)
    L2 = np.kron(I, p["W2s"]) + np.kron(Ad, p["W2n"])
    h2 = L2 @ h1 + np.tile(p["b2"], s.NH)
    ref = np.kron(I, p["w3"][None, :]) @ h2 + p["b3"][0]
    np.testing.assert_allclose(o, ref, rtol=1e-12)


def test_zero_network_is_its_bias(graph):
    s, A, st = graph
    p = {name: np.zeros(shape) for name, shape in mpnn.PARAM_SHAPES}
    p["b3"] = np.array([0.25])
    f, _ = mpnn.features(np.ones(s.NH), st)
    o, _ = mpnn.forward(mpnn.pack(p), A, f)
    np.testing.assert_allclose(o, 0.25)


def test_boundary_distance_feature():
    """Heart-boundary vertices have distance 0; the slab centre is farthest."""
    cfg = w.slab3d(n=4)
    s = bd.System(cfg)
    st = mpnn.static_features(cfg, s.Sm)
    dcol = 12   # 3D: 6 + 6 conductivity entries, then the distance
    b = mpnn.heart_boundary_vertices(cfg)
    assert len(b) == 5**3 - 3**3     # surface vertices of the 4^3 cube
    np.testing.assert_allclose(st[b, dcol], 0.0)
    centre = np.argmin(np.linalg.norm(cfg["xyz"] - 0.5, axis=1))
    assert st[centre, dcol] == st[:, dcol].max() == 1.0
    # conductivity features: first column is sigma_i xx / max diagonal value
    assert 0 < st[:, 0].max() <= 1.0


def test_stencil_is_symmetric_and_gradient_matches_fd(graph):
    """The learned stencil C is symmetric on the S_m pattern; the gradient of
    the regression loss matches central differences."""
    s, A, st = graph
    P = s.Sm
    f = mpnn.static_input(st)
    rng = np.random.default_rng(6)
    theta = mpnn.init_params(4)
    theta[-33:] = rng.normal(0, 0.3, 33)
    C = mpnn.stencil_matrix(theta, A, f, P).toarray()
    np.testing.assert_allclose(C, C.T, atol=1e-14)
    Pc = P.tocsr()
    stored = set(zip(np.repeat(np.arange(Pc.shape[0]), np.diff(Pc.indptr)).tolist(), Pc.indices.tolist()))
    assert set(zip(*np.nonzero(C))) <= stored     # C lives on the stored S_m pattern
    Zh = rng.normal(size=(3, s.NH))
    Bh = rng.normal(size=(3, s.NH)) * 0.1
    loss, g = mpnn.stencil_loss_and_grad(theta, A, f, P, Zh, Bh)
    for k in rng.choice(mpnn.N_PARAMS, size=50, replace=False):
        e = np.zeros_like(theta)
        e[k] = 1e-6
        fd = (mpnn.stencil_loss_and_grad(theta + e, A, f, P, Zh, Bh)[0]
              - mpnn.stencil_loss_and_grad(theta - e, A, f, P, Zh, Bh)[0]) / 2e-6
        assert abs(fd - g[k]) <= 1e-6 * max(1.0, abs(fd)), (k, fd, g[k])


def test_stencil_regression_recovers_a_known_correction():
    """If the targets come from K_m + C0 with C0 a constant multiple of the
    identity, the loss of the network that outputs that multiple is zero."""
    s = bd.System(w.square2d(n=10))
    A = mpnn.aggregation_matrix(s.Sm)
    f = mpnn.static_input(mpnn.static_features(s.cfg, s.Sm))
    p = {name: np.zeros(shape) for name, shape in mpnn.PARAM_SHAPES}
    p["b3"] = np.array([0.05])
    theta = mpnn.pack(p)
    rng = np.random.default_rng(1)
    Zh = rng.normal(size=(2, s.NH))
    Bh = 0.05 * Zh                      # C^ = 0.05 I exactly
    loss, _ = mpnn.stencil_loss_and_grad(theta, A, f, s.Sm, Zh, Bh)
    assert loss < 1e-24
