"""Changing the time step (bido_set_dt): gamma = chi cm / dt enters only the
v-v diagonal of Lambda and K_m = gamma M_H + S_m (Sec. 3.2, Sec. 5.2).  The
host update must give the same matrices as a set-up at the new step, and
the refactored K_m the same inner solve."""
import numpy as np
import pytest
import scipy.sparse as sp

import workloads as w


@pytest.mark.parametrize("scheme", [0, 1, 2], ids=["euler", "cn", "strang"])
@pytest.mark.parametrize("mk", [lambda: w.thorax2d(n_target=3000, seed=11), lambda: w.slab3d(n=6)],
                         ids=["thorax3000", "slab6"])
def test_host_set_dt_equals_setup_at_new_step(mk, scheme):
    import paper_1711_08708_amd as B
    cfg = mk()
    dt2 = 0.37 * cfg["dt"]
    a = B.HostSetup(cfg, eps_h=0.0, scheme=scheme)
    a.set_dt(dt2, refactor=True)
    b = B.HostSetup(cfg, eps_h=0.0, scheme=scheme, dt=dt2)
    for which in (B.MAT_LAMBDA, B.MAT_KM):
        x, y = a.csr(which), b.csr(which)
        assert np.array_equal(x.indptr, y.indptr) and np.array_equal(x.indices, y.indices)
        assert np.array_equal(x.data, y.data), which
    rng = np.random.default_rng(0)
    t = rng.normal(size=b.csr(B.MAT_KM).shape[0])
    za, zb = a.factor_apply(B.FACTOR_PK, t), b.factor_apply(B.FACTOR_PK, t)
    assert np.abs(za - zb).max() <= 1e-13 * np.abs(zb).max()
    # P_1 does not depend on dt
    n = a.csr(B.MAT_LAMBDA).shape[0] - len(t)
    s = rng.normal(size=n)
    assert np.array_equal(a.factor_apply(B.FACTOR_P1, s), b.factor_apply(B.FACTOR_P1, s))


def test_host_set_dt_against_oracle_lambda():
    """The updated Lambda is the oracle's Lambda at the new step (internal
    order mapped back), gamma included."""
    import paper_1711_08708_amd as B
    from oracle import bidomain as bd
    cfg = w.thorax2d(n_target=3000, seed=11)
    dt2 = 0.05
    h = B.HostSetup(cfg)
    h.set_dt(dt2, refactor=False)
    s = bd.System(cfg, dt=dt2)
    L = h.csr(B.MAT_LAMBDA)
    upos, vpos = h.index(B.IDX_UPOS), h.index(B.IDX_VPOS)
    # oracle order: heart-first u (s.perm), then heart-local v
    perm_u = upos[s.perm]
    idx = np.concatenate([perm_u, s.N + vpos])
    P = sp.csr_matrix((np.ones(len(idx)), (np.arange(len(idx)), idx)), shape=L.shape)
    Lo = P @ L @ P.T
    assert abs(Lo - s.Lam).max() <= 1e-12 * abs(s.Lam).max()


def test_host_set_dt_rejects_bad_steps():
    import paper_1711_08708_amd as B
    h = B.HostSetup(w.square2d(n=6))
    for dt in (0.0, -1.0, float("nan"), float("inf")):
        with pytest.raises(B.BidoError):
            h.set_dt(dt)
