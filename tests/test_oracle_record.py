"""Pins of the recording oracle (activation times, probe potentials; the
recordings of the test cases of Sec. 6) and the library's host point
location against it."""
import numpy as np
import pytest

import workloads as w
from oracle import record as rc


def _inside_points(cfg, k, seed):
    """k points strictly inside random elements (random convex weights)."""
    rng = np.random.default_rng(seed)
    xyz, el = cfg["xyz"], cfg["elems"]
    e = rng.integers(0, len(el), size=k)
    lam = rng.dirichlet(np.ones(el.shape[1]), size=k)
    return np.einsum("kv,kvd->kd", lam, xyz[el[e]])


@pytest.mark.parametrize("mk", [lambda: w.thorax2d(n_target=3000, seed=11), lambda: w.slab3d(n=4)],
                         ids=["thorax3000", "slab4"])
def test_probe_of_an_affine_field_is_exact(mk):
    cfg = mk()
    xyz = cfg["xyz"]
    a = np.array([0.7, -1.3, 2.1])[:xyz.shape[1]]
    u = xyz @ a + 0.25
    pts = _inside_points(cfg, 12, 1)
    got = rc.probe_values(xyz, cfg["elems"], u, pts)
    assert np.abs(got - (pts @ a + 0.25)).max() < 1e-12


def test_probe_at_electrode_vertices():
    cfg = w.thorax2d(n_target=3000, seed=11)
    xyz = cfg["xyz"]
    u = np.random.default_rng(2).normal(size=len(xyz))
    el = cfg["electrodes"]
    assert el.shape == (6, 2)
    idx = [int(np.argmin(np.linalg.norm(xyz - p, axis=1))) for p in el]
    assert np.allclose(xyz[idx], el, rtol=0, atol=0)             # electrodes are mesh vertices
    r = np.hypot(el[:, 0] / 15.0, el[:, 1] / 10.0)
    assert np.abs(r - 1.0).max() < 1e-9                         # on the torso boundary
    got = rc.probe_values(xyz, cfg["elems"], u, el)
    assert np.abs(got - u[idx]).max() < 1e-12


def test_probe_outside_the_mesh_is_refused():
    cfg = w.square2d(n=6)
    with pytest.raises(ValueError):
        rc.locate(cfg["xyz"], cfg["elems"], np.array([-1.0, 0.5]))


def test_activation_of_linear_ramps():
    """V_i(t) = s_i t (linear in time, so the interpolation is exact): the
    activation time is v_act / s_i; a vertex that never reaches the level
    gets -1; a vertex already above it at the start gets the start time."""
    dt, t0, v_act = 0.1, 2.0, 64.0
    s = np.array([100.0, 37.0, 3.0, 640.0, 1.0])
    V = [s * (k * dt) for k in range(30)]
    V = [np.concatenate([v, [80.0]]) for v in V]                 # last vertex: above from the start
    act = rc.activation_times(V, t0, dt, v_act)
    expect = np.concatenate([t0 + v_act / s, [t0]])
    expect[2] = expect[4] = -1.0                                 # 3 * 2.9 and 1 * 2.9 stay below 64
    assert np.allclose(act, expect, rtol=1e-14, atol=1e-14)


@pytest.mark.parametrize("mk", [lambda: w.thorax2d(n_target=3000, seed=11), lambda: w.slab3d(n=4)],
                         ids=["thorax3000", "slab4"])
def test_library_probe_location_against_oracle(mk):
    """The host point location of bido_record: weights form a convex
    combination reproducing the point, affine fields are exact, and the
    values agree with the oracle's interpolant."""
    import paper_1711_08708_amd as B
    cfg = mk()
    xyz = cfg["xyz"]
    pts = _inside_points(cfg, 10, 3)
    if "electrodes" in cfg:
        pts = np.vstack([pts, cfg["electrodes"]])
    hs = B.HostSetup(cfg)
    ids, wts = hs.locate(pts)
    assert wts.min() >= -1e-9 and np.abs(wts.sum(axis=1) - 1.0).max() < 1e-12
    assert np.abs(np.einsum("kv,kvd->kd", wts, xyz[ids]) - pts).max() < 1e-12
    u = np.random.default_rng(4).normal(size=len(xyz))
    got = np.einsum("kv,kv->k", wts, u[ids])
    ref = rc.probe_values(xyz, cfg["elems"], u, pts)
    assert np.abs(got - ref).max() < 1e-12
    with pytest.raises(B.BidoError, match="outside"):
        hs.locate(np.full((1, xyz.shape[1]), 1e3))
