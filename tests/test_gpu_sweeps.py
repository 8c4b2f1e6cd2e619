"""GPU triangular sweeps against the host application of the same factor.

The inner solves P_1^-1 and P_K^-1 (Sec. 5.3) run as device sweeps over an
execution plan (subtree phase + level phases); the host applies the same
stored factor node by node in post-order.  Both must agree to rounding."""
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


CASES = {
    "square5": lambda: w.square2d(n=5),
    "square48": lambda: w.square2d(n=48),
    "slab6": lambda: w.slab3d(n=6),
    "slab10": lambda: w.slab3d(n=10),
    "slab16": lambda: w.slab3d(n=16),
    "thorax3000": lambda: w.thorax2d(n_target=3000, seed=11),
    "thorax40k": lambda: w.thorax2d(n_target=40000, seed=12),
}


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("which", [0, 1])
def test_inner_solve_matches_host(torch, name, which):
    import paper_1711_08708_amd as B
    cfg = CASES[name]()
    hs = B.HostSetup(cfg, eps_h=0.0)
    solver = B.Solver(cfg, eps_h=0.0)
    n = solver.N if which == 0 else solver.NH
    rng = np.random.default_rng(1)
    b = rng.normal(size=n)
    ref = hs.factor_apply(which, b)
    bd = torch.tensor(b, device="cuda")
    xd = torch.full((n,), float("nan"), dtype=torch.float64, device="cuda")
    print(f"{name} factor {which}: plan {hs.factor_plan(which)}", flush=True)
    solver.inner_solve(which, bd, xd)
    x = xd.cpu().numpy()
    err = np.abs(x - ref).max() / np.abs(ref).max()
    print(f"  max rel diff {err:.2e}", flush=True)
    assert np.isfinite(x).all()
    assert err < 1e-12


@pytest.mark.parametrize("name", ["thorax40k", "slab10", "square48"])
@pytest.mark.parametrize("which", [0, 1])
def test_dense_top_at_lowest_cut(torch, name, which):
    """The dense top forced down to the lowest cut it can take (every level
    phase replaced, or as many as fit the top-size bound) still reproduces
    the host factor on the device."""
    import paper_1711_08708_amd as B
    cfg = CASES[name]()
    hs = B.HostSetup(cfg, eps_h=0.0)
    hc = hs.factor_plan(which)["hc"]
    H = hs.factor_stats(which)["height"]
    hs.set_plan(which, top_h=hc + 1)               # raised to the lowest admissible cut
    top = hs.factor_top(which)
    cut = top["top_h"]
    if cut > H:
        pytest.skip("no admissible dense top")
    print(f"{name} factor {which}: cut {cut} (hc {hc}, height {H}), n_top {top['n_top']}", flush=True)
    solver = B.Solver(cfg, eps_h=0.0)
    solver.set_plan(which, top_h=hc + 1)     # the same forced cut on the device
    assert solver.get_plan(which)["top_h"] == cut
    n = solver.N if which == 0 else solver.NH
    b = np.random.default_rng(2).normal(size=n)
    ref = hs.factor_apply(which, b)
    xd = torch.full((n,), float("nan"), dtype=torch.float64, device="cuda")
    solver.inner_solve(which, torch.tensor(b, device="cuda"), xd)
    x = xd.cpu().numpy()
    err = np.abs(x - ref).max() / np.abs(ref).max()
    print(f"  max rel diff {err:.2e}", flush=True)
    assert np.isfinite(x).all() and err < 1e-12


@pytest.mark.parametrize("name", ["thorax40k", "slab10"])
@pytest.mark.parametrize("eps", [1e-10, 1e-4])
def test_hierarchical_top_matches_emulation(torch, name, eps):
    """With eps_h > 0 the top inverse is applied in hierarchical low-rank
    form; the device application equals the CPU emulation of the same plan
    to rounding, and stays within about eps of the exact factor."""
    import paper_1711_08708_amd as B
    cfg = CASES[name]()
    hs = B.HostSetup(cfg, eps_h=eps)
    solver = B.Solver(cfg, eps_h=eps)
    for which in (0, 1):                      # lowest admissible cut: the largest top
        hs.set_plan(which, top_h=0)
        solver.set_plan(which, top_h=0)
    for which in (0, 1):
        n = solver.N if which == 0 else solver.NH
        b = np.random.default_rng(4 + which).normal(size=n)
        emu = hs.factor_emulate(which, b)
        exact = hs.factor_apply(which, b)
        xd = torch.full((n,), float("nan"), dtype=torch.float64, device="cuda")
        solver.inner_solve(which, torch.tensor(b, device="cuda"), xd)
        x = xd.cpu().numpy()
        e_emu = np.abs(x - emu).max() / np.abs(emu).max()
        e_ex = np.linalg.norm(x - exact) / np.linalg.norm(exact)
        print(f"{name} eps {eps:.0e} factor {which}: top {hs.factor_top(which)}, vs emulation {e_emu:.2e}, "
              f"vs exact {e_ex:.2e}", flush=True)
        assert np.isfinite(x).all() and e_emu < 1e-12
        assert e_ex <= 1e3 * eps + 1e-12


def test_autotune_keeps_the_factor(torch):
    """The autotuner times candidate plans on the device and keeps the
    fastest; the inner solves still reproduce the host factor."""
    import paper_1711_08708_amd as B
    cfg = CASES["thorax40k"]()
    hs = B.HostSetup(cfg, eps_h=0.0)
    solver = B.Solver(cfg, eps_h=0.0)
    rep = solver.autotune(reps=3)
    print("autotune:", rep, flush=True)
    assert rep["candidates"] > 0
    assert all(a <= b * 1.05 for a, b in zip(rep["us_after"], rep["us_before"]))
    for which in (0, 1):
        n = solver.N if which == 0 else solver.NH
        b = np.random.default_rng(6 + which).normal(size=n)
        ref = hs.factor_apply(which, b)
        xd = torch.full((n,), float("nan"), dtype=torch.float64, device="cuda")
        solver.inner_solve(which, torch.tensor(b, device="cuda"), xd)
        x = xd.cpu().numpy()
        assert np.isfinite(x).all() and np.abs(x - ref).max() / np.abs(ref).max() < 1e-12
