"""The allocation-free inner solve (bido_inner_solve_noalloc) against the
inner solve on the context's own buffers.

Both run the same sweep kernels in the same order, so the results must be
bit-identical.  The fixed workspace is shared by every call on the GPU and
keeps the last call's contents: each case makes two calls in a row on
different contexts, the second on a smaller problem, and checks both."""
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


def _apply_pair(torch, solver, which, seed, noalloc):
    n = solver.N if which == 0 else solver.NH
    b = torch.tensor(np.random.default_rng(seed).normal(size=n), device="cuda")
    x = torch.full((n,), float("nan"), dtype=torch.float64, device="cuda")
    if noalloc:
        need = solver.inner_solve_noalloc(which, b, x)
        assert 0 < need <= (8 << 20)
    else:
        solver.inner_solve(which, b, x)
    return x


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("which", [0, 1])
@pytest.mark.parametrize("eps_h", [0.0, 1e-6])
def test_noalloc_equals_inner_solve(torch, precision, which, eps_h):
    import paper_1711_08708_amd as B
    big = B.Solver(w.thorax2d(n_target=20000, seed=21), eps_h=eps_h, precision=precision)
    small = B.Solver(w.square2d(n=24), eps_h=eps_h, precision=precision)
    print(f"noalloc: precision {precision} factor {which} eps_h {eps_h}: "
          f"N {big.N} then {small.N}", flush=True)
    refs = [_apply_pair(torch, s, which, 7, False) for s in (big, small)]
    outs = [_apply_pair(torch, s, which, 7, True) for s in (big, small)]   # big, then smaller
    torch.cuda.synchronize()
    for r, o in zip(refs, outs):
        assert torch.isfinite(r).all()
        assert torch.equal(r, o)
    # the big one again after the small one left its contents behind
    again = _apply_pair(torch, big, which, 7, True)
    assert torch.equal(refs[0], again)


def test_noalloc_chebyshev_pk(torch):
    import paper_1711_08708_amd as B
    big = B.Solver(w.thorax2d(n_target=20000, seed=21))
    small = B.Solver(w.slab3d(n=6))
    for s in (big, small):
        s.set_pk(B.PK_CHEBYSHEV, steps=3)
    print("noalloc: Chebyshev P_K", flush=True)
    refs = [_apply_pair(torch, s, 1, 3, False) for s in (big, small)]
    outs = [_apply_pair(torch, s, 1, 3, True) for s in (big, small)]
    for r, o in zip(refs, outs):
        assert torch.equal(r, o)
