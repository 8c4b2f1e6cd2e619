"""CPU checks of the C ABI library: it loads, exports every declared symbol,
and its host set-up (assembly, orderings, factors) agrees with the oracle."""
import ctypes
import os
import re

import numpy as np
import pytest

import workloads as w

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    names = set()
    for h in ("bido.h", "bido_host.h"):
        txt = open(os.path.join(ROOT, "include", h)).read()
        txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
        for m in re.finditer(r"\b(bido_\w+)\s*\(", txt):
            names.add(m.group(1))
    return sorted(names)


def test_library_exports_every_declared_symbol():
    import paper_1711_08708_amd as B
    names = _declared_functions()
    assert "bido_create" in names and "bido_solve" in names
    missing = [n for n in names if not hasattr(B.lib, n)]
    assert not missing, missing
    for n in names:
        assert n in B.ABI, f"binding does not wrap {n}"


def test_struct_sizes_match_header():
    import paper_1711_08708_amd as B
    # bido_params: 6 doubles + 11 ints (+ 4 bytes of tail padding); bido_stats:
    # 2 ints, 2 doubles, int, double, int64
    assert ctypes.sizeof(B.Params) == 6 * 8 + 11 * 4 + 4
    assert B.default_params().scheme == B.SCHEME_EULER
    assert ctypes.sizeof(B.Stats) == 48
    p = B.default_params()
    assert p.leaf == 64 and p.max_iter == 200 and p.tol == 1e-10


def test_create_without_gpu_reports_device_error():
    import torch
    import paper_1711_08708_amd as B
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    cfg = w.square2d(n=6)
    mesh, tissue, keep = B._marshal(cfg)
    p = B.make_params(cfg)
    ctx = ctypes.c_void_p()
    code = B.lib.bido_create(ctypes.byref(mesh), ctypes.byref(tissue), ctypes.byref(p), None,
                             ctypes.byref(ctx))
    assert code == -2 and not ctx.value


@pytest.mark.parametrize("mk", [lambda: w.square2d(n=20), lambda: w.slab3d(n=5),
                                lambda: w.thorax2d(n_target=4000, seed=9)])
def test_host_assembly_matches_oracle(mk):
    import paper_1711_08708_amd as B
    from oracle import fem
    cfg = mk()
    hs = B.HostSetup(cfg, eps_h=0.0)
    A = fem.assemble(cfg)
    for which, ref in ((B.MAT_S1, A["S1"]), (B.MAT_SI, A["Si"]), (B.MAT_SM, A["Sm"])):
        M = hs.csr(which)
        assert abs(M - ref).max() <= 1e-13 * abs(ref).max()
    np.testing.assert_allclose(hs.vec(B.VEC_M), A["m"], rtol=1e-13)
    np.testing.assert_allclose(hs.vec(B.VEC_MH), A["mH"], rtol=1e-13)
    assert np.array_equal(hs.index(B.IDX_HEART), A["hn"])


def test_host_lambda_is_the_oracle_lambda_reordered():
    import paper_1711_08708_amd as B
    from oracle import bidomain as bd
    cfg = w.square2d(n=16)
    hs = B.HostSetup(cfg, eps_h=0.0)
    s = bd.System(cfg)
    upos, vpos = hs.index(B.IDX_UPOS), hs.index(B.IDX_VPOS)
    N, NH = s.N, s.NH
    assert sorted(upos.tolist()) == list(range(N)) and sorted(vpos.tolist()) == list(range(NH))
    o2i = np.concatenate([upos[s.perm], N + vpos])
    P = np.empty(N + NH, dtype=np.int64)
    P[o2i] = np.arange(N + NH)
    L = hs.csr(B.MAT_LAMBDA)
    Lo = s.Lam[P][:, P]
    assert abs(L - Lo).max() <= 1e-13 * abs(Lo).max()


def _blocked_product(b, x):
    """(Lambda x) from the blocked form: u rows then v rows."""
    n = len(b["gm"])
    xu, xv = x[:n], x[n:]
    rows = np.repeat(np.arange(n), np.diff(b["ptr"]))
    c = b["col"]
    yu = np.bincount(rows, b["val"][:, 0] * xu[c] + b["val"][:, 1] * xv[c], minlength=n)
    yv = np.bincount(rows, b["val"][:, 1] * (xu[c] + xv[c]), minlength=n) + b["gm"] * xv
    return np.concatenate([yu, yv])


def test_blocked_lambda_is_the_oracle_lambda():
    """A slab (heart = whole mesh, one order for u and v) has Lambda's blocked
    form; its product equals the oracle's Lambda (reordered) times x, also
    after a change of time step; a mesh with torso rows has none."""
    import paper_1711_08708_amd as B
    from oracle import bidomain as bd
    cfg = w.slab3d(n=7)
    hs = B.HostSetup(cfg, eps_h=0.0)
    b = hs.lambda_blocked()
    assert b is not None
    s = bd.System(cfg)
    upos, vpos = hs.index(B.IDX_UPOS), hs.index(B.IDX_VPOS)
    N, NH = s.N, s.NH
    assert np.array_equal(upos[s.perm], vpos)      # one order for u and v
    o2i = np.concatenate([upos[s.perm], N + vpos])
    P = np.empty(N + NH, dtype=np.int64)
    P[o2i] = np.arange(N + NH)
    Lo = s.Lam[P][:, P]
    x = np.random.default_rng(3).normal(size=N + NH)
    y = Lo @ x
    assert np.abs(_blocked_product(b, x) - y).max() <= 1e-13 * np.abs(y).max()
    # 20 bytes per position against 12 per entry of the four CSR blocks
    assert 20 * len(b["col"]) < 12 * hs.csr(B.MAT_LAMBDA).nnz
    hs.set_dt(0.05)
    b2 = hs.lambda_blocked()
    L2 = hs.csr(B.MAT_LAMBDA)
    assert np.abs(_blocked_product(b2, x) - L2 @ x).max() <= 1e-13 * np.abs(L2 @ x).max()
    assert np.allclose(b2["gm"], 2.0 * b["gm"], rtol=1e-12)   # gamma ~ 1/dt
    assert B.HostSetup(w.square2d(n=12), eps_h=0.0).lambda_blocked() is None


@pytest.mark.parametrize("mk", [lambda: w.square2d(n=30), lambda: w.slab3d(n=7),
                                lambda: w.thorax2d(n_target=6000, seed=4)])
def test_exact_factors_invert_the_inner_matrices(mk):
    """With eps = 0 the factors are exact Cholesky factors: P_1 is the
    grounded inverse of S_1 (entry N-1 fixed to zero), P_K inverts K_m."""
    import paper_1711_08708_amd as B
    from oracle import fem
    cfg = mk()
    hs = B.HostSetup(cfg, eps_h=0.0, leaf=16)
    A = fem.assemble(cfg)
    upos, vpos = hs.index(B.IDX_UPOS), hs.index(B.IDX_VPOS)
    iu, iv = np.argsort(upos), np.argsort(vpos)
    S1 = A["S1"][iu][:, iu]
    gamma = cfg["chi"] * cfg["cm"] / cfg["dt"]
    import scipy.sparse as sp
    Km = (A["Sm"] + gamma * sp.diags(A["mH"]))[iv][:, iv]
    rng = np.random.default_rng(0)
    x = rng.normal(size=S1.shape[0])
    x[-1] = 0.0
    y = hs.factor_apply(B.FACTOR_P1, S1 @ x)
    assert np.linalg.norm(y - x) <= 1e-9 * np.linalg.norm(x)
    xk = rng.normal(size=Km.shape[0])
    yk = hs.factor_apply(B.FACTOR_PK, Km @ xk)
    assert np.linalg.norm(yk - xk) <= 1e-11 * np.linalg.norm(xk)
    st = hs.factor_stats(B.FACTOR_P1)
    nodes = hs.factor_nodes(B.FACTOR_P1)
    nI, nB = nodes[:, 0].astype(np.int64), nodes[:, 1].astype(np.int64)
    assert st["entries"] == int((nI * (nI + 1) // 2 + nI * nB).sum())
    assert nI.sum() == S1.shape[0] and st["max_sep"] == nI.max()


def test_bad_inputs_are_rejected():
    import paper_1711_08708_amd as B
    cfg = w.square2d(n=6)
    bad = dict(cfg)
    bad["elems"] = cfg["elems"].copy()
    bad["elems"][0, 0] = 10**6
    with pytest.raises(B.BidoError) as e:
        B.HostSetup(bad)
    assert e.value.code == -1
    with pytest.raises(B.BidoError):
        B.HostSetup(cfg, dt=-1.0)
    no_heart = dict(cfg)
    no_heart["region"] = np.zeros_like(cfg["region"])
    with pytest.raises(B.BidoError):
        B.HostSetup(no_heart)


@pytest.mark.parametrize("mk", [lambda: w.thorax2d(n_target=3000, seed=2), lambda: w.slab3d(n=10),
                                lambda: w.square2d(n=48)], ids=["thorax3000", "slab10", "square48"])
def test_dense_top_at_every_cut(mk):
    """Forcing the dense top at every possible cut height (down to the
    lowest level above the subtree phase) leaves the sweep result unchanged:
    S_top^-1 is the inverse of the Schur complement of the top vertices."""
    import paper_1711_08708_amd as B
    cfg = mk()
    hs = B.HostSetup(cfg, eps_h=0.0)
    for which, idx in ((B.FACTOR_P1, B.IDX_UPOS), (B.FACTOR_PK, B.IDX_VPOS)):
        n = len(hs.index(idx))
        b = np.random.default_rng(3 + which).normal(size=n)
        ref = hs.factor_apply(which, b)
        hc = hs.factor_plan(which)["hc"]
        H = hs.factor_stats(which)["height"]
        cuts = []
        for th in range(hc + 1, H + 2):
            hs.set_plan(which, top_h=th)
            top = hs.factor_top(which)
            if top["top_h"] != th:               # raised to fit the top-size bound
                continue
            emu = hs.factor_emulate(which, b)
            assert np.isfinite(emu).all()
            assert np.abs(emu - ref).max() <= 1e-12 * np.abs(ref).max(), (which, th)
            cuts.append((th, top["n_top"]))
        print(which, "hc", hc, "height", H, "cuts (top_h, n_top)", cuts)
        assert cuts[-1][1] == 0 and (len(cuts) == 1 or cuts[0][1] > 0)


@pytest.mark.parametrize("mk", [lambda: w.square2d(n=48), lambda: w.slab3d(n=12),
                                lambda: w.thorax2d(n_target=40000, seed=12)])
def test_device_plan_emulation_matches_host_factor(mk):
    """The device execution plan of each factor (subtree phase, level phases
    with split tiles) run by a bounds-checked CPU emulation of the sweep
    kernels reproduces the host application of the same factor."""
    import paper_1711_08708_amd as B
    cfg = mk()
    hs = B.HostSetup(cfg, eps_h=0.0)
    for which, idx in ((B.FACTOR_P1, B.IDX_UPOS), (B.FACTOR_PK, B.IDX_VPOS)):
        n = len(hs.index(idx))
        b = np.random.default_rng(which).normal(size=n)
        ref = hs.factor_apply(which, b)
        emu = hs.factor_emulate(which, b)
        assert np.isfinite(emu).all()
        assert np.abs(emu - ref).max() <= 1e-13 * np.abs(ref).max()


@pytest.mark.parametrize("mk", [lambda: w.thorax2d(n_target=6000, seed=3), lambda: w.slab3d(n=12)],
                         ids=["thorax6000", "slab12"])
def test_hierarchical_top_accuracy(mk):
    """With eps_h > 0 the inverse of the top separators' Schur complement is
    held in hierarchical low-rank form (Sec. 5.3).  The emulated inner solve
    then differs from the exact factor by an amount that shrinks with eps,
    and the storage shrinks as eps grows."""
    import paper_1711_08708_amd as B
    cfg = mk()
    exact = B.HostSetup(cfg, eps_h=0.0)
    exact.set_plan(B.FACTOR_P1, top_h=0)              # lowest admissible cut: largest top
    n = len(exact.index(B.IDX_UPOS))
    b = np.random.default_rng(9).normal(size=n)
    ref = exact.factor_apply(B.FACTOR_P1, b)
    dense = exact.factor_top(B.FACTOR_P1)
    rows = []
    for eps in (1e-12, 1e-8, 1e-5, 1e-3):
        hs = B.HostSetup(cfg, eps_h=eps)
        hs.set_plan(B.FACTOR_P1, top_h=0)
        top = hs.factor_top(B.FACTOR_P1)
        emu = hs.factor_emulate(B.FACTOR_P1, b)
        err = np.linalg.norm(emu - ref) / np.linalg.norm(ref)
        rows.append((eps, err, top["stored_entries"], top["max_rank"]))
    print("n_top", dense["n_top"], "dense entries", dense["stored_entries"])
    for r in rows:
        print("  eps %.0e  rel err %.2e  stored %d  max rank %d" % r)
    assert rows[0][1] < 1e-9
    for (e0, r0, s0, _), (e1, r1, s1, _) in zip(rows, rows[1:]):
        assert r1 >= r0 * 0.5 and s1 <= s0
    assert rows[-1][2] < dense["stored_entries"]
    for eps, err, _, _ in rows:
        assert err <= 1e3 * eps + 1e-12


def test_hierarchical_top_is_compressed():
    """At eps_h = 1e-6 the hierarchical top stores fewer values than the
    dense inverse, with low-rank blocks of positive rank."""
    import paper_1711_08708_amd as B
    cfg = w.thorax2d(n_target=6000, seed=3)
    hs = B.HostSetup(cfg, eps_h=1e-6)
    top = hs.factor_top(B.FACTOR_P1)
    assert top["max_rank"] > 0
    assert top["stored_entries"] < top["n_top"] ** 2


@pytest.mark.parametrize("eps", [0.0, 1e-6])
def test_forest_of_slices_emulates_each_slice(eps):
    """The factor of a batch of independent slices is the forest of their
    factors; its device plan (one subtree phase, merged level phases, one
    hierarchical top per tree) run by the CPU emulation gives, on every
    slice's range, that slice's own inner solve (exact, or within about eps
    for the hierarchical tops)."""
    import paper_1711_08708_amd as B
    cfgs = [w.thorax2d(n_target=3000, seed=31), w.thorax2d(n_target=6000, seed=32, sigma_scale=0.8),
            w.square2d(n=24, seed=3), w.thorax2d(n_target=1500, seed=33)]
    parts = [B.HostSetup(c, eps_h=eps) for c in cfgs]
    merged = B.HostSetup.merged(parts)
    sizes = [(len(p.index(B.IDX_UPOS)), len(p.index(B.IDX_VPOS))) for p in parts]
    ntot = sum(a + b for a, b in sizes)
    rng = np.random.default_rng(12)
    for which in (B.FACTOR_P1, B.FACTOR_PK):
        b = rng.normal(size=ntot)
        emu = merged.factor_emulate(which, b)
        print("forest plan", which, merged.factor_plan(which), merged.factor_top(which))
        off = 0
        for p, (N, NH) in zip(parts, sizes):
            lo, n = (off, N) if which == B.FACTOR_P1 else (off + N, NH)
            ref = p.factor_apply(which, b[lo:lo + n])
            err = np.abs(emu[lo:lo + n] - ref).max() / np.abs(ref).max()
            assert np.isfinite(emu[lo:lo + n]).all()
            assert err <= 1e-11 + 1e3 * eps, (which, err)
            off += N + NH


def test_forest_takes_over_each_slice_hierarchical_top():
    """A merged tree whose slice already built its hierarchical top at the
    same cut reuses it (no second inversion: zero host seconds for the
    forest's tops) and then sweeps exactly like that slice's own plan."""
    import paper_1711_08708_amd as B
    eps = 1e-6
    cfgs = [w.thorax2d(n_target=3000, seed=31), w.thorax2d(n_target=6000, seed=32, sigma_scale=0.8),
            w.thorax2d(n_target=1500, seed=33)]
    parts = [B.HostSetup(c, eps_h=eps) for c in cfgs]
    sizes = [(len(p.index(B.IDX_UPOS)), len(p.index(B.IDX_VPOS))) for p in parts]
    ntot = sum(a + b for a, b in sizes)
    rng = np.random.default_rng(5)
    for which in (B.FACTOR_P1, B.FACTOR_PK):
        b = rng.normal(size=ntot)
        refs, off = [], 0
        for p, (N, NH) in zip(parts, sizes):
            lo, n = (off, N) if which == B.FACTOR_P1 else (off + N, NH)
            refs.append((lo, n, p.factor_emulate(which, b[lo:lo + n])))   # builds the slice's top
            off += N + NH
        merged = B.HostSetup.merged(parts)
        top = merged.factor_top(which)
        assert top["n_top"] > 0 and top["seconds"] == 0.0, top
        emu = merged.factor_emulate(which, b)
        for lo, n, ref in refs:
            err = np.abs(emu[lo:lo + n] - ref).max() / np.abs(ref).max()
            assert err <= 1e-13, (which, err)


def test_hierarchical_top_with_a_decoupled_block():
    """The heart of this slice falls into two parts, so the inverse of its
    top Schur complement has an off-diagonal block that is zero up to
    rounding (entries near 1e-162).  Truncation relative to that block alone
    would keep a full-rank basis of underflowing noise (NaN in the sweep);
    the block must get rank 0 and the sweep stay accurate."""
    import paper_1711_08708_amd as B
    cfg = w.thorax2d(n_target=32084, seed=1007, sigma_scale=0.7472320903063928)
    hs = B.HostSetup(cfg, eps_h=1e-8)
    n = len(hs.index(B.IDX_VPOS))
    b = np.random.default_rng(7).normal(size=n)
    ref = hs.factor_apply(B.FACTOR_PK, b)
    emu = hs.factor_emulate(B.FACTOR_PK, b)
    top = hs.factor_top(B.FACTOR_PK)
    print("top", top)
    assert np.isfinite(emu).all()
    assert np.abs(emu - ref).max() <= 1e-6 * np.abs(ref).max()
    assert top["stored_entries"] < top["n_top"] ** 2 // 4


@pytest.mark.parametrize("sub_h", ["0", "1", "2"])
def test_capped_subtree_cut_emulates_each_slice(sub_h):
    """Capping every tree's subtree cut (more of the sweep in level phases,
    tops chosen again where a tree had none) leaves the forest an exact
    solve of every slice (eps_h = 0: tops exact up to rounding)."""
    import paper_1711_08708_amd as B
    cfgs = [w.thorax2d(n_target=3000, seed=31), w.thorax2d(n_target=6000, seed=32, sigma_scale=0.8),
            w.square2d(n=24, seed=3)]
    parts = [B.HostSetup(c, eps_h=0.0) for c in cfgs]
    sizes = [(len(p.index(B.IDX_UPOS)), len(p.index(B.IDX_VPOS))) for p in parts]
    ntot = sum(a + b for a, b in sizes)
    rng = np.random.default_rng(11)
    for which in (B.FACTOR_P1, B.FACTOR_PK):
        b = rng.normal(size=ntot)
        refs, off = [], 0
        for p, (N, NH) in zip(parts, sizes):
            lo, n = (off, N) if which == B.FACTOR_P1 else (off + N, NH)
            refs.append((lo, n, p.factor_apply(which, b[lo:lo + n])))
            off += N + NH
        merged = B.HostSetup.merged(parts)
        merged.set_plan(which, sub_h=int(sub_h))
        plan = merged.factor_plan(which)
        emu = merged.factor_emulate(which, b)
        assert plan["hc"] <= int(sub_h)
        for lo, n, ref in refs:
            assert np.abs(emu[lo:lo + n] - ref).max() <= 1e-11 * np.abs(ref).max()


@pytest.mark.parametrize("total", ["4", "64"])
def test_forest_with_shared_subtree_budget(total):
    """A forest that shares a subtree budget over its trees (bigger subtrees
    per tree, cuts kept below the trees' top cuts) is still an exact solve of
    every slice (eps_h = 0)."""
    import paper_1711_08708_amd as B
    cfgs = [w.thorax2d(n_target=3000, seed=31), w.thorax2d(n_target=6000, seed=32, sigma_scale=0.8),
            w.square2d(n=24, seed=3), w.thorax2d(n_target=1500, seed=33)]
    parts = [B.HostSetup(c, eps_h=0.0) for c in cfgs]
    sizes = [(len(p.index(B.IDX_UPOS)), len(p.index(B.IDX_VPOS))) for p in parts]
    ntot = sum(a + b for a, b in sizes)
    rng = np.random.default_rng(21)
    for which in (B.FACTOR_P1, B.FACTOR_PK):
        b = rng.normal(size=ntot)
        refs, off = [], 0
        for p, (N, NH) in zip(parts, sizes):
            lo, n = (off, N) if which == B.FACTOR_P1 else (off + N, NH)
            p.factor_emulate(which, b[lo:lo + n])           # records the slice's top cut
            refs.append((lo, n, p.factor_apply(which, b[lo:lo + n])))
            off += N + NH
        merged = B.HostSetup.merged(parts)
        merged.set_plan(which, sub_total=int(total))
        plan = merged.factor_plan(which)
        top = merged.factor_top(which)
        emu = merged.factor_emulate(which, b)
        print(which, total, plan, top)
        for lo, n, ref in refs:
            assert np.abs(emu[lo:lo + n] - ref).max() <= 1e-11 * np.abs(ref).max()


def test_tall_backward_tiles_are_split_and_still_exact():
    """3D separators give level tiles of thousands of rows; the default plan
    cuts them into row ranges (with a combine step) when a level would
    otherwise have too few work items, and the host emulation of that plan
    still reproduces the factor."""
    import paper_1711_08708_amd as B
    cfg = w.slab3d(n=40)
    items = {}
    h = B.HostSetup(cfg, eps_h=0.0)
    for want in (512, 0):
        h.set_plan(B.FACTOR_P1, level_items=want)
        items[want] = h.factor_plan(B.FACTOR_P1)["n_bwd_items"]
        N = len(h.index(B.IDX_UPOS))
        b = np.random.default_rng(0).normal(size=N)
        x1, x2 = h.factor_apply(B.FACTOR_P1, b), h.factor_emulate(B.FACTOR_P1, b)
        assert np.abs(x1 - x2).max() <= 1e-12 * np.abs(x1).max()
    assert items[512] > items[0], items


@pytest.mark.parametrize("case,msg", [
    ("index", "out of range"), ("negative", "out of range"), ("degenerate", "degenerate"),
    ("nan_xyz", "non-finite vertex"), ("inf_sigma", "conductivities"), ("zero_sigma", "conductivities"),
    ("nan_fibre", "fibre"), ("stim_window", "stimulus"), ("no_heart", "no heart")])
def test_setup_refuses_malformed_input(case, msg):
    """Malformed meshes, tissues and stimuli are refused at set-up with
    BIDO_ERR_ARG and a message naming the problem, before any factorisation."""
    import paper_1711_08708_amd as B
    base = w.square2d(n=6)
    cfg = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in base.items()}
    heart_e = int(np.nonzero(cfg["region"] == 1)[0][0])
    if case == "index":
        cfg["elems"][0, 0] = len(cfg["xyz"]) + 5
    elif case == "negative":
        cfg["elems"][0, 1] = -3
    elif case == "degenerate":
        cfg["elems"][0] = [0, 0, 1]
    elif case == "nan_xyz":
        cfg["xyz"][3, 0] = np.nan
    elif case == "inf_sigma":
        cfg["sigma_i"] = np.array([np.inf, 1.0])
    elif case == "zero_sigma":
        cfg["sigma_e"] = np.array([1.0, 0.0])
    elif case == "nan_fibre":
        cfg["fibre"][heart_e, 0, 0] = np.nan
    elif case == "stim_window":
        cfg["stim_t0"], cfg["stim_t1"] = 2.0, 1.0
    elif case == "no_heart":
        cfg["region"] = np.zeros_like(cfg["region"])
        cfg["stim_mask"] = np.zeros_like(cfg["stim_mask"])
    with pytest.raises(B.BidoError, match=msg) as ei:
        B.HostSetup(cfg)
    assert ei.value.code == -1


@pytest.mark.parametrize("field,value", [("amg_columns", 2), ("amg_columns", -1), ("guess_states", 17), ("guess_states", -1),
                                         ("inner_pk", 9), ("inner_p1", 4)])
def test_setup_refuses_bad_options(field, value):
    """Option fields outside their documented values are refused at set-up
    with BIDO_ERR_ARG and a message naming the field."""
    import paper_1711_08708_amd as B
    with pytest.raises(B.BidoError, match=field) as ei:
        B.HostSetup(w.square2d(n=6), **{field: value})
    assert ei.value.code == -1


def test_default_options():
    """Defaults: 16-bit multigrid columns where they fit, initial guesses
    projected onto the span of 8 previous states."""
    import paper_1711_08708_amd as B
    p = B.default_params()
    assert p.amg_columns == 0 and p.guess_states == 8
