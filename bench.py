"""Throughput benchmark of the bidomain per-step solve on one MI355X.

A step is one pass of the whole hot path (Steps 1-3 of the resolution
algorithm: ionic RHS and gating, the block-LU preconditioned CG solve of
Lambda X = Y, the normalisation of U) over the synthetic thorax-like slice
of about 200k vertices.  Prints ONE JSON line.

Roofline: the same timed steps are replayed (from the same saved state) with
HIP events around every launch; the dominant kernel class is the one with
the largest summed duration, and `achieved` is its algorithmic bytes (inputs
read once, outputs written once) divided by its summed event time.

CPU baseline: the FP64 oracle (sparse direct solve of the normalised system)
timed on a bounded sample of the same workload's steps on the host.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "bidomain time steps/sec at 1e-8 rel error; learned+mixed vs plain PCG; HBM GB/s"
HBM_PEAK_GBS = 8000.0
V_ACT = 64.0    # activation level, mV above rest (the -20 mV level of the paper with a rest near -84 mV)


def _parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None,
                    help="timed steps (default 100; 10 per variant on slab128)")
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--config", default="slab128",
                    help="slab128 (the 3D slab of 2,146,689 vertices: plain vs learned+mixed, the headline), "
                         "thorax200k, slab64, square48 or batch64")
    ap.add_argument("--tol", type=float, default=1e-10)
    ap.add_argument("--eps", type=float, default=1e-8,
                    help="accuracy of the hierarchical top of the inner solves (0: exact)")
    ap.add_argument("--precision", default="fp64", choices=["fp64", "mixed"])
    ap.add_argument("--scheme", default="euler", choices=["euler", "cn", "strang"],
                    help="time scheme: semi-implicit (Sec. 3.2), Crank-Nicolson or Strang splitting")
    ap.add_argument("--pk", default="cholesky", choices=["cholesky", "chebyshev", "amg"],
                    help="P_K inside the block-LU preconditioner: the factor of K_m, "
                         "Chebyshev-accelerated Jacobi steps on K_m, or a multigrid V-cycle")
    ap.add_argument("--p1", default="cholesky", choices=["cholesky", "amg"],
                    help="P_1 inside the block-LU preconditioner: the factor of the grounded S_1, "
                         "or a multigrid V-cycle (no factorisation)")
    ap.add_argument("--pk-steps", type=int, default=3, help="Chebyshev steps of --pk chebyshev")
    ap.add_argument("--no-record", action="store_true",
                    help="do not record activation times (and the electrode potentials of the thorax workloads)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--no-parity", action="store_true", help="skip the sampled parity check")
    ap.add_argument("--cpu-steps", type=int, default=8,
                    help="oracle steps timed for the CPU baseline (about 10-30 s of host work)")
    ap.add_argument("--no-variants", action="store_true",
                    help="skip the mixed / learned / learned+mixed comparison")
    ap.add_argument("--collect-steps", type=int, default=40,
                    help="plain steps whose CG iterations provide training pairs")
    ap.add_argument("--variant-steps", type=int, default=50)
    ap.add_argument("--epochs", type=int, default=30)
    ap.add_argument("--no-tune", action="store_true", help="skip the autotuning of the inner-solve plans")
    ap.add_argument("--graphs", type=int, default=-1, choices=[-1, 0, 1],
                    help="replay captured iteration graphs: 1 always, 0 never, -1 the library default")
    ap.add_argument("--batch-streams", type=int, default=4, help="streams of the batch (batch64, --batch-mode streams)")
    ap.add_argument("--batch-mode", choices=["fused", "streams"], default="fused",
                    help="batch64: one union PCG for all slices (fused) or lockstep slices on streams; "
                         "the learned stencil runs on streams")
    ap.add_argument("--batch-learned", action="store_true",
                    help="batch64: train the learned stencil of every slice first")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain 256 MiB device copy three times (counter calibration)")
    return ap.parse_args()


COPY_BYTES = 256 << 20


def _calibrate_copy():
    """A plain device-to-device copy of known size, for scaling the HBM
    byte counters (FETCH_SIZE, WRITE_SIZE) of a profiler run."""
    import torch
    a = torch.ones(COPY_BYTES // 8, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": COPY_BYTES, "launches": 3}))


def _traffic(kernel, workload, precision):
    """HBM bytes per launch of `kernel` from the committed counter summary,
    or None when there is none or the kernel source changed since."""
    import hashlib
    import re
    path = os.path.join(ROOT, "profiles", f"traffic_{kernel}_{workload}_{precision}.md")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    m = re.search(r"kernel_source_sha256:\s*([0-9a-f]{64})", text)
    t = re.search(r"traffic_bytes_per_launch:\s*([0-9.eE+]+)", text)
    if not m or not t:
        return None
    src = os.path.join(ROOT, "paper_1711_08708_amd", "csrc", _kernel_source(kernel))
    if hashlib.sha256(open(src, "rb").read()).hexdigest() != m.group(1):
        return None
    return float(t.group(1))


def _kernel_source(kernel):
    """The source file of a profiler class's kernels."""
    if kernel.startswith("amg_"):
        return "amg.hip"
    if kernel.startswith("seg_"):
        return "batch.hip"
    return "kernels.hip"


def _timed_steps(torch, solver, state, n0, k):
    v, h, u = state
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    iters = 0
    t0 = time.perf_counter()
    e0.record()
    for n in range(n0, n0 + k):
        st = solver.step(v, h, u, n)
        iters += st["iterations"]
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return e0.elapsed_time(e1) / 1000.0, wall, iters


def main():
    args = _parse()
    if args.steps is None:
        args.steps = 10 if args.config == "slab128" else 100
    if args.gpus != 1:
        print(json.dumps({"error": "the solver runs on one GPU; --gpus must be 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    if args.calibrate_copy:
        _calibrate_copy()
        return
    if args.config == "batch64":
        _bench_batch(args)
        return
    if args.config == "slab128":
        _bench_slab128(args)
        return
    import numpy as np
    import torch

    import paper_1711_08708_amd as B
    import workloads as w

    torch.cuda.set_device(0)
    cfg = w.make_config(args.config)
    prec = B.PREC_MIXED if args.precision == "mixed" else B.PREC_FP64
    t_setup = time.perf_counter()
    scheme = {"euler": B.SCHEME_EULER, "cn": B.SCHEME_CN, "strang": B.SCHEME_STRANG}[args.scheme]
    inner_p1 = B.P1_AMG if args.p1 == "amg" else B.P1_CHOLESKY
    inner_pk = {"cholesky": B.PK_CHOLESKY, "chebyshev": B.PK_CHEBYSHEV, "amg": B.PK_AMG}[args.pk]
    solver = B.Solver(cfg, tol=args.tol, eps_h=args.eps, precision=prec, scheme=scheme,
                      inner_p1=inner_p1, inner_pk=inner_pk)
    t_setup = time.perf_counter() - t_setup
    tune = None if args.no_tune else solver.autotune()
    if args.pk == "chebyshev":
        solver.set_pk(B.PK_CHEBYSHEV, args.pk_steps)
    recording = not args.no_record
    if recording:       # activation times, and the electrode potentials where the workload has electrodes
        solver.record(V_ACT, cfg.get("electrodes"), max_steps=args.warmup + args.steps if "electrodes" in cfg else 0)
    if args.graphs >= 0:
        solver.set_graphs(bool(args.graphs))
    info = solver.info
    print(f"[bench] {cfg['name']}: N={solver.N} N_H={solver.NH} setup {t_setup:.2f}s "
          f"P1 {info['bytes_p1']/1e6:.1f} MB PK {info['bytes_pk']/1e6:.1f} MB", file=sys.stderr,
          flush=True)

    v, h, u = solver.state()
    for n in range(args.warmup):
        solver.step(v, h, u, n)
    saved = [t.clone() for t in (v, h, u)]
    n0 = args.warmup
    gpu_s, wall_s, iters = _timed_steps(torch, solver, (v, h, u), n0, args.steps)
    steps_per_s = args.steps / wall_s
    print(f"[bench] {args.steps} steps: {wall_s*1e3/args.steps:.3f} ms/step (events "
          f"{gpu_s*1e3/args.steps:.3f}), {iters/args.steps:.2f} CG iterations/step",
          file=sys.stderr, flush=True)

    # replay the timed steps from the saved state with per-launch events
    v2, h2, u2 = [t.clone() for t in saved]
    solver.profile(True)
    last_state = None
    for n in range(n0, n0 + args.steps):
        if n == n0 + args.steps - 1:
            last_state = [t.cpu().numpy().copy() for t in (v2, h2, u2)]
        solver.step(v2, h2, u2, n)
    prof = solver.profile_read()
    solver.profile(False)
    dom_name, dom = max(prof.items(), key=lambda kv: kv[1]["ms"])
    achieved = dom["bytes"] / (dom["ms"] / 1e3) / 1e9
    total_bytes = sum(p["bytes"] for p in prof.values())
    total_ms = sum(p["ms"] for p in prof.values())
    roofline = {"bound": "hbm", "kernel": dom_name, "achieved": round(achieved, 1),
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": _traffic(dom_name, cfg["name"], args.precision),
                "launches": dom["launches"], "avg_launch_us": round(dom["ms"] * 1e3 / dom["launches"], 2),
                "bytes_per_launch": round(dom["bytes"] / dom["launches"]),
                "step_bytes": round(total_bytes / args.steps),
                "step_kernel_ms": round(total_ms / args.steps, 4)}
    kernels = {k: {"launches": p["launches"], "ms": round(p["ms"], 3),
                   "GBps": round(p["bytes"] / max(p["ms"], 1e-9) / 1e6, 1)} for k, p in prof.items()}

    result = {
        "metric": METRIC, "value": round(steps_per_s, 3), "unit": "steps/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(wall_s * 1e3 / args.steps, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64" if prec == B.PREC_FP64 else "f64+f32",
        "data": "synthetic",
        "config": {"workload": f"{cfg['name']}: " + (
                       f"2D thorax-like slice, {solver.N} vertices ({solver.NH} heart)" if cfg["dim"] == 2 else
                       f"3D orthotropic slab, {solver.N} vertices (isolated heart)") +
                       {"cn": ", Crank-Nicolson", "strang": ", Strang splitting (Crank-Nicolson diffusion)",
                        "euler": ", semi-implicit"}[args.scheme] +
                       f" bidomain step, block-LU/monodomain PCG, {args.precision} preconditioner" +
                       (", multigrid P_1" if args.p1 == "amg" else "") +
                       (f", Chebyshev P_K ({args.pk_steps} steps)" if args.pk == "chebyshev" else
                        ", multigrid P_K" if args.pk == "amg" else ""),
                   "scheme": args.scheme, "pk": solver.pk(),
                   "n_nodes": solver.N, "n_heart": solver.NH, "dt_ms": cfg["dt"],
                   "tol": args.tol, "eps_h": args.eps, "precision": args.precision,
                   "first_step": n0, "cg_iterations_per_step": round(iters / args.steps, 3),
                   "setup_s": round(t_setup, 2),
                   "tune": None if tune is None else {
                       "seconds": round(tune["seconds"], 2), "candidates": tune["candidates"],
                       "us_before": [round(x, 1) for x in tune["us_before"]],
                       "us_after": [round(x, 1) for x in tune["us_after"]],
                       "top_h": tune["top_h"], "fwd_cols": tune["fwd_cols"], "bwd_rows": tune["bwd_rows"]}},
        "roofline": roofline,
        "kernels": kernels,
    }

    if not args.no_parity and last_state is not None:
        from oracle import bidomain as bd
        s = bd.System(cfg, scheme=args.scheme)
        Uo, Vo, _ = s.step(last_state[0], last_state[1], n0 + args.steps - 1, U0=s.from_global_u(last_state[2]))
        Uo = s.to_global_u(Uo)
        U, V = u2.cpu().numpy(), v2.cpu().numpy()
        result["parity"] = {"step": n0 + args.steps - 1,
                            "e_u": float(np.linalg.norm(U - Uo) / np.linalg.norm(Uo)),
                            "e_v": float(np.linalg.norm(V - Vo) / np.linalg.norm(Vo))}
        if recording and "electrodes" in cfg:
            from oracle import record as rc
            rows = solver.record_read()[1]
            ecg_o = rc.probe_values(cfg["xyz"], cfg["elems"], Uo, cfg["electrodes"])
            result["parity"]["e_ecg"] = float(np.abs(rows[-1] - ecg_o).max() / np.abs(Uo).max())

    if recording:
        act, rows = solver.record_read()
        result["recording"] = {"v_act_mV": V_ACT, "electrodes": len(cfg.get("electrodes", [])), "rows": len(rows),
                               "activated": int((act >= 0).sum()), "heart_vertices": solver.NH,
                               "latest_activation_ms": float(act.max())}
        if len(rows):
            result["recording"]["ecg_last_row"] = [round(float(x), 4) for x in rows[-1]]

    if not args.no_cpu:
        result["cpu_baseline"] = _cpu_baseline(cfg, args.cpu_steps, args.scheme)

    if not args.no_variants:
        result["variants"] = _variants(torch, B, solver, args, cfg)
    print(json.dumps(result), flush=True)


def _variants(torch, B, solver, args, w_cfg):
    """Plain FP64 vs mixed vs learned vs learned+mixed on the same steps, and
    the factored P_K against the Chebyshev one (FP64 and mixed).

    The learned Schur-complement stencil is trained on pairs recorded during
    the first `collect_steps` plain steps from rest and K_m + C is factored;
    every variant then runs the following `variant_steps` steps from the
    same saved state, and one more step that is checked against the oracle's
    step from the same state (e_u, e_v)."""
    import numpy as np
    out = {}
    v, h, u = solver.state()
    solver.set_precond(B.PRECOND_PLAIN)
    solver.set_precision(B.PREC_FP64)
    t0 = time.perf_counter()
    col = solver.learn_collect(v, h, u, 0, args.collect_steps, max_samples=16 * args.collect_steps)
    t_col = time.perf_counter() - t0
    n_val = max(1, col["samples"] // 10)
    ts = solver.learn_train(kind=B.LEARN_STENCIL, epochs=args.epochs, batch=8, lr=2e-3, seed=0, n_val=n_val)
    out["training"] = {"kind": "stencil", "collect_steps": args.collect_steps, "pairs": col["samples"],
                       "collect_s": round(t_col, 3), "train_s": round(ts["seconds"], 3),
                       "refactor_s": round(ts["refactor_seconds"], 3), "spd": ts["spd"],
                       "epochs": args.epochs, "loss_zero": round(ts["loss_zero"], 3),
                       "loss_trained": round(ts["loss_last"], 3),
                       "loss_zero_val": round(ts["loss_zero_val"], 3),
                       "loss_val": round(ts["loss_val"], 3)}
    saved = [t.clone() for t in (v, h, u)]
    n1 = args.collect_steps
    main_pk = solver.pk()
    chol, cheb = B.PK_CHOLESKY, B.PK_CHEBYSHEV
    runs = [("plain_fp64", B.PREC_FP64, B.PRECOND_PLAIN, chol), ("mixed", B.PREC_MIXED, B.PRECOND_PLAIN, chol),
            ("chebyshev_pk_fp64", B.PREC_FP64, B.PRECOND_PLAIN, cheb),
            ("chebyshev_pk_mixed", B.PREC_MIXED, B.PRECOND_PLAIN, cheb)]
    if ts["spd"]:
        runs += [("learned_fp64", B.PREC_FP64, B.PRECOND_LEARNED, chol),
                 ("learned_mixed", B.PREC_MIXED, B.PRECOND_LEARNED, chol)]
    sysm = None
    if not args.no_parity:
        from oracle import bidomain as bd
        sysm = bd.System(w_cfg, scheme=args.scheme)
    for name, prec, pc, pk in runs:
        solver.set_precision(prec)
        solver.set_precond(pc)
        solver.set_pk(pk, args.pk_steps)
        solver.reset_guess()                      # every variant starts its span of states afresh
        st = [t.clone() for t in saved]
        _, ws, it = _timed_steps(torch, solver, st, n1, args.variant_steps)
        out[name] = {"steps_per_s": round(args.variant_steps / ws, 3),
                     "cg_iterations_per_step": round(it / args.variant_steps, 3)}
        if sysm is not None:    # one more step of the variant against the oracle's step from its state
            n = n1 + args.variant_steps
            V0, h0, U0 = [t.cpu().numpy().copy() for t in st]
            solver.step(st[0], st[1], st[2], n)
            Uo, Vo, _ = sysm.step(V0, h0, n, U0=sysm.from_global_u(U0))
            Uo = sysm.to_global_u(Uo)
            U, V = st[2].cpu().numpy(), st[0].cpu().numpy()
            out[name]["e_u"] = float(np.linalg.norm(U - Uo) / np.linalg.norm(Uo))
            out[name]["e_v"] = float(np.linalg.norm(V - Vo) / np.linalg.norm(Vo))
    base = out["plain_fp64"]["steps_per_s"]
    for name in [r[0] for r in runs[1:]]:
        out[name]["speedup_vs_plain"] = round(out[name]["steps_per_s"] / base, 3)
    out["steps"] = [n1, n1 + args.variant_steps]
    out["chebyshev_pk_steps"] = args.pk_steps
    # a change of time step: the factored P_K refactors K_m on the host, the
    # Chebyshev P_K only updates device copies; then steps at dt / 2
    solver.set_precision(B.PREC_FP64)
    solver.set_precond(B.PRECOND_PLAIN)
    dt0 = solver.dt
    out["dt_change"] = {"dt_ms": [dt0, dt0 / 2]}
    for name, pk in (("cholesky", chol), ("chebyshev", cheb)):
        solver.set_pk(pk, args.pk_steps)
        sec = solver.set_dt(dt0 / 2)
        st = [t.clone() for t in saved]
        _, ws, it = _timed_steps(torch, solver, st, n1, 10)
        out["dt_change"][name] = {"set_dt_s": round(sec, 4), "steps_per_s": round(10 / ws, 2),
                                  "cg_iterations_per_step": round(it / 10, 2)}
        solver.set_dt(dt0)
    solver.set_precision(B.PREC_FP64)
    solver.set_precond(B.PRECOND_PLAIN)
    solver.set_pk(main_pk["kind"], max(1, main_pk["steps"]), main_pk["lo"], main_pk["hi"])
    return out


def _bench_slab128(args):
    """The 3D orthotropic slab at 128^3 hexes (2,146,689 vertices, isolated
    heart): plain FP64 block-LU PCG against the learned correction with
    mixed precision, at tol 1e-10.

    Both inner solves are multigrid V-cycles (no factorisation: exact or
    hierarchical factors of this mesh do not fit a set-up budget).  The
    learned Schur-complement stencil is trained on the residual/error pairs
    of the first `collect_steps` (default 100) plain steps from rest; the
    preconditioner then uses a multigrid hierarchy of K_m + C.  Every variant
    runs the same `steps` steps from the state after the collection, then
    one more step whose solution is checked against the oracle on sampled
    rows (Lambda X - Y assembled row by row from the elements of 4,096
    sampled vertices) and for the normalisation (M U, 1) = 0."""
    import numpy as np
    import torch

    import paper_1711_08708_amd as B
    import workloads as w
    from oracle import bidomain as bd

    torch.cuda.set_device(0)
    if args.collect_steps == 40:        # the parser's default is sized for the 2D slice
        args.collect_steps = 100
    cfg = w.make_config("slab128")
    t0 = time.perf_counter()
    solver = B.Solver(cfg, tol=args.tol, eps_h=0.0, precision=B.PREC_FP64, inner_p1=B.P1_AMG,
                      inner_pk=B.PK_AMG)
    t_setup = time.perf_counter() - t0
    info = solver.info
    print(f"[bench] slab128: N={solver.N} setup {t_setup:.1f} s; one V-cycle reads P1 "
          f"{info['bytes_p1'] / 1e6:.0f} MB, PK {info['bytes_pk'] / 1e6:.0f} MB", file=sys.stderr, flush=True)
    v, h, u = solver.state()
    t0 = time.perf_counter()
    col = solver.learn_collect(v, h, u, 0, args.collect_steps, max_samples=200)
    t_col = time.perf_counter() - t0
    print(f"[bench] collected {col['samples']} pairs over {args.collect_steps} plain steps in {t_col:.1f} s",
          file=sys.stderr, flush=True)
    n_val = max(1, col["samples"] // 10)
    ts = solver.learn_train(kind=B.LEARN_STENCIL, epochs=args.epochs, batch=8, lr=2e-3, seed=0, n_val=n_val)
    print(f"[bench] trained the stencil in {ts['seconds']:.1f} s (hierarchy of K_m + C "
          f"{ts['refactor_seconds']:.1f} s), loss {ts['loss_zero']:.3g} -> {ts['loss_last']:.3g}, "
          f"held-out {ts['loss_zero_val']:.3g} -> {ts['loss_val']:.3g}, kept epoch {ts['best_epoch']}",
          file=sys.stderr, flush=True)
    saved = [t.clone() for t in (v, h, u)]
    n1 = args.collect_steps
    rng = np.random.default_rng(11)
    sample = np.sort(rng.choice(solver.N, size=4096, replace=False))
    runs = [("plain_fp64", B.PREC_FP64, B.PRECOND_PLAIN), ("mixed", B.PREC_MIXED, B.PRECOND_PLAIN)]
    if ts["spd"]:
        runs += [("learned_fp64", B.PREC_FP64, B.PRECOND_LEARNED), ("learned_mixed", B.PREC_MIXED, B.PRECOND_LEARNED)]
    variants = {}
    m = cfg_mass(cfg)
    for name, prec, pc in runs:
        solver.set_precision(prec)
        solver.set_precond(pc)
        solver.reset_guess()                      # every variant starts its span of states afresh
        st = [t.clone() for t in saved]
        for n in range(n1, n1 + args.warmup):                 # warm-up steps of this variant
            solver.step(st[0], st[1], st[2], n)
        gpu_s, wall_s, it = _timed_steps(torch, solver, st, n1 + args.warmup, args.steps)
        variants[name] = {"steps_per_s": round(args.steps / wall_s, 3), "ms_per_step": round(wall_s * 1e3 / args.steps, 3),
                          "cg_iterations_per_step": round(it / args.steps, 3)}
        # one more step, checked on sampled rows against the oracle
        n = n1 + args.warmup + args.steps
        Vn, hn = st[0].cpu().numpy().copy(), st[1].cpu().numpy().copy()
        solver.step(st[0], st[1], st[2], n)
        U1, V1 = st[2].cpu().numpy(), st[0].cpu().numpy()
        ru, rv, yv = bd.sampled_residual(cfg, sample, Vn, hn, n, U1, V1)
        variants[name]["parity"] = {"sampled_rows": int(len(sample)),
                                    "max_abs_residual_over_max_abs_y": float(max(np.abs(ru).max(), np.abs(rv).max())
                                                                            / np.abs(yv).max()),
                                    "mean_u_over_max_u": float(abs(m @ U1) / m.sum() / np.abs(U1).max())}
        print(f"[bench] {name}: {variants[name]}", file=sys.stderr, flush=True)
    plain = variants["plain_fp64"]["steps_per_s"]
    for name in variants:
        variants[name]["speedup_vs_plain"] = round(variants[name]["steps_per_s"] / plain, 3)
    head = "learned_mixed" if "learned_mixed" in variants else "mixed"

    # replay the headline variant's timed steps with per-launch events
    solver.set_precision(B.PREC_MIXED)
    solver.set_precond(B.PRECOND_LEARNED if head == "learned_mixed" else B.PRECOND_PLAIN)
    solver.reset_guess()
    st = [t.clone() for t in saved]
    for n in range(n1, n1 + args.warmup):
        solver.step(st[0], st[1], st[2], n)
    solver.profile(True)
    for n in range(n1 + args.warmup, n1 + args.warmup + args.steps):
        solver.step(st[0], st[1], st[2], n)
    prof = solver.profile_read()
    solver.profile(False)
    # the roofline names one kernel: the class with the most time among those
    # that are one kernel on one operand (amg_coarser gathers every kernel of
    # the coarser levels, misc the small vector kernels)
    single = {k: p for k, p in prof.items() if k not in ("amg_coarser", "misc")}
    dom_name, dom = max(single.items(), key=lambda kv: kv[1]["ms"])
    achieved = dom["bytes"] / (dom["ms"] / 1e3) / 1e9
    total_ms = sum(p["ms"] for p in prof.values())
    roofline = {"bound": "hbm", "kernel": dom_name, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": _traffic(dom_name, cfg["name"], "mixed"),
                "launches": dom["launches"], "avg_launch_us": round(dom["ms"] * 1e3 / dom["launches"], 2),
                "bytes_per_launch": round(dom["bytes"] / dom["launches"]),
                "share_of_step": round(dom["ms"] / total_ms, 4),
                "step_bytes": round(sum(p["bytes"] for p in prof.values()) / args.steps),
                "step_kernel_ms": round(total_ms / args.steps, 4)}
    if "amg_coarser" in prof:
        c = prof["amg_coarser"]
        roofline["coarser_levels"] = {"share_of_step": round(c["ms"] / total_ms, 4),
                                      "GBps": round(c["bytes"] / max(c["ms"], 1e-9) / 1e6, 1)}
    kernels = {k: {"launches": p["launches"], "ms": round(p["ms"], 3),
                   "GBps": round(p["bytes"] / max(p["ms"], 1e-9) / 1e6, 1)} for k, p in prof.items()}
    # a change of time step: the multigrid K_m moves to the new gamma on the
    # device (no new aggregation); then plain FP64 steps at dt / 2, the last
    # one checked on the sampled rows at the new step
    solver.set_precision(B.PREC_FP64)
    solver.set_precond(B.PRECOND_PLAIN)
    dt0 = cfg["dt"]
    sec = solver.set_dt(dt0 / 2)
    st = [t.clone() for t in saved]
    _, ws, it = _timed_steps(torch, solver, st, n1, 5)
    n = n1 + 5
    Vn, hn = st[0].cpu().numpy().copy(), st[1].cpu().numpy().copy()
    solver.step(st[0], st[1], st[2], n)
    U1, V1 = st[2].cpu().numpy(), st[0].cpu().numpy()
    ru, rv, yv = bd.sampled_residual(dict(cfg, dt=dt0 / 2), sample, Vn, hn, n, U1, V1)
    dt_change = {"dt_ms": [dt0, dt0 / 2], "set_dt_s": round(sec, 4), "steps_per_s": round(5 / ws, 3),
                 "cg_iterations_per_step": round(it / 5, 2),
                 "parity": {"sampled_rows": int(len(sample)),
                            "max_abs_residual_over_max_abs_y": float(max(np.abs(ru).max(), np.abs(rv).max())
                                                                    / np.abs(yv).max())}}
    print(f"[bench] dt change: {dt_change}", file=sys.stderr, flush=True)
    solver.set_dt(dt0)
    hv = variants[head]
    result = {
        "metric": METRIC, "value": hv["steps_per_s"], "unit": "steps/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": hv["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64+f32",
        "data": "synthetic",
        "config": {"workload": f"slab3d_n128: 3D orthotropic slab [0,1]^3 cm, 128^3 hexes x 6 tets, "
                               f"{solver.N} vertices (isolated heart), semi-implicit bidomain step, "
                               f"block-LU/monodomain flexible PCG to tol {args.tol:g}, multigrid P_1 and P_K, "
                               f"{head.replace('_', ' + ')} (value) against plain FP64 (plain_fp64)",
                   "n_nodes": solver.N, "n_heart": solver.NH, "dt_ms": cfg["dt"], "tol": args.tol,
                   "first_timed_step": n1 + args.warmup, "setup_s": round(t_setup, 2),
                   "p1": "multigrid", "pk": "multigrid",
                   "multigrid_bytes_per_vcycle_fp64": {"p1": info["bytes_p1"], "pk": info["bytes_pk"]},
                   "cg_iterations_per_step": hv["cg_iterations_per_step"]},
        "plain_fp64": variants["plain_fp64"],
        "speedup_vs_plain": hv["speedup_vs_plain"],
        "variants": variants,
        "training": {"kind": "stencil", "collect_steps": args.collect_steps, "pairs": col["samples"],
                     "collect_s": round(t_col, 2), "train_s": round(ts["seconds"], 2),
                     "hierarchy_s": round(ts["refactor_seconds"], 2), "spd": ts["spd"], "epochs": args.epochs,
                     "loss_zero": ts["loss_zero"], "loss_trained": ts["loss_last"],
                     "loss_zero_val": ts["loss_zero_val"], "loss_val": ts["loss_val"],
                     "best_epoch": ts["best_epoch"]},
        "roofline": roofline,
        "kernels": kernels,
        "dt_change": dt_change,
    }
    if not args.no_cpu:
        result["cpu_baseline"] = _cpu_baseline_slab(solver.N)
    print(json.dumps(result), flush=True)


def cfg_mass(cfg):
    """Lumped mass of every vertex (the weight of the normalisation (M U, 1))."""
    import numpy as np
    from oracle import fem
    return fem.lumped_mass(cfg["xyz"], cfg["elems"].astype(np.int64), len(cfg["xyz"]))


def _cpu_baseline_slab(n_target):
    """The oracle on the host: one step from rest of a 32^3 and a 40^3 slab
    (FP64 Jacobi-CG with the condition-aware stop; assembly excluded),
    extrapolated to n_target vertices with the exponent the two sizes give."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    import workloads as w
    from oracle import bidomain as bd
    pts = []
    with threadpool_limits(limits=1):
        for n in (32, 40):
            s = bd.System(w.slab3d(n=n))
            V = np.zeros(s.NH)
            hh = np.ones(s.NH)
            t0 = time.perf_counter()
            s.step(V, hh, 0, U0=np.zeros(s.N))
            pts.append((s.N, time.perf_counter() - t0))
    (n0, t0_), (n1, t1_) = pts
    alpha = float(np.log(t1_ / t0_) / np.log(n1 / n0))
    t_full = t1_ * (n_target / n1) ** alpha
    return {"value": round(1.0 / t_full, 6), "unit": "steps/s", "cores": 1, "kind": "oracle", "threads": 1,
            "host_cpus": os.cpu_count(), "cpu_model": _cpu_model(),
            "sample": f"one oracle step (FP64 NumPy/SciPy: Step 1, Jacobi-CG with the condition-aware stop, "
                      f"normalisation, Step 3; assembly excluded) of the 32^3 slab ({n0} vertices, {t0_:.2f} s) "
                      f"and the 40^3 slab ({n1} vertices, {t1_:.2f} s); value extrapolated to {n_target} "
                      f"vertices as t ~ N^{alpha:.2f}",
            "measured_steps_per_s": {str(n0): round(1.0 / t0_, 4), str(n1): round(1.0 / t1_, 4)}}


def _gen_slice(kw):
    import workloads as w
    return w.thorax2d(**kw)


def _bench_batch(args):
    """64 independent thorax-like slices (vertex counts log-uniform in
    [20k, 300k], seeded sites and conductivity scales) stepped together;
    the value is slice-steps per second of the whole batch."""
    if args.scheme != "euler":
        raise SystemExit("batch64 runs the semi-implicit scheme of its configuration (no --scheme)")
    import concurrent.futures as cf

    import numpy as np
    import torch

    import paper_1711_08708_amd as B
    import workloads as w

    torch.cuda.set_device(0)
    prec = B.PREC_MIXED if args.precision == "mixed" else B.PREC_FP64
    kws = w.make_config("batch64")
    t0 = time.perf_counter()
    with cf.ProcessPoolExecutor(max_workers=min(16, os.cpu_count() or 1)) as ex:
        cfgs = list(ex.map(_gen_slice, kws))
    t_mesh = time.perf_counter() - t0
    t0 = time.perf_counter()
    solvers = [B.Solver(c, tol=args.tol, eps_h=args.eps, precision=prec) for c in cfgs]
    if args.pk == "chebyshev":
        for sv in solvers:
            sv.set_pk(B.PK_CHEBYSHEV, args.pk_steps)
    t_setup = time.perf_counter() - t0
    n_nodes = sum(s.N for s in solvers)
    union_rows = sum(s.N + s.NH for s in solvers)
    union_nnz = sum(s.info["nnz_lambda"] for s in solvers)
    print(f"[bench] batch64: {len(solvers)} slices, {n_nodes} vertices, meshes {t_mesh:.1f}s, "
          f"set-up {t_setup:.1f}s", file=sys.stderr, flush=True)
    sample = [int(np.argmin([s.N for s in solvers])), int(np.argmax([s.N for s in solvers]))]
    keep = {k: cfgs[k] for k in sample}
    del cfgs
    training = None
    if args.batch_learned:
        t0 = time.perf_counter()
        spd = 0
        for sv in solvers:
            v, h, u = sv.state()
            col = sv.learn_collect(v, h, u, 0, args.collect_steps, max_samples=16 * args.collect_steps)
            n_val = max(1, col["samples"] // 10)
            ts = sv.learn_train(kind=B.LEARN_STENCIL, epochs=args.epochs, batch=8, lr=2e-3, seed=0, n_val=n_val)
            spd += ts["spd"]
            if ts["spd"]:
                sv.set_precond(B.PRECOND_LEARNED)
        training = {"collect_steps": args.collect_steps, "epochs": args.epochs, "spd_slices": spd,
                    "seconds": round(time.perf_counter() - t0, 1)}
    mode = args.batch_mode
    t0 = time.perf_counter()
    batch = B.Batch(solvers, n_streams=args.batch_streams, fused=mode == "fused")
    t_batch = time.perf_counter() - t0
    states = [s.state() for s in solvers]
    batch.run(states, 0, args.warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    tot, per = batch.run(states, args.warmup, args.steps - 1)
    before = {k: (states[k][0].cpu().numpy().copy(), states[k][1].cpu().numpy().copy()) for k in sample}
    tot2, per2 = batch.run(states, args.warmup + args.steps - 1, 1)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    S = len(solvers)
    n_last = args.warmup + args.steps - 1
    result = {
        "metric": METRIC, "value": round(S * args.steps / wall, 3), "unit": "slice-steps/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(wall * 1e3 / args.steps, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if prec == B.PREC_FP64 else "f64+f32", "data": "synthetic",
        "config": {"workload": f"batch64: {S} thorax-like slices, {n_nodes} vertices in total, "
                               f"vertex counts log-uniform in [20k, 300k], PCG per slice",
                   "slices": S, "total_nodes": n_nodes, "precision": args.precision, "tol": args.tol,
                   "mode": mode, "streams": args.batch_streams if mode == "streams" else 1,
                   "pk": args.pk if args.pk == "cholesky" else f"chebyshev ({args.pk_steps} steps)",
                   "union_rows": union_rows, "union_nnz_lambda": union_nnz,
                   "learned": bool(args.batch_learned), "batch_setup_s": round(t_batch, 1),
                   "mean_iterations_per_slice_step": round((tot["total_iterations"] + tot2["total_iterations"])
                                                           / (S * args.steps), 3),
                   "max_iterations_per_step": max(tot["iterations"], tot2["iterations"]),
                   "mesh_s": round(t_mesh, 1), "setup_s": round(t_setup, 1)},
    }
    if training:
        result["config"]["training"] = training
    from oracle import bidomain as bd
    par = {}
    for k in sample:
        sy = bd.System(keep[k])
        Uo, Vo, _ = sy.step(before[k][0], before[k][1], n_last)
        Uo = sy.to_global_u(Uo)
        U, V = states[k][2].cpu().numpy(), states[k][0].cpu().numpy()
        par[keep[k]["name"]] = {"e_u": float(np.linalg.norm(U - Uo) / np.linalg.norm(Uo)),
                                "e_v": float(np.linalg.norm(V - Vo) / np.linalg.norm(Vo))}
    result["parity"] = {"step": n_last, "slices": par}
    if mode == "fused":
        # the stopping test runs on the device: host waits per step
        cnt = batch.counters()
        result["config"]["host_waits_per_step"] = round(cnt["host_waits"] / max(cnt["steps"], 1), 2)
        result["config"]["kernels_per_step"] = round(cnt["kernels"] / max(cnt["steps"], 1), 1)
        # three more steps with per-launch events on the union's sweeps: the
        # roofline of the dominant class (the segmented vector kernels are
        # not bracketed; rocprofv3 covers them)
        batch.profile(True)
        batch.run(states, n_last + 1, 3)
        prof = batch.profile_read()
        batch.profile(False)
        if prof:
            dom_name, dom = max(prof.items(), key=lambda kv: kv[1]["ms"])
            achieved = dom["bytes"] / (dom["ms"] / 1e3) / 1e9
            result["roofline"] = {"bound": "hbm", "kernel": dom_name, "achieved": round(achieved, 1),
                                  "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                                  "traffic": None, "launches": dom["launches"],
                                  "avg_launch_us": round(dom["ms"] * 1e3 / dom["launches"], 2),
                                  "bytes_per_launch": round(dom["bytes"] / dom["launches"]),
                                  "bytes_basis": "nominal: every slice's trees; slices that have met their "
                                                 "stopping test skip theirs, so the bytes moved are lower"}
            result["kernels"] = {k: {"launches": p["launches"], "ms": round(p["ms"], 3),
                                     "GBps": round(p["bytes"] / max(p["ms"], 1e-9) / 1e6, 1)}
                                 for k, p in prof.items()}
    if not args.no_cpu:
        k = sample[0]
        cb = _cpu_baseline(keep[k], args.cpu_steps)
        cb["value"] = round(cb["value"], 5)
        cb["unit"] = "slice-steps/s"
        cb["sample"] = "smallest slice: " + cb["sample"]
        result["cpu_baseline"] = cb
    batch.close()
    print(json.dumps(result), flush=True)


def _cpu_baseline(cfg, n_steps, scheme="euler"):
    """Oracle steps from rest on the host (sparse direct solve per step)."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    from oracle import bidomain as bd
    with threadpool_limits(limits=1):
        s = bd.System(cfg, scheme=scheme)
        V = np.zeros(s.NH)
        h = np.ones(s.NH)
        U = np.zeros(s.N)
        t0 = time.perf_counter()
        for n in range(n_steps):
            U, V, h = s.step(V, h, n, U0=U)
        el = time.perf_counter() - t0
    how = ("sparse LU of the grounded Lambda" if cfg["dim"] == 2 or s.N + s.NH <= 6000
           else "Jacobi-CG with the condition-aware stop")
    return {"value": round(n_steps / el, 5), "unit": "steps/s", "cores": 1, "kind": "oracle",
            "threads": 1, "host_cpus": os.cpu_count(), "cpu_model": _cpu_model(),
            "sample": f"{n_steps} steps of {cfg['name']} from rest (FP64 NumPy/SciPy oracle: "
                      f"Step 1, {how}, normalisation, Step 3; assembly excluded; BLAS and "
                      f"OpenMP pools limited to 1 thread), {el:.1f} s"}


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


if __name__ == "__main__":
    main()
