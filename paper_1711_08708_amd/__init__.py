"""Python binding of libbido, the MI355X bidomain per-step solver.

Argument marshalling only: every step of the solve runs inside libbido.so
(HIP kernels for gfx950 plus its host set-up).  PyTorch supplies device
memory and the stream.  Importing this package fails loudly when the
library has not been built.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libbido.so")

BIDO_OK = 0
ERRORS = {-1: "BIDO_ERR_ARG", -2: "BIDO_ERR_DEVICE", -3: "BIDO_ERR_NOT_SPD",
          -4: "BIDO_ERR_NOT_CONVERGED", -5: "BIDO_ERR_DT_MISMATCH",
          -6: "BIDO_ERR_RANGE", -7: "BIDO_ERR_STATE"}
PREC_FP64, PREC_MIXED = 0, 1
PRECOND_PLAIN, PRECOND_LEARNED, PRECOND_LEARNED_ADDITIVE = 0, 1, 2
SCHEME_EULER, SCHEME_CN, SCHEME_STRANG = 0, 1, 2
PK_CHOLESKY, PK_CHEBYSHEV, PK_AMG = 0, 1, 2
P1_CHOLESKY, P1_AMG = 0, 1
PK_MAX_STEPS, PK_LANCZOS_STEPS = 64, 20
LEARN_STENCIL, LEARN_ADDITIVE = 0, 1
MAT_S1, MAT_SI, MAT_SM, MAT_LAMBDA, MAT_GNN_AGG, MAT_KM = 0, 1, 2, 3, 4, 5
VEC_M, VEC_MH, VEC_GNN_STATIC = 0, 1, 2
IDX_UPOS, IDX_VPOS, IDX_HEART = 0, 1, 2
FACTOR_P1, FACTOR_PK = 0, 1

_c_double_p = ctypes.POINTER(ctypes.c_double)
_c_i64_p = ctypes.POINTER(ctypes.c_int64)
_c_i32_p = ctypes.POINTER(ctypes.c_int32)


class Mesh(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int), ("n_nodes", ctypes.c_int64),
                ("xyz", ctypes.c_void_p), ("n_elems", ctypes.c_int64),
                ("elems", ctypes.c_void_p), ("region", ctypes.c_void_p)]


class Tissue(ctypes.Structure):
    _fields_ = [("sigma_i", ctypes.c_double * 3), ("sigma_e", ctypes.c_double * 3),
                ("fibre", ctypes.c_void_p), ("region_sigma", ctypes.c_void_p),
                ("n_region_sigma", ctypes.c_int), ("stim_mask", ctypes.c_void_p),
                ("stim_amp", ctypes.c_double), ("stim_t0", ctypes.c_double),
                ("stim_t1", ctypes.c_double)]


class Params(ctypes.Structure):
    _fields_ = [("chi", ctypes.c_double), ("cm", ctypes.c_double), ("dt", ctypes.c_double),
                ("eps_h", ctypes.c_double), ("eta", ctypes.c_double), ("tol", ctypes.c_double),
                ("leaf", ctypes.c_int), ("max_iter", ctypes.c_int), ("precision", ctypes.c_int),
                ("precond", ctypes.c_int), ("ionic", ctypes.c_int), ("n_threads", ctypes.c_int),
                ("scheme", ctypes.c_int), ("inner_p1", ctypes.c_int), ("inner_pk", ctypes.c_int),
                ("amg_columns", ctypes.c_int), ("guess_states", ctypes.c_int)]


class Stats(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int), ("converged", ctypes.c_int),
                ("rel_residual", ctypes.c_double), ("ms", ctypes.c_double),
                ("fallbacks", ctypes.c_int), ("range_removed", ctypes.c_double),
                ("total_iterations", ctypes.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class Info(ctypes.Structure):
    _fields_ = [("n_nodes", ctypes.c_int64), ("n_heart", ctypes.c_int64),
                ("n_elems", ctypes.c_int64), ("nnz_lambda", ctypes.c_int64),
                ("bytes_lambda", ctypes.c_int64), ("bytes_p1", ctypes.c_int64),
                ("bytes_pk", ctypes.c_int64), ("dense_bytes_p1", ctypes.c_int64),
                ("dense_bytes_pk", ctypes.c_int64), ("levels_p1", ctypes.c_int),
                ("levels_pk", ctypes.c_int), ("lowrank_blocks", ctypes.c_int64),
                ("setup_seconds", ctypes.c_double), ("ground_index", ctypes.c_int),
                ("launches_per_sweep_p1", ctypes.c_int), ("launches_per_sweep_pk", ctypes.c_int)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class TrainStats(ctypes.Structure):
    _fields_ = [("samples", ctypes.c_int), ("train_samples", ctypes.c_int), ("epochs", ctypes.c_int),
                ("loss_zero", ctypes.c_double), ("loss_zero_val", ctypes.c_double),
                ("loss_first", ctypes.c_double), ("loss_last", ctypes.c_double),
                ("loss_val", ctypes.c_double), ("seconds", ctypes.c_double),
                ("spd", ctypes.c_int), ("refactor_seconds", ctypes.c_double), ("best_epoch", ctypes.c_int)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


GNN_P = 3169


class TuneReport(ctypes.Structure):
    _fields_ = [("candidates", ctypes.c_int), ("seconds", ctypes.c_double),
                ("us_before", ctypes.c_double * 2), ("us_after", ctypes.c_double * 2),
                ("top_h", ctypes.c_int * 2), ("fwd_cols", ctypes.c_int * 2), ("bwd_rows", ctypes.c_int * 2)]

    def as_dict(self):
        return {k: (list(getattr(self, k)) if k not in ("candidates", "seconds") else getattr(self, k))
                for k, _ in self._fields_}


class Plan(ctypes.Structure):
    """bido_plan: execution-plan options of an inner solve (see bido.h)."""
    _fields_ = [(k, ctypes.c_int) for k in ("top_h", "fwd_cols", "bwd_rows", "bwd_wide", "level_items",
                                            "sub_h", "sub_want", "sub_total", "bwd_group_max",
                                            "spmv_group")]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


def default_plan(**kw):
    """bido_default_plan with the given fields overridden."""
    q = Plan()
    lib.bido_default_plan(ctypes.byref(q))
    for k, v in kw.items():
        if not hasattr(q, k):
            raise KeyError(k)
        setattr(q, k, int(v))
    return q


class KProf(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 24), ("launches", ctypes.c_int64),
                ("ms", ctypes.c_double), ("bytes", ctypes.c_double)]


# name -> (restype, argtypes); mirrors include/bido.h and include/bido_host.h
ABI = {
    "bido_last_error": (ctypes.c_char_p, []),
    "bido_default_params": (None, [ctypes.POINTER(Params)]),
    "bido_create": (ctypes.c_int, [ctypes.POINTER(Mesh), ctypes.POINTER(Tissue),
                                   ctypes.POINTER(Params), ctypes.c_void_p,
                                   ctypes.POINTER(ctypes.c_void_p)]),
    "bido_destroy": (None, [ctypes.c_void_p]),
    "bido_get_info": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(Info)]),
    "bido_heart_nodes": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(_c_i64_p),
                                        ctypes.POINTER(ctypes.c_int64)]),
    "bido_step": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                 ctypes.c_void_p, ctypes.c_double, ctypes.c_int64,
                                 ctypes.POINTER(Stats)]),
    "bido_run": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                ctypes.c_void_p, ctypes.c_double, ctypes.c_int64,
                                ctypes.c_int64, ctypes.POINTER(Stats)]),
    "bido_solve": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                  ctypes.c_double, ctypes.POINTER(Stats)]),
    "bido_set_precision": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int]),
    "bido_set_solver": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_double, ctypes.c_int]),
    "bido_inner_solve": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p,
                                        ctypes.c_void_p]),
    "bido_inner_solve_noalloc": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p,
                                                ctypes.c_void_p, _c_i64_p]),
    "bido_set_precond": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int]),
    "bido_reset_guess": (ctypes.c_int, [ctypes.c_void_p]),
    "bido_set_dt": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_double, _c_double_p]),
    "bido_set_pk": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                   ctypes.c_double]),
    "bido_record": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_double, ctypes.c_int, _c_double_p,
                                   ctypes.c_int64]),
    "bido_record_read": (ctypes.c_int, [ctypes.c_void_p, _c_double_p, _c_double_p, _c_i64_p]),
    "bido_get_pk": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int),
                                   _c_double_p, _c_double_p]),
    "bido_set_graphs": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int]),
    "bido_autotune": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(TuneReport)]),
    "bido_default_plan": (None, [ctypes.POINTER(Plan)]),
    "bido_set_plan": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(Plan)]),
    "bido_get_plan": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(Plan)]),
    "bido_learn_collect": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                          ctypes.c_void_p, ctypes.c_double, ctypes.c_int64,
                                          ctypes.c_int64, ctypes.c_int, ctypes.POINTER(Stats)]),
    "bido_learn_samples": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int)]),
    "bido_learn_train": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                        ctypes.c_float, ctypes.c_uint64, ctypes.c_int,
                                        ctypes.POINTER(TrainStats)]),
    "bido_weights_io": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_float), ctypes.c_int,
                                       ctypes.c_int]),
    "bido_gnn_eval": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "bido_gnn_loss_grad": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                          ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_float)]),
    "bido_stencil_check": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                          ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_float)]),
    "bido_batch_create": (ctypes.c_int, [ctypes.POINTER(ctypes.c_void_p), ctypes.c_int, ctypes.c_int,
                                         ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p)]),
    "bido_batch_run": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p),
                                      ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(ctypes.c_void_p),
                                      ctypes.c_double, ctypes.c_int64, ctypes.c_int64, ctypes.POINTER(Stats),
                                      ctypes.POINTER(Stats)]),
    "bido_batch_destroy": (None, [ctypes.c_void_p]),
    "bido_batch_create_fused": (ctypes.c_int, [ctypes.POINTER(ctypes.c_void_p), ctypes.c_int, ctypes.c_void_p,
                                               ctypes.POINTER(ctypes.c_void_p)]),
    "bido_batch_set_graphs": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int]),
    "bido_batch_counters": (ctypes.c_int, [ctypes.c_void_p, _c_i64_p, _c_i64_p, _c_i64_p, _c_i64_p]),
    "bido_batch_info": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int),
                                       ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_double)]),
    "bido_profile": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int]),
    "bido_profile_read": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(KProf), ctypes.c_int,
                                         ctypes.POINTER(ctypes.c_int)]),
    "bido_batch_profile_read": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(KProf), ctypes.c_int,
                                         ctypes.POINTER(ctypes.c_int)]),
    "bido_batch_profile": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int]),
    "bido_host_last_error": (ctypes.c_char_p, []),
    "bido_host_setup": (ctypes.c_int, [ctypes.POINTER(Mesh), ctypes.POINTER(Tissue),
                                       ctypes.POINTER(Params), ctypes.POINTER(ctypes.c_void_p)]),
    "bido_host_free": (None, [ctypes.c_void_p]),
    "bido_host_csr": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, _c_i64_p, _c_i64_p,
                                     ctypes.POINTER(_c_i64_p), ctypes.POINTER(_c_i32_p),
                                     ctypes.POINTER(_c_double_p)]),
    "bido_host_vec": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, _c_i64_p,
                                     ctypes.POINTER(_c_double_p)]),
    "bido_host_pk_interval": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, _c_double_p]),
    "bido_host_pk_emulate": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                            _c_double_p, _c_double_p]),
    "bido_host_set_dt": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_double, ctypes.c_int]),
    "bido_host_locate": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, _c_double_p, _c_i64_p, _c_double_p]),
    "bido_host_index": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, _c_i64_p,
                                       ctypes.POINTER(_c_i64_p)]),
    "bido_host_factor_stats": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, _c_i64_p,
                                              ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)]),
    "bido_host_factor_nodes": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, _c_i64_p, _c_i32_p,
                                              ctypes.c_int64]),
    "bido_host_factor_emulate": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, _c_double_p,
                                                _c_double_p]),
    "bido_host_factor_plan": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(ctypes.c_int),
                                             ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int),
                                             _c_i64_p, _c_i64_p, _c_i64_p]),
    "bido_host_set_plan": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(Plan)]),
    "bido_host_amg_info": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(ctypes.c_int), _c_i64_p,
                                          _c_double_p, _c_double_p, ctypes.POINTER(ctypes.c_int)]),
    "bido_host_lambda_blocked": (ctypes.c_int, [ctypes.c_void_p, _c_i64_p, _c_i64_p, ctypes.POINTER(_c_i64_p),
                                                ctypes.POINTER(_c_i32_p), ctypes.POINTER(_c_double_p),
                                                ctypes.POINTER(_c_double_p)]),
    "bido_host_amg_level": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int, _c_i64_p,
                                           _c_i64_p, ctypes.POINTER(_c_i64_p), ctypes.POINTER(_c_i32_p),
                                           ctypes.POINTER(_c_double_p)]),
    "bido_host_amg_smoother": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int,
                                              ctypes.POINTER(_c_double_p), _c_double_p, _c_double_p,
                                              ctypes.POINTER(ctypes.c_int)]),
    "bido_host_amg_apply": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, _c_double_p, _c_double_p]),
    "bido_host_merge": (ctypes.c_int, [ctypes.POINTER(ctypes.c_void_p), ctypes.c_int,
                                       ctypes.POINTER(ctypes.c_void_p)]),
    "bido_host_factor_top": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(ctypes.c_int), _c_i64_p,
                                            ctypes.POINTER(ctypes.c_double), _c_i64_p, ctypes.POINTER(ctypes.c_int),
                                            _c_i64_p]),
    "bido_host_factor_apply": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, _c_double_p,
                                              _c_double_p]),
}


class BidoError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"libbido.so not built ({LIB_PATH}); run "
                          "`python -c 'import __graft_entry__ as g; g.build()'`")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in ABI.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


lib = _load()


def _check(code, host=False):
    if code != BIDO_OK:
        msg = (lib.bido_host_last_error() if host else lib.bido_last_error()) or b""
        raise BidoError(code, msg.decode())


def default_params(**kw):
    p = Params()
    lib.bido_default_params(ctypes.byref(p))
    for k, v in kw.items():
        setattr(p, k, v)
    return p


def _arr(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


def _marshal(cfg):
    """ctypes views of a workload dict (see workloads.meshes); the returned
    list keeps the numpy buffers alive."""
    keep = []

    def ptr(a, dtype):
        a = _arr(a, dtype)
        keep.append(a)
        return a.ctypes.data

    d = int(cfg["dim"])
    mesh = Mesh(d, len(cfg["xyz"]), ptr(cfg["xyz"], np.float64), len(cfg["elems"]),
                ptr(cfg["elems"], np.int32), ptr(cfg["region"], np.int8))
    si = (ctypes.c_double * 3)(*list(cfg["sigma_i"]) + [0.0] * (3 - d))
    se = (ctypes.c_double * 3)(*list(cfg["sigma_e"]) + [0.0] * (3 - d))
    tissue = Tissue(si, se, ptr(cfg["fibre"], np.float64), ptr(cfg["region_sigma"], np.float64),
                    len(cfg["region_sigma"]), ptr(cfg["stim_mask"], np.uint8),
                    float(cfg["stim_amp"]), float(cfg["stim_t0"]), float(cfg["stim_t1"]))
    return mesh, tissue, keep


def make_params(cfg, **kw):
    p = default_params(chi=float(cfg["chi"]), cm=float(cfg["cm"]), dt=float(cfg["dt"]),
                       tol=float(cfg.get("tol", 1e-10)))
    for k, v in kw.items():
        setattr(p, k, v)
    return p


class Solver:
    """One solver context on the current HIP device and torch stream."""

    def __init__(self, cfg, stream=None, **params):
        import torch
        if not torch.cuda.is_available():
            raise BidoError(-2, "no GPU visible to torch")
        self.torch = torch
        mesh, tissue, keep = _marshal(cfg)
        self.params = make_params(cfg, **params)
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        ctx = ctypes.c_void_p()
        _check(lib.bido_create(ctypes.byref(mesh), ctypes.byref(tissue),
                               ctypes.byref(self.params), ctypes.c_void_p(stream.cuda_stream),
                               ctypes.byref(ctx)))
        del keep
        self.ctx = ctx
        info = Info()
        _check(lib.bido_get_info(self.ctx, ctypes.byref(info)))
        self.info = info.as_dict()
        ids = _c_i64_p()
        nh = ctypes.c_int64()
        _check(lib.bido_heart_nodes(self.ctx, ctypes.byref(ids), ctypes.byref(nh)))
        self.heart_nodes = np.ctypeslib.as_array(ids, shape=(nh.value,)).copy()
        self.N = int(self.info["n_nodes"])
        self.NH = int(self.info["n_heart"])
        self.dt = float(self.params.dt)
        self.dim = int(cfg["dim"])
        self._rec_np, self._rec_act = 0, False

    def _dev(self, t, n):
        torch = self.torch
        if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64
                and t.is_contiguous() and t.numel() == n):
            raise BidoError(-1, f"expected a contiguous float64 CUDA tensor of {n} entries")
        return ctypes.c_void_p(t.data_ptr())

    def state(self, device="cuda"):
        """Rest state (V = 0, h = 1, U = 0) as float64 device tensors."""
        torch = self.torch
        v = torch.zeros(self.NH, dtype=torch.float64, device=device)
        w = torch.ones(self.NH, dtype=torch.float64, device=device)
        u = torch.zeros(self.N, dtype=torch.float64, device=device)
        return v, w, u

    def step(self, v, w, u, n):
        st = Stats()
        _check(lib.bido_step(self.ctx, self._dev(v, self.NH), self._dev(w, self.NH),
                             self._dev(u, self.N), self.dt, int(n), ctypes.byref(st)))
        return st.as_dict()

    def run(self, v, w, u, n0, n_steps, check=True):
        st = Stats()
        code = lib.bido_run(self.ctx, self._dev(v, self.NH), self._dev(w, self.NH),
                            self._dev(u, self.N), self.dt, int(n0), int(n_steps),
                            ctypes.byref(st))
        if check:
            _check(code)
        return st.as_dict()

    def solve(self, rhs, x, tol=0.0):
        st = Stats()
        n2 = self.N + self.NH
        _check(lib.bido_solve(self.ctx, self._dev(rhs, n2), self._dev(x, n2), float(tol),
                              ctypes.byref(st)))
        return st.as_dict()

    def inner_solve(self, which, b, x):
        n = self.N if which == FACTOR_P1 else self.NH
        _check(lib.bido_inner_solve(self.ctx, int(which), self._dev(b, n), self._dev(x, n)))

    def inner_solve_noalloc(self, which, b, x):
        """bido_inner_solve on the fixed workspace; returns the doubles it used."""
        n = self.N if which == FACTOR_P1 else self.NH
        need = ctypes.c_int64()
        _check(lib.bido_inner_solve_noalloc(self.ctx, int(which), self._dev(b, n), self._dev(x, n),
                                            ctypes.byref(need)))
        return need.value

    def set_dt(self, dt):
        """Change the time step; returns the seconds the change took."""
        sec = ctypes.c_double()
        _check(lib.bido_set_dt(self.ctx, float(dt), ctypes.byref(sec)))
        self.dt = float(dt)
        self.params.dt = float(dt)
        return sec.value

    def set_pk(self, kind, steps=3, lo=0.0, hi=0.0):
        """P_K by its factor (PK_CHOLESKY) or by `steps` Chebyshev-accelerated
        Jacobi steps on K_m over [lo, hi] (0, 0: estimated by the library)."""
        _check(lib.bido_set_pk(self.ctx, int(kind), int(steps), float(lo), float(hi)))

    def pk(self):
        kind, steps = ctypes.c_int(), ctypes.c_int()
        lo, hi = ctypes.c_double(), ctypes.c_double()
        _check(lib.bido_get_pk(self.ctx, ctypes.byref(kind), ctypes.byref(steps), ctypes.byref(lo),
                               ctypes.byref(hi)))
        return dict(kind=kind.value, steps=steps.value, lo=lo.value, hi=hi.value)

    def record(self, v_act=float("nan"), points=None, max_steps=0):
        """Record activation times (level v_act; NaN: none) and the potential
        u at probe points (n x dim) for the first max_steps later steps."""
        pts = np.ascontiguousarray(np.zeros((0, self.dim)) if points is None else points, dtype=np.float64)
        self._rec_np = len(pts)
        self._rec_act = not np.isnan(v_act)
        _check(lib.bido_record(self.ctx, float(v_act), len(pts),
                               pts.ctypes.data_as(_c_double_p) if len(pts) else None, int(max_steps)))

    def record_read(self):
        """(activation times or None, probe rows) as numpy arrays."""
        n = ctypes.c_int64()
        _check(lib.bido_record_read(self.ctx, None, None, ctypes.byref(n)))
        act = np.empty(self.NH) if self._rec_act else None
        rows = np.empty((n.value, self._rec_np))
        _check(lib.bido_record_read(self.ctx, act.ctypes.data_as(_c_double_p) if act is not None else None,
                                    rows.ctypes.data_as(_c_double_p) if rows.size else None, ctypes.byref(n)))
        return act, rows

    # ---- learned correction -------------------------------------------------
    def set_precond(self, precond):
        _check(lib.bido_set_precond(self.ctx, int(precond)))

    def reset_guess(self):
        """The next step starts a new span of states for its initial guess."""
        _check(lib.bido_reset_guess(self.ctx))

    def learn_collect(self, v, w, u, n0, n_steps, max_samples):
        st = Stats()
        _check(lib.bido_learn_collect(self.ctx, self._dev(v, self.NH), self._dev(w, self.NH),
                                      self._dev(u, self.N), self.dt, int(n0), int(n_steps),
                                      int(max_samples), ctypes.byref(st)))
        n = ctypes.c_int()
        _check(lib.bido_learn_samples(self.ctx, ctypes.byref(n)))
        d = st.as_dict()
        d["samples"] = n.value
        return d

    def learn_train(self, kind=LEARN_STENCIL, epochs=20, batch=8, lr=1e-3, seed=0, n_val=0):
        ts = TrainStats()
        _check(lib.bido_learn_train(self.ctx, int(kind), int(epochs), int(batch), float(lr), int(seed),
                                    int(n_val), ctypes.byref(ts)))
        return ts.as_dict()

    def weights(self):
        buf = (ctypes.c_float * GNN_P)()
        _check(lib.bido_weights_io(self.ctx, buf, GNN_P, 0))
        return np.ctypeslib.as_array(buf).astype(np.float64).copy()

    def set_weights(self, theta):
        buf = (ctypes.c_float * GNN_P)(*np.asarray(theta, dtype=np.float32).tolist())
        _check(lib.bido_weights_io(self.ctx, buf, GNN_P, 1))

    def gnn_eval(self, t):
        out = self.torch.zeros_like(t)
        _check(lib.bido_gnn_eval(self.ctx, self._dev(t, self.NH), ctypes.c_void_p(out.data_ptr())))
        return out

    def gnn_loss_grad(self, that, y):
        torch = self.torch
        for a in (that, y):
            if not (a.is_cuda and a.dtype == torch.float32 and a.numel() == self.NH and a.is_contiguous()):
                raise BidoError(-1, "expected contiguous float32 CUDA tensors of N_H entries")
        loss = ctypes.c_double()
        grad = (ctypes.c_float * GNN_P)()
        _check(lib.bido_gnn_loss_grad(self.ctx, ctypes.c_void_p(that.data_ptr()),
                                      ctypes.c_void_p(y.data_ptr()), ctypes.byref(loss), grad))
        return loss.value, np.ctypeslib.as_array(grad).astype(np.float64).copy()

    def stencil_check(self, zh, bh, grad=True):
        """(r, loss, grad) of the learned stencil with the current weights:
        r = C^ zh - bh (FP32 CUDA tensor), loss = |r|^2, grad = d loss / d theta."""
        torch = self.torch
        for a in (zh, bh):
            if not (a.is_cuda and a.dtype == torch.float32 and a.numel() == self.NH and a.is_contiguous()):
                raise BidoError(-1, "expected contiguous float32 CUDA tensors of N_H entries")
        r = torch.empty_like(zh)
        loss = ctypes.c_double()
        g = (ctypes.c_float * GNN_P)() if grad else None
        _check(lib.bido_stencil_check(self.ctx, ctypes.c_void_p(zh.data_ptr()), ctypes.c_void_p(bh.data_ptr()),
                                      ctypes.c_void_p(r.data_ptr()), ctypes.byref(loss), g))
        return r, loss.value, (np.ctypeslib.as_array(g).astype(np.float64).copy() if grad else None)

    def autotune(self, reps=10):
        """Time candidate plans of the inner solves on the device and keep the fastest."""
        r = TuneReport()
        _check(lib.bido_autotune(self.ctx, int(reps), ctypes.byref(r)))
        return r.as_dict()

    def set_plan(self, which, **kw):
        """Rebuild factor `which`'s sweep plan with bido_plan fields kw (others default)."""
        q = default_plan(**kw)
        _check(lib.bido_set_plan(self.ctx, int(which), ctypes.byref(q)))

    def get_plan(self, which):
        q = Plan()
        _check(lib.bido_get_plan(self.ctx, int(which), ctypes.byref(q)))
        return q.as_dict()

    def set_graphs(self, on):
        """True: always replay captured graphs, False: never, None: only in a batch."""
        _check(lib.bido_set_graphs(self.ctx, -1 if on is None else (1 if on else 0)))

    def set_precision(self, precision):
        _check(lib.bido_set_precision(self.ctx, int(precision)))

    def set_solver(self, tol=0.0, max_iter=0):
        _check(lib.bido_set_solver(self.ctx, float(tol), int(max_iter)))

    def profile(self, enable=True):
        _check(lib.bido_profile(self.ctx, 1 if enable else 0))

    def profile_read(self):
        buf = (KProf * 16)()
        n = ctypes.c_int()
        _check(lib.bido_profile_read(self.ctx, buf, 16, ctypes.byref(n)))
        return {buf[i].name.decode(): dict(launches=buf[i].launches, ms=buf[i].ms,
                                           bytes=buf[i].bytes) for i in range(min(n.value, 16))}

    def close(self):
        if getattr(self, "ctx", None):
            lib.bido_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Independent slices (Solver objects on one device) stepped together.

    While the batch exists the solvers run on its streams and must not be
    used on their own; close() gives them back.  fused=True lays the slices
    side by side in one union and runs each PCG phase as one launch for all
    of them (bido_batch_create_fused); otherwise the slices are spread over
    n_streams streams."""

    def __init__(self, solvers, n_streams=0, stream=None, fused=False):
        import torch
        self.torch = torch
        self.solvers = list(solvers)
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        arr = (ctypes.c_void_p * len(self.solvers))(*[s.ctx.value for s in self.solvers])
        b = ctypes.c_void_p()
        if fused:
            _check(lib.bido_batch_create_fused(arr, len(self.solvers), ctypes.c_void_p(stream.cuda_stream),
                                               ctypes.byref(b)))
        else:
            _check(lib.bido_batch_create(arr, len(self.solvers), int(n_streams),
                                         ctypes.c_void_p(stream.cuda_stream), ctypes.byref(b)))
        self.b = b

    def profile(self, on=True):
        """Fused batches: per-launch events on the union's sweeps (see profile_read)."""
        _check(lib.bido_batch_profile(self.b, 1 if on else 0))

    def profile_read(self):
        buf = (KProf * 16)()
        n = ctypes.c_int()
        _check(lib.bido_batch_profile_read(self.b, buf, 16, ctypes.byref(n)))
        return {buf[i].name.decode(): dict(launches=buf[i].launches, ms=buf[i].ms,
                                           bytes=buf[i].bytes) for i in range(min(n.value, 16))}

    def set_graphs(self, on):
        """Fused batches: replay captured iteration graphs (default) or not."""
        _check(lib.bido_batch_set_graphs(self.b, 1 if on else 0))

    def info(self):
        f, n, t = ctypes.c_int(), ctypes.c_int64(), ctypes.c_double()
        _check(lib.bido_batch_info(self.b, ctypes.byref(f), ctypes.byref(n), ctypes.byref(t)))
        return {"fused": bool(f.value), "n_union": n.value, "setup_seconds": t.value}

    def counters(self):
        """Fused batches: steps, PCG iterations launched, host waits inside the
        iterations, kernel launches of the captured iteration graphs."""
        v = [ctypes.c_int64() for _ in range(4)]
        _check(lib.bido_batch_counters(self.b, *[ctypes.byref(x) for x in v]))
        return dict(zip(("steps", "iterations", "host_waits", "kernels"), [x.value for x in v]))

    def run(self, states, n0, n_steps, check=True):
        """states: one (v, w, u) tuple of device tensors per solver.  Returns
        (total, per_slice) statistics dicts."""
        S = len(self.solvers)
        if len(states) != S:
            raise BidoError(-1, "one state per solver expected")
        v = (ctypes.c_void_p * S)(*[sv._dev(st[0], sv.NH).value for sv, st in zip(self.solvers, states)])
        w = (ctypes.c_void_p * S)(*[sv._dev(st[1], sv.NH).value for sv, st in zip(self.solvers, states)])
        u = (ctypes.c_void_p * S)(*[sv._dev(st[2], sv.N).value for sv, st in zip(self.solvers, states)])
        per = (Stats * S)()
        tot = Stats()
        code = lib.bido_batch_run(self.b, v, w, u, self.solvers[0].dt, int(n0), int(n_steps), per,
                                  ctypes.byref(tot))
        if check:
            _check(code)
        return tot.as_dict(), [p.as_dict() for p in per]

    def close(self):
        if getattr(self, "b", None):
            lib.bido_batch_destroy(self.b)
            self.b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class HostSetup:
    """Host-only set-up (no GPU) exposing assembled matrices, orderings and
    factor statistics for checks."""

    def __init__(self, cfg, **params):
        mesh, tissue, keep = _marshal(cfg)
        self.params = make_params(cfg, **params)
        h = ctypes.c_void_p()
        _check(lib.bido_host_setup(ctypes.byref(mesh), ctypes.byref(tissue),
                                   ctypes.byref(self.params), ctypes.byref(h)), host=True)
        del keep
        self.h = h

    @classmethod
    def merged(cls, parts):
        """Host object of the forest of the parts' factors (test hook): slice s
        at offset sum_{t<s} (N_t + N_H,t), P_1 first, then P_K."""
        obj = cls.__new__(cls)
        arr = (ctypes.c_void_p * len(parts))(*[p.h.value for p in parts])
        h = ctypes.c_void_p()
        _check(lib.bido_host_merge(arr, len(parts), ctypes.byref(h)), host=True)
        obj.h = h
        obj.parts = list(parts)
        obj.params = parts[0].params
        return obj

    def csr(self, which):
        import scipy.sparse as sp
        n = ctypes.c_int64()
        nnz = ctypes.c_int64()
        ptr, col, val = _c_i64_p(), _c_i32_p(), _c_double_p()
        _check(lib.bido_host_csr(self.h, which, ctypes.byref(n), ctypes.byref(nnz),
                                 ctypes.byref(ptr), ctypes.byref(col), ctypes.byref(val)), host=True)
        p = np.ctypeslib.as_array(ptr, shape=(n.value + 1,)).copy()
        c = np.ctypeslib.as_array(col, shape=(nnz.value,)).copy() if nnz.value else np.zeros(0, np.int32)
        v = np.ctypeslib.as_array(val, shape=(nnz.value,)).copy() if nnz.value else np.zeros(0)
        return sp.csr_matrix((v, c, p), shape=(n.value, n.value))

    def pk_emulate(self, steps, lo, hi, b):
        b = _arr(b, np.float64)
        x = np.zeros_like(b)
        _check(lib.bido_host_pk_emulate(self.h, int(steps), float(lo), float(hi), b.ctypes.data_as(_c_double_p),
                                        x.ctypes.data_as(_c_double_p)), host=True)
        return x

    def set_dt(self, dt, refactor=True):
        _check(lib.bido_host_set_dt(self.h, float(dt), 1 if refactor else 0), host=True)

    def locate(self, points):
        """(vertex ids, barycentric weights) of the element holding each point."""
        pts = np.ascontiguousarray(points, dtype=np.float64)
        n, d = pts.shape
        ids = np.empty((n, d + 1), dtype=np.int64)
        wts = np.empty((n, d + 1))
        _check(lib.bido_host_locate(self.h, n, pts.ctypes.data_as(_c_double_p), ids.ctypes.data_as(_c_i64_p),
                                    wts.ctypes.data_as(_c_double_p)), host=True)
        return ids, wts

    def pk_interval(self, lanczos_steps=PK_LANCZOS_STEPS):
        out = (ctypes.c_double * 6)()
        _check(lib.bido_host_pk_interval(self.h, int(lanczos_steps), out), host=True)
        keys = ("lo", "hi", "ritz_lo", "ritz_hi", "bound_lo", "bound_hi")
        return dict(zip(keys, list(out)))

    def vec(self, which):
        n = ctypes.c_int64()
        d = _c_double_p()
        _check(lib.bido_host_vec(self.h, which, ctypes.byref(n), ctypes.byref(d)), host=True)
        return np.ctypeslib.as_array(d, shape=(n.value,)).copy()

    def index(self, which):
        n = ctypes.c_int64()
        d = _c_i64_p()
        _check(lib.bido_host_index(self.h, which, ctypes.byref(n), ctypes.byref(d)), host=True)
        return np.ctypeslib.as_array(d, shape=(n.value,)).copy()

    def factor_stats(self, which):
        de = ctypes.c_int64()
        h, ms = ctypes.c_int(), ctypes.c_int()
        _check(lib.bido_host_factor_stats(self.h, which, ctypes.byref(de), ctypes.byref(h), ctypes.byref(ms)),
               host=True)
        return dict(entries=de.value, height=h.value, max_sep=ms.value)

    def factor_nodes(self, which):
        """(n_nodes, 5) int32: nI, nB, height, depth, parent."""
        n = ctypes.c_int64()
        _check(lib.bido_host_factor_nodes(self.h, which, ctypes.byref(n), None, 0), host=True)
        out = np.zeros((n.value, 5), dtype=np.int32)
        _check(lib.bido_host_factor_nodes(self.h, which, ctypes.byref(n),
                                          out.ctypes.data_as(_c_i32_p), n.value), host=True)
        return out

    def factor_emulate(self, which, b):
        """CPU emulation of the GPU sweep kernels over the device plan."""
        b = _arr(b, np.float64)
        x = np.zeros_like(b)
        _check(lib.bido_host_factor_emulate(self.h, which, b.ctypes.data_as(_c_double_p),
                                            x.ctypes.data_as(_c_double_p)), host=True)
        return x

    def factor_plan(self, which):
        hc, ns, nl = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        nf, nb, nsp = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        _check(lib.bido_host_factor_plan(self.h, which, ctypes.byref(hc), ctypes.byref(ns),
                                         ctypes.byref(nl), ctypes.byref(nf), ctypes.byref(nb),
                                         ctypes.byref(nsp)), host=True)
        return dict(hc=hc.value, n_sub=ns.value, n_levels=nl.value, n_fwd_items=nf.value,
                    n_bwd_items=nb.value, n_bwd_split=nsp.value)

    def amg_info(self, which):
        lv, nc, oc, sec, st = ctypes.c_int(), ctypes.c_int64(), ctypes.c_double(), ctypes.c_double(), ctypes.c_int()
        _check(lib.bido_host_amg_info(self.h, which, ctypes.byref(lv), ctypes.byref(nc), ctypes.byref(oc),
                                      ctypes.byref(sec), ctypes.byref(st)), host=True)
        return dict(levels=lv.value, n_coarse=nc.value, op_complexity=oc.value, seconds=sec.value,
                    smooth_steps=st.value)

    def lambda_blocked(self):
        """dict(ptr, col, val (n_pos x 2: S_1, S_i), gm) of Lambda's blocked
        form (copies), or None when it has none."""
        n, npos = ctypes.c_int64(), ctypes.c_int64()
        p, c, v, g = _c_i64_p(), _c_i32_p(), _c_double_p(), _c_double_p()
        code = lib.bido_host_lambda_blocked(self.h, ctypes.byref(n), ctypes.byref(npos), ctypes.byref(p),
                                            ctypes.byref(c), ctypes.byref(v), ctypes.byref(g))
        if code == -7:                      # BIDO_ERR_STATE: no blocked form
            return None
        _check(code, host=True)
        nn, m = n.value, npos.value
        return dict(ptr=np.ctypeslib.as_array(p, (nn + 1,)).copy(), col=np.ctypeslib.as_array(c, (m,)).copy(),
                    val=np.ctypeslib.as_array(v, (2 * m,)).copy().reshape(m, 2),
                    gm=np.ctypeslib.as_array(g, (nn,)).copy())

    def amg_level(self, which, level):
        """dict(A=scipy CSR, P=scipy CSR or None, dinv, lo, hi, steps) of one level
        (copies; steps: Chebyshev steps per smoothing on the level)."""
        import scipy.sparse as sp
        info = self.amg_info(which)
        out = {}
        for what, key in ((0, "A"), (1, "P")):
            if what == 1 and level + 1 == info["levels"]:
                out[key] = None
                continue
            n, nnz = ctypes.c_int64(), ctypes.c_int64()
            p, c, v = _c_i64_p(), _c_i32_p(), _c_double_p()
            _check(lib.bido_host_amg_level(self.h, which, level, what, ctypes.byref(n), ctypes.byref(nnz),
                                           ctypes.byref(p), ctypes.byref(c), ctypes.byref(v)), host=True)
            ptr = np.ctypeslib.as_array(p, shape=(n.value + 1,)).copy()
            col = np.ctypeslib.as_array(c, shape=(max(nnz.value, 1),))[:nnz.value].copy()
            val = np.ctypeslib.as_array(v, shape=(max(nnz.value, 1),))[:nnz.value].copy()
            ncols = n.value if what == 0 else self.amg_level_size(which, level + 1)
            out[key] = sp.csr_matrix((val, col, ptr), shape=(n.value, ncols))
        d = _c_double_p()
        lo, hi, st = ctypes.c_double(), ctypes.c_double(), ctypes.c_int()
        _check(lib.bido_host_amg_smoother(self.h, which, level, ctypes.byref(d), ctypes.byref(lo),
                                          ctypes.byref(hi), ctypes.byref(st)), host=True)
        out["dinv"] = np.ctypeslib.as_array(d, shape=(out["A"].shape[0],)).copy()
        out["lo"], out["hi"], out["steps"] = lo.value, hi.value, st.value
        return out

    def amg_level_size(self, which, level):
        n, nnz = ctypes.c_int64(), ctypes.c_int64()
        p, c, v = _c_i64_p(), _c_i32_p(), _c_double_p()
        _check(lib.bido_host_amg_level(self.h, which, level, 0, ctypes.byref(n), ctypes.byref(nnz),
                                       ctypes.byref(p), ctypes.byref(c), ctypes.byref(v)), host=True)
        return n.value

    def amg_apply(self, which, b):
        b = _arr(b, np.float64)
        x = np.zeros_like(b)
        _check(lib.bido_host_amg_apply(self.h, which, b.ctypes.data_as(_c_double_p),
                                       x.ctypes.data_as(_c_double_p)), host=True)
        return x

    def set_plan(self, which, **kw):
        """Plan options of the later factor_emulate / factor_plan / factor_top queries."""
        q = default_plan(**kw)
        _check(lib.bido_host_set_plan(self.h, int(which), ctypes.byref(q)), host=True)

    def factor_top(self, which):
        th, nt, sec = ctypes.c_int(), ctypes.c_int64(), ctypes.c_double()
        st, mr, nl = ctypes.c_int64(), ctypes.c_int(), ctypes.c_int64()
        _check(lib.bido_host_factor_top(self.h, which, ctypes.byref(th), ctypes.byref(nt), ctypes.byref(sec),
                                        ctypes.byref(st), ctypes.byref(mr), ctypes.byref(nl)), host=True)
        return dict(top_h=th.value, n_top=nt.value, seconds=sec.value, stored_entries=st.value,
                    max_rank=mr.value, n_lowrank=nl.value)

    def factor_apply(self, which, b):
        b = _arr(b, np.float64)
        x = np.zeros_like(b)
        _check(lib.bido_host_factor_apply(self.h, which, b.ctypes.data_as(_c_double_p),
                                          x.ctypes.data_as(_c_double_p)), host=True)
        return x

    def close(self):
        if getattr(self, "h", None):
            lib.bido_host_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
