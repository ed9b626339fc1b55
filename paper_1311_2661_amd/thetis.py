"""Python binding of libthetis (ctypes).

Argument marshalling only: every step of the solve runs in the library's
HIP kernels.  The functions carry the names of the C entry points declared
in ``include/thetis.h``; ``Instance`` and ``Solver`` wrap them with
ownership.  PyTorch supplies the device workspace (a uint8 tensor on the
current device) and the stream (torch's current stream).

There is no fallback: if the library is missing or no GPU is present the
calls raise.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

import numpy as np

try:
    import torch  # loads the HIP runtime that libthetis binds to
except ImportError:  # pragma: no cover - torch is part of the image
    torch = None

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libthetis.so")

OK, EINVAL, ENOMEM, EDEVICE, EDIVERGED, EBUSY, EBUDGET, EUNSUPPORTED = 0, -1, -2, -3, -4, -5, -6, -7
STEP_PER_COORD, STEP_GLOBAL_LMAX = 0, 1
SCHED_DET, SCHED_ASYNC = 0, 1
PREC_FP32, PREC_FP64, PREC_BF16X = 0, 1, 2
ROUND_VC_THRESH, ROUND_MIS_THRESH, ROUND_MIS_RAND, ROUND_MC_CKR = 1, 2, 3, 4
ROUND_COVER_THRESH, ROUND_COVER_RAND, ROUND_PACK_RAND = 5, 6, 7
ROUND_MAP_ARGMAX, ROUND_MAP_SAMPLE = 8, 9
LABEL_RULES = (ROUND_MC_CKR, ROUND_MAP_ARGMAX, ROUND_MAP_SAMPLE)
SHAPE_COVER, SHAPE_SET_COVER, SHAPE_PACK = 1, 2, 4

EXPORTED = [
    "thetis_params_default", "thetis_inst_create_csr", "thetis_inst_set_simplex_blocks",
    "thetis_inst_classes", "thetis_inst_rounding_shape", "thetis_inst_set_pairwise", "thetis_inst_destroy", "thetis_solver_workspace_bytes",
    "thetis_solver_create", "thetis_solver_create_static", "thetis_solver_reset", "thetis_set_beta",
    "thetis_set_step_rule",
    "thetis_run_epochs", "thetis_solver_autotune", "thetis_multiplier_step", "thetis_run_multipliers",
    "thetis_get_multipliers", "thetis_solver_save", "thetis_solver_load", "thetis_residual", "thetis_objective", "thetis_get_x",
    "thetis_set_y",
    "thetis_epoch", "thetis_round", "thetis_check_feasible", "thetis_set_timing",
    "thetis_get_timing", "thetis_epoch_traffic", "thetis_solver_destroy", "thetis_calibrate_random",
    "thetis_last_error",
    "thetis_batch_create", "thetis_batch_set", "thetis_batch_run", "thetis_batch_autotune",
    "thetis_batch_configure", "thetis_batch_set_window", "thetis_batch_destroy",
]


class ThetisError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"thetis error {code}: {msg}")
        self.code = code


class thetis_mul_stats(C.Structure):
    _fields_ = [("lp_value", C.c_double), ("linf", C.c_double), ("lp_dual", C.c_double),
                ("lp_gap", C.c_double), ("device_ms", C.c_double), ("alg_bytes", C.c_double)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


class thetis_params(C.Structure):
    _fields_ = [("beta", C.c_double), ("step_rule", C.c_int32), ("step_scale", C.c_double),
                ("prox", C.c_int32), ("ybar", C.c_void_p), ("ubar", C.c_void_p),
                ("schedule", C.c_int32), ("precision", C.c_int32),
                ("refresh_every", C.c_int32), ("seed", C.c_uint64)]


_lib = None


def lib():
    """Loads libthetis.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with paper_1311_2661_amd.build.build()")
        L = C.CDLL(LIB_PATH)
        vp, i32, i64, dbl, u64 = C.c_void_p, C.c_int32, C.c_int64, C.c_double, C.c_uint64
        P = C.POINTER
        sig = {
            "thetis_params_default": [P(thetis_params)],
            "thetis_inst_create_csr": [i64, i64, i64, vp, vp, vp, vp, vp, vp, vp, P(vp)],
            "thetis_inst_set_simplex_blocks": [vp, i64, i32, vp, vp],
            "thetis_inst_classes": [vp, P(i32), P(i64), vp],
            "thetis_inst_rounding_shape": [vp, P(i32), P(dbl)],
            "thetis_inst_set_pairwise": [vp, i64, vp, vp],
            "thetis_inst_destroy": [vp],
            "thetis_solver_workspace_bytes": [vp, P(thetis_params), P(C.c_size_t)],
            "thetis_solver_create": [vp, P(thetis_params), vp, C.c_size_t, vp, P(vp)],
            "thetis_solver_create_static": [vp, P(thetis_params), vp, P(vp)],
            "thetis_solver_reset": [vp],
            "thetis_set_beta": [vp, dbl],
            "thetis_set_step_rule": [vp, i32, dbl],
            "thetis_run_epochs": [vp, i32, dbl, P(i32)],
            "thetis_solver_autotune": [vp, i32, vp],
            "thetis_multiplier_step": [vp, i32, dbl, P(thetis_mul_stats)],
            "thetis_run_multipliers": [vp, i32, i32, dbl, dbl, dbl, dbl, dbl, i32, P(i32), P(i64),
                                       P(thetis_mul_stats)],
            "thetis_get_multipliers": [vp, vp, vp],
            "thetis_solver_save": [vp, vp, P(C.c_size_t)],
            "thetis_solver_load": [vp, vp, C.c_size_t],
            "thetis_residual": [vp, P(dbl), P(dbl), P(dbl)],
            "thetis_objective": [vp, P(dbl), P(dbl), P(dbl), P(dbl)],
            "thetis_get_x": [vp, vp, vp],
            "thetis_set_y": [vp, vp],
            "thetis_epoch": [vp, P(i64)],
            "thetis_round": [vp, i32, u64, i32, vp, P(dbl), vp],
            "thetis_check_feasible": [vp, i32, vp, P(i32), P(i64)],
            "thetis_set_timing": [vp, i32],
            "thetis_get_timing": [vp, i32, P(dbl), P(i64), P(dbl)],
            "thetis_epoch_traffic": [vp, P(dbl), P(dbl), P(i64)],
            "thetis_solver_destroy": [vp],
            "thetis_calibrate_random": [i32, i32, vp, vp],
            "thetis_batch_create": [i32, vp, i32, i32, vp, P(vp)],
            "thetis_batch_set": [vp, i32, vp],
            "thetis_batch_run": [vp, i32, dbl, vp, vp],
            "thetis_batch_autotune": [vp, i32, vp],
            "thetis_batch_configure": [vp, i32, i32, i32, i32],
            "thetis_batch_set_window": [vp, i32],
            "thetis_batch_destroy": [vp],
        }
        for name, args in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = i32
        L.thetis_last_error.argtypes = []
        L.thetis_last_error.restype = C.c_char_p
        _lib = L
    return _lib


def _check(code: int) -> None:
    if code != OK:
        raise ThetisError(code, lib().thetis_last_error().decode(errors="replace"))


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else C.c_void_p(a.ctypes.data)


def _c(a, dtype):
    return None if a is None else np.ascontiguousarray(a, dtype=dtype)


# ------------------------------------------------------------ C-named calls

def thetis_last_error() -> str:
    return lib().thetis_last_error().decode(errors="replace")


def thetis_params_default() -> thetis_params:
    p = thetis_params()
    _check(lib().thetis_params_default(C.byref(p)))
    return p


def thetis_inst_create_csr(m, n, nnz, row_ptr, col_idx, val, b, c, u, sense):
    keep = [_c(row_ptr, np.int64), _c(col_idx, np.int32), _c(val, np.float64), _c(b, np.float64),
            _c(c, np.float64), _c(u, np.float64), _c(sense, np.int8)]
    h = C.c_void_p()
    _check(lib().thetis_inst_create_csr(m, n, nnz, *[_ptr(a) for a in keep], C.byref(h)))
    return h


def thetis_inst_set_simplex_blocks(h, nblocks, k, first_col, fixed_label=None):
    f = _c(first_col, np.int64)
    fx = _c(fixed_label, np.int32)
    _check(lib().thetis_inst_set_simplex_blocks(h, nblocks, k, _ptr(f), _ptr(fx)))


def thetis_inst_set_pairwise(h, ends, first_col):
    e = np.ascontiguousarray(ends, dtype=np.int32).reshape(-1)
    f = np.ascontiguousarray(first_col, dtype=np.int64)
    _check(lib().thetis_inst_set_pairwise(h, f.size, _ptr(e), _ptr(f)))


def thetis_inst_rounding_shape(h):
    fl, q = C.c_int32(), C.c_double()
    _check(lib().thetis_inst_rounding_shape(h, C.byref(fl), C.byref(q)))
    return fl.value, q.value


def thetis_inst_classes(h):
    nc, nu = C.c_int32(), C.c_int64()
    _check(lib().thetis_inst_classes(h, C.byref(nc), C.byref(nu), None))
    out = np.zeros(nu.value, np.int32)
    _check(lib().thetis_inst_classes(h, None, None, _ptr(out)))
    return nc.value, nu.value, out


def thetis_inst_destroy(h):
    _check(lib().thetis_inst_destroy(h))


def thetis_solver_workspace_bytes(h, params: thetis_params) -> int:
    b = C.c_size_t()
    _check(lib().thetis_solver_workspace_bytes(h, C.byref(params), C.byref(b)))
    return b.value


def thetis_solver_create(h, params: thetis_params, workspace_ptr: int, ws_bytes: int, stream_ptr: int):
    s = C.c_void_p()
    _check(lib().thetis_solver_create(h, C.byref(params), C.c_void_p(workspace_ptr or None), ws_bytes,
                                      C.c_void_p(stream_ptr or None), C.byref(s)))
    return s


def thetis_solver_create_static(h, params: thetis_params, stream_ptr: int):
    s = C.c_void_p()
    _check(lib().thetis_solver_create_static(h, C.byref(params), C.c_void_p(stream_ptr or None), C.byref(s)))
    return s


def thetis_solver_reset(s):
    _check(lib().thetis_solver_reset(s))


def thetis_set_beta(s, beta: float):
    _check(lib().thetis_set_beta(s, beta))


def thetis_set_step_rule(s, rule: int, scale: float = 1.0):
    _check(lib().thetis_set_step_rule(s, rule, scale))


def thetis_run_epochs(s, max_epochs: int, gap_tol: float = 0.0) -> int:
    done = C.c_int32()
    _check(lib().thetis_run_epochs(s, max_epochs, gap_tol, C.byref(done)))
    return done.value


def thetis_multiplier_step(s, move_centre: bool = False, new_beta: float = 0.0) -> dict:
    st = thetis_mul_stats()
    _check(lib().thetis_multiplier_step(s, int(move_centre), float(new_beta), C.byref(st)))
    return st.as_dict()


def thetis_run_multipliers(s, max_outer: int, inner_epochs: int, inner_gap_tol: float = 0.0,
                           beta_growth: float = 1.0, beta_max: float = 0.0, feas_tol: float = 0.0,
                           lp_gap_tol: float = 0.0, move_centre: bool = False):
    outer, epochs, st = C.c_int32(), C.c_int64(), thetis_mul_stats()
    _check(lib().thetis_run_multipliers(s, max_outer, inner_epochs, inner_gap_tol, beta_growth,
                                        beta_max, feas_tol, lp_gap_tol, int(move_centre),
                                        C.byref(outer), C.byref(epochs), C.byref(st)))
    return outer.value, epochs.value, st.as_dict()


def thetis_get_multipliers(s, m: int, n: int, multiplier: bool = True, centre: bool = False):
    u = np.zeros(m) if multiplier else None
    yb = np.zeros(n + m) if centre else None
    _check(lib().thetis_get_multipliers(s, _ptr(u), _ptr(yb)))
    return u, yb


def thetis_solver_save(s) -> bytes:
    n = C.c_size_t()
    _check(lib().thetis_solver_save(s, None, C.byref(n)))
    buf = C.create_string_buffer(n.value)
    _check(lib().thetis_solver_save(s, buf, C.byref(n)))
    return buf.raw[: n.value]


def thetis_solver_load(s, blob: bytes):
    buf = C.create_string_buffer(blob, len(blob))
    _check(lib().thetis_solver_load(s, buf, len(blob)))


def thetis_residual(s):
    a, b, c = C.c_double(), C.c_double(), C.c_double()
    _check(lib().thetis_residual(s, C.byref(a), C.byref(b), C.byref(c)))
    return a.value, b.value, c.value


def thetis_objective(s):
    a, b, c, d = C.c_double(), C.c_double(), C.c_double(), C.c_double()
    _check(lib().thetis_objective(s, C.byref(a), C.byref(b), C.byref(c), C.byref(d)))
    return a.value, b.value, c.value, d.value


def thetis_get_x(s, n: int, m: int = 0, slacks: bool = False):
    x = np.zeros(n)
    sl = np.zeros(m) if slacks else None
    _check(lib().thetis_get_x(s, _ptr(x), _ptr(sl)))
    return (x, sl) if slacks else x


def thetis_set_y(s, y):
    y = _c(y, np.float64)
    _check(lib().thetis_set_y(s, _ptr(y)))


def thetis_epoch(s) -> int:
    e = C.c_int64()
    _check(lib().thetis_epoch(s, C.byref(e)))
    return e.value


def thetis_round(s, rule: int, seed: int, reps: int, nsol: int):
    sol = np.zeros(nsol, np.int32)
    cost = C.c_double()
    aux = np.zeros(2)
    _check(lib().thetis_round(s, rule, seed, reps, _ptr(sol), C.byref(cost), _ptr(aux)))
    return sol, cost.value, aux


def thetis_check_feasible(s, rule: int, sol=None):
    sl = _c(sol, np.int32)
    f, nv = C.c_int32(), C.c_int64()
    _check(lib().thetis_check_feasible(s, rule, _ptr(sl), C.byref(f), C.byref(nv)))
    return bool(f.value), nv.value


def thetis_set_timing(s, every: int):
    _check(lib().thetis_set_timing(s, int(every)))


K_SWEEP_COLUMNS, K_SWEEP_BLOCK, K_SWEEP_SLACK, K_REFRESH = 0, 1, 2, 3
KERNEL_NAMES = {K_SWEEP_COLUMNS: "k_sweep", K_SWEEP_BLOCK: "k_sweep_block",
                K_SWEEP_SLACK: "k_sweep_slack", K_REFRESH: "refresh (k_rows+k_dual+k_finalize)"}


def thetis_get_timing(s, kind: int):
    a, b, c = C.c_double(), C.c_int64(), C.c_double()
    _check(lib().thetis_get_timing(s, kind, C.byref(a), C.byref(b), C.byref(c)))
    return dict(ms=a.value, launches=b.value, alg_bytes=c.value)


def thetis_epoch_traffic(s):
    a, b, c = C.c_double(), C.c_double(), C.c_int64()
    _check(lib().thetis_epoch_traffic(s, C.byref(a), C.byref(b), C.byref(c)))
    return dict(sweep_bytes=a.value, refresh_bytes=b.value, updates_per_epoch=c.value)


def thetis_solver_destroy(s):
    _check(lib().thetis_solver_destroy(s))


def _hv(h):
    if h is None:
        return None
    return h.value if isinstance(h, C.c_void_p) else h


def thetis_batch_create(capacity: int, solver_handles, precision: int, unit_values: bool, stream_ptr: int = 0):
    arr = None
    if solver_handles is not None:
        arr = (C.c_void_p * capacity)(*[_hv(h) for h in solver_handles])
    b = C.c_void_p()
    _check(lib().thetis_batch_create(capacity, None if arr is None else C.cast(arr, C.c_void_p), precision,
                                     int(unit_values), C.c_void_p(stream_ptr or None), C.byref(b)))
    return b


def thetis_batch_set(b, slot: int, solver_handle):
    _check(lib().thetis_batch_set(b, slot, C.c_void_p(_hv(solver_handle))))


def thetis_batch_run(b, count: int, max_epochs: int, gap_tol: float = 0.0):
    done = np.zeros(count, np.int32)
    status = np.zeros(count, np.int32)
    _check(lib().thetis_batch_run(b, max_epochs, gap_tol, _ptr(done), _ptr(status)))
    return done, status


def thetis_calibrate_random(words_log2: int, iters: int = 10):
    """Random-access calibration on the current torch stream: mean ms per pass
    of (random gather, random read-modify-write, copy, random
    read-modify-write inside each XCD's eighth) over 2^words_log2 4-byte
    words."""
    import torch
    out = np.zeros(4, np.float64)
    st = torch.cuda.current_stream().cuda_stream
    _check(lib().thetis_calibrate_random(words_log2, iters, C.c_void_p(st), _ptr(out)))
    return tuple(float(v) for v in out)


def thetis_batch_autotune(b, epochs_per_candidate: int = 2):
    ch = np.zeros(4, np.int32)
    _check(lib().thetis_batch_autotune(b, epochs_per_candidate, _ptr(ch)))
    return tuple(int(v) for v in ch)


def thetis_batch_configure(b, widen: int, grid_mult: int, strided: int = 1, cols: int = 1):
    _check(lib().thetis_batch_configure(b, widen, grid_mult, strided, cols))


def thetis_batch_destroy(b):
    _check(lib().thetis_batch_destroy(b))


# ------------------------------------------------------------ owning wrappers

class Instance:
    """An LP instance (``instances.LPInstance``) handed to the library."""

    def __init__(self, inst):
        self.inst = inst
        self.h = thetis_inst_create_csr(inst.m, inst.n, inst.nnz, inst.row_ptr, inst.col_idx,
                                        inst.val, inst.b, inst.c, inst.u, inst.sense)
        if inst.block_first_col is not None:
            thetis_inst_set_simplex_blocks(self.h, len(inst.block_first_col), inst.block_k,
                                           inst.block_first_col, inst.fixed_label)
        if getattr(inst, "pair_ends", None) is not None:
            thetis_inst_set_pairwise(self.h, inst.pair_ends, inst.pair_first)
        self.m, self.n = inst.m, inst.n

    def classes(self):
        return thetis_inst_classes(self.h)

    def rounding_shape(self):
        """(flags, q(P)): SHAPE_* bits the general roundings accept, and the
        covering lemma's q."""
        return thetis_inst_rounding_shape(self.h)

    def close(self):
        if getattr(self, "h", None):
            thetis_inst_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Solver:
    """Device state of one solve.  The workspace is a torch uint8 tensor on
    the current device (or, with ``static_workspace``, the library's fixed
    per-device array: thetis_solver_create_static, no allocation); launches
    go to torch's current stream."""

    def __init__(self, instance: Instance, beta: float = 10.0, step_rule: int = STEP_PER_COORD,
                 step_scale: float = 1.0, prox: bool = False, ybar=None, ubar=None,
                 schedule: int = SCHED_DET, precision: int = PREC_FP32, refresh_every: int = 5,
                 seed: int = 0, device=None, static_workspace: bool = False):
        if torch is None or not torch.cuda.is_available():
            raise RuntimeError("libthetis needs a HIP device")
        self.instance = instance
        p = thetis_params_default()
        p.beta, p.step_rule, p.step_scale, p.prox = beta, step_rule, step_scale, int(prox)
        self._yb = _c(ybar, np.float64)
        self._ub = _c(ubar, np.float64)
        p.ybar = None if self._yb is None else self._yb.ctypes.data
        p.ubar = None if self._ub is None else self._ub.ctypes.data
        p.schedule, p.precision, p.refresh_every, p.seed = schedule, precision, refresh_every, seed
        self.params = p
        dev = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
        with torch.cuda.device(dev):
            self.stream = torch.cuda.current_stream(dev)
            if static_workspace:
                self.workspace = None
                self.h = thetis_solver_create_static(instance.h, p, self.stream.cuda_stream)
            else:
                nbytes = thetis_solver_workspace_bytes(instance.h, p)
                self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=dev)
                self.h = thetis_solver_create(instance.h, p, self.workspace.data_ptr(), nbytes,
                                              self.stream.cuda_stream)
        self.n, self.m = instance.n, instance.m
        self.nclasses = thetis_inst_classes(instance.h)[0]
        bf = instance.inst.block_first_col
        self.nblocks = 0 if bf is None else len(bf)
        v = instance.inst.val
        self.instance_unit_values = v is None or bool(np.all(v == 1.0))

    # thin forwards
    def reset(self):
        thetis_solver_reset(self.h)

    def run(self, epochs: int, gap_tol: float = 0.0) -> int:
        return thetis_run_epochs(self.h, epochs, gap_tol)

    def autotune(self, epochs_per_candidate: int = 2) -> list:
        """Per-class columns per lane group, chosen by timing real epochs
        (1 + 3 x epochs_per_candidate epochs of the solve)."""
        nc = self.nclasses
        out = np.zeros(max(nc, 1), np.int32)
        _check(lib().thetis_solver_autotune(self.h, epochs_per_candidate, _ptr(out)))
        return [int(v) for v in out[:nc]]

    def multiplier_step(self, move_centre: bool = False, beta: float = 0.0) -> dict:
        """ubar -= beta (A y - b); ybar <- y with move_centre; then beta <- beta
        when > 0.  Returns the step's figures at the current y."""
        return thetis_multiplier_step(self.h, move_centre, beta)

    def run_multipliers(self, max_outer: int, inner_epochs: int, inner_gap_tol: float = 0.0,
                        beta_growth: float = 1.0, beta_max: float = 0.0, feas_tol: float = 0.0,
                        lp_gap_tol: float = 0.0, move_centre: bool = False):
        """Outer loop: (outer steps done, epochs done, last step's figures)."""
        return thetis_run_multipliers(self.h, max_outer, inner_epochs, inner_gap_tol, beta_growth,
                                      beta_max, feas_tol, lp_gap_tol, move_centre)

    @property
    def ubar(self) -> np.ndarray:
        return thetis_get_multipliers(self.h, self.m, self.n)[0]

    @property
    def ybar(self) -> np.ndarray:
        return thetis_get_multipliers(self.h, self.m, self.n, multiplier=False, centre=True)[1]

    def save(self) -> bytes:
        """Checkpoint of the device state (bit-exact resume)."""
        return thetis_solver_save(self.h)

    def load(self, blob: bytes):
        thetis_solver_load(self.h, blob)

    def residual(self):
        linf, l2, viol = thetis_residual(self.h)
        return dict(linf=linf, l2=l2, max_viol=viol)

    def objective(self):
        lp, F, phi, gap = thetis_objective(self.h)
        return dict(lp_value=lp, F=F, dual_bound=phi, gap=gap)

    def metrics(self) -> dict:
        d = self.objective()
        d.update(self.residual())
        return d

    @property
    def x(self) -> np.ndarray:
        return thetis_get_x(self.h, self.n)

    @property
    def y(self) -> np.ndarray:
        x, s = thetis_get_x(self.h, self.n, self.m, slacks=True)
        return np.concatenate([x, s])

    @y.setter
    def y(self, v):
        thetis_set_y(self.h, v)

    @property
    def epoch(self) -> int:
        return thetis_epoch(self.h)

    def round(self, rule: int, seed: int = 0, reps: int = 1):
        nsol = self.nblocks if rule in LABEL_RULES else self.n
        return thetis_round(self.h, rule, seed, reps, nsol)

    def check(self, rule: int, sol=None):
        return thetis_check_feasible(self.h, rule, sol)

    def set_timing(self, every: int = 1):
        """HIP-event timing of every launch of every `every`-th epoch (0: off)."""
        thetis_set_timing(self.h, int(every))

    def timing(self) -> dict:
        return {KERNEL_NAMES[k]: thetis_get_timing(self.h, k) for k in KERNEL_NAMES}

    def traffic(self) -> dict:
        return thetis_epoch_traffic(self.h)

    def close(self):
        if getattr(self, "h", None):
            thetis_solver_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Slots of solvers advanced by one launch sequence per epoch.

    Batch(solvers) fills the slots with the given solvers; Batch(capacity=k,
    precision=..., unit_values=...) starts empty (see ``set``)."""

    def __init__(self, solvers=None, stream=None, capacity=None, precision=None, unit_values=None):
        self.solvers = list(solvers) if solvers is not None else []
        cap = capacity if capacity is not None else len(self.solvers)
        self.solvers += [None] * (cap - len(self.solvers))
        first = next((s for s in self.solvers if s is not None), None)
        if precision is None:
            precision = first.params.precision if first is not None else PREC_FP32
        if unit_values is None:
            unit_values = first.instance_unit_values if first is not None else True
        sp = 0 if stream is None else stream.cuda_stream
        self.capacity = cap
        self.h = thetis_batch_create(cap, [None if s is None else s.h for s in self.solvers], precision,
                                     unit_values, sp)
        self.last_status = None

    def set(self, slot: int, solver):
        thetis_batch_set(self.h, slot, None if solver is None else solver.h)
        self.solvers[slot] = solver

    def run(self, max_epochs: int, gap_tol: float = 0.0) -> np.ndarray:
        done, status = thetis_batch_run(self.h, self.capacity, max_epochs, gap_tol)
        self.last_status = status
        return done

    def autotune(self, epochs_per_candidate: int = 2):
        return thetis_batch_autotune(self.h, epochs_per_candidate)

    def configure(self, widen: int, grid_mult: int, strided: int = 1, cols: int = 1):
        thetis_batch_configure(self.h, widen, grid_mult, strided, cols)

    def set_window(self, window: int):
        """At most `window` instances run at once (0: all); the others wait
        in slot order and start on the device as running ones retire."""
        _check(lib().thetis_batch_set_window(self.h, window))

    def close(self):
        if getattr(self, "h", None):
            thetis_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
