"""ctypes shim over the plain serial FP64 oracle (``thetis_oracle.c``).

TEST INFRASTRUCTURE ONLY: the test suite, the package smoke check and the
benchmark's CPU-baseline leg are the only callers.  Nothing here is shared
with the HIP library; the oracle is built from its own C source with gcc.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "thetis_oracle.c")
# THETIS_ORACLE_LIB names another build of the oracle to load instead: the
# mutation check of the pins points it at builds with a planted mistake
LIB = os.environ.get("THETIS_ORACLE_LIB") or os.path.join(HERE, "liborc.so")

SCHED_DET, SCHED_PERM, SCHED_UNIFORM = 0, 1, 2
STEP_PER_COORD, STEP_GLOBAL_LMAX = 0, 1
RULE_VC_THRESH, RULE_MIS_THRESH, RULE_MIS_RAND, RULE_MC_CKR = 1, 2, 3, 4
RULE_COVER_THRESH, RULE_COVER_RAND, RULE_PACK_RAND = 5, 6, 7
RULE_MAP_ARGMAX, RULE_MAP_SAMPLE = 8, 9


def build(force: bool = False) -> str:
    """Compile the oracle with gcc: -O2, no contraction, strict IEEE."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
                               "-shared", "-o", tmp, SRC, "-lm"])
        os.replace(tmp, LIB)
    return LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = C.CDLL(LIB)
        P = C.c_void_p
        dp = np.ctypeslib.ndpointer(np.float64, flags="C")
        i64p = np.ctypeslib.ndpointer(np.int64, flags="C")
        i32p = np.ctypeslib.ndpointer(np.int32, flags="C")
        i8p = np.ctypeslib.ndpointer(np.int8, flags="C")
        u64p = np.ctypeslib.ndpointer(np.uint64, flags="C")
        L.orc_philox.argtypes = [u64p, u64p, u64p]
        L.orc_lp_create.restype = P
        L.orc_lp_create.argtypes = [C.c_int64, C.c_int64, i64p, i32p, C.c_void_p, dp, dp,
                                    C.c_void_p, C.c_void_p]
        L.orc_lp_free.argtypes = [P]
        L.orc_lp_set_blocks.argtypes = [P, C.c_int64, C.c_int32, i64p, C.c_void_p]
        L.orc_num_units.restype = C.c_int64
        L.orc_num_units.argtypes = [P]
        L.orc_num_classes.restype = C.c_int32
        L.orc_num_classes.argtypes = [P]
        L.orc_units.argtypes = [P, i8p, i64p, i32p]
        L.orc_class_order.argtypes = [P, C.c_uint64, C.c_int64, i32p]
        L.orc_simplex_project.argtypes = [dp, C.c_int32, dp]
        L.orc_solver_create.restype = P
        L.orc_solver_create.argtypes = [P, C.c_double, C.c_int32, C.c_double, C.c_int32,
                                        C.c_void_p, C.c_void_p, C.c_int32, C.c_uint64]
        L.orc_solver_free.argtypes = [P]
        L.orc_run_epochs.argtypes = [P, C.c_int32, C.c_int32, C.c_void_p]
        L.orc_trace_epoch.restype = C.c_int64
        L.orc_trace_epoch.argtypes = [P, dp, C.c_int64]
        L.orc_step_unit.argtypes = [P, C.c_int64]
        L.orc_get_y.argtypes = [P, dp]
        L.orc_get_r.argtypes = [P, dp]
        L.orc_set_y.argtypes = [P, dp]
        L.orc_epoch.restype = C.c_int64
        L.orc_epoch.argtypes = [P]
        L.orc_set_epoch.argtypes = [P, C.c_int64]
        L.orc_lmax.restype = C.c_double
        L.orc_lmax.argtypes = [P]
        L.orc_penalty.restype = C.c_double
        L.orc_penalty.argtypes = [P]
        L.orc_metrics.argtypes = [P, dp]
        L.orc_multiplier_step.argtypes = [P, C.c_int32, C.c_double, dp]
        L.orc_get_ubar.argtypes = [P, dp]
        L.orc_get_ybar.argtypes = [P, dp]
        L.orc_beta.restype = C.c_double
        L.orc_beta.argtypes = [P]
        L.orc_round.restype = C.c_int32
        L.orc_round.argtypes = [P, dp, C.c_int32, C.c_uint64, C.c_int32, i32p, C.POINTER(C.c_double), dp]
        L.orc_lp_set_pairwise.argtypes = [P, C.c_int64, i32p, i64p]
        L.orc_cover_q.restype = C.c_double
        L.orc_cover_q.argtypes = [P]
        L.orc_check.restype = C.c_int32
        L.orc_check.argtypes = [P, C.c_int32, i32p, C.POINTER(C.c_int32), C.POINTER(C.c_int64)]
        _lib = L
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def philox(ctr, key) -> np.ndarray:
    out = np.zeros(4, dtype=np.uint64)
    lib().orc_philox(np.asarray(ctr, dtype=np.uint64), np.asarray(key, dtype=np.uint64), out)
    return out


def simplex_project(v) -> np.ndarray:
    v = np.ascontiguousarray(v, dtype=np.float64)
    out = np.zeros_like(v)
    lib().orc_simplex_project(v, v.size, out)
    return out


class OracleLP:
    """The LP with its slack columns, CSC and DET colour classes."""

    def __init__(self, inst):
        L = lib()
        self.inst = inst
        self._keep = [np.ascontiguousarray(inst.row_ptr, dtype=np.int64),
                      np.ascontiguousarray(inst.col_idx, dtype=np.int32),
                      None if inst.val is None else np.ascontiguousarray(inst.val, dtype=np.float64),
                      np.ascontiguousarray(inst.b, dtype=np.float64),
                      np.ascontiguousarray(inst.c, dtype=np.float64),
                      np.ascontiguousarray(inst.u, dtype=np.float64),
                      np.ascontiguousarray(inst.sense, dtype=np.int8)]
        rp, ci, v, b, c, u, s = self._keep
        self.h = L.orc_lp_create(inst.m, inst.n, rp, ci, _ptr(v), b, c, _ptr(u), _ptr(s))
        if not self.h:
            raise ValueError("oracle rejected the instance")
        if inst.block_first_col is not None:
            first = np.ascontiguousarray(inst.block_first_col, dtype=np.int64)
            fx = None if inst.fixed_label is None else np.ascontiguousarray(inst.fixed_label, dtype=np.int32)
            if L.orc_lp_set_blocks(self.h, first.size, inst.block_k, first, _ptr(fx)) != 0:
                raise ValueError("oracle rejected the blocks")
            self._keep += [first, fx]
        if getattr(inst, "pair_ends", None) is not None:
            pe = np.ascontiguousarray(inst.pair_ends, dtype=np.int32).reshape(-1)
            pf = np.ascontiguousarray(inst.pair_first, dtype=np.int64)
            if L.orc_lp_set_pairwise(self.h, pf.size, pe, pf) != 0:
                raise ValueError("oracle rejected the pairwise factors")
            self._keep += [pe, pf]
        self.m, self.n, self.N = inst.m, inst.n, inst.n + inst.m

    def __del__(self):
        # at interpreter exit the module's globals may already be gone
        if getattr(self, "h", None) and callable(globals().get("lib")):
            lib().orc_lp_free(self.h)
            self.h = None

    def units(self):
        L = lib()
        U = L.orc_num_units(self.h)
        kind = np.zeros(U, np.int8)
        uid = np.zeros(U, np.int64)
        col = np.zeros(U, np.int32)
        L.orc_units(self.h, kind, uid, col)
        return kind, uid, col

    @property
    def nclasses(self) -> int:
        return lib().orc_num_classes(self.h)

    def class_order(self, seed: int, epoch: int) -> np.ndarray:
        out = np.zeros(self.nclasses, np.int32)
        lib().orc_class_order(self.h, seed, epoch, out)
        return out

    def cover_q(self) -> float:
        """q(P) of the covering lemma (-1: not an integer covering program)."""
        return lib().orc_cover_q(self.h)

    def round(self, x, rule: int, seed: int = 0, reps: int = 1):
        x = np.ascontiguousarray(x, dtype=np.float64)
        labels = rule in (RULE_MC_CKR, RULE_MAP_ARGMAX, RULE_MAP_SAMPLE)
        nsol = self.inst.fixed_label.size if labels else self.n
        sol = np.zeros(nsol, np.int32)
        cost = C.c_double()
        aux = np.zeros(4)
        if lib().orc_round(self.h, x, rule, seed, reps, sol, C.byref(cost), aux) != 0:
            raise ValueError("rule does not fit this instance")
        return sol, cost.value, aux

    def check(self, rule: int, sol):
        sol = np.ascontiguousarray(sol, dtype=np.int32)
        f = C.c_int32()
        nv = C.c_int64()
        if lib().orc_check(self.h, rule, sol, C.byref(f), C.byref(nv)) != 0:
            raise ValueError("bad rule")
        return bool(f.value), int(nv.value)


class OracleSolver:
    def __init__(self, lp: OracleLP, beta: float = 10.0, step_rule: int = STEP_PER_COORD,
                 step_scale: float = 1.0, prox: bool = False, ybar=None, ubar=None,
                 schedule: int = SCHED_DET, seed: int = 0):
        self.lp = lp
        self._yb = None if ybar is None else np.ascontiguousarray(ybar, dtype=np.float64)
        self._ub = None if ubar is None else np.ascontiguousarray(ubar, dtype=np.float64)
        self.h = lib().orc_solver_create(lp.h, beta, step_rule, step_scale, int(prox),
                                         _ptr(self._yb), _ptr(self._ub), schedule, seed)
        if not self.h:
            raise ValueError("oracle rejected the parameters")

    def __del__(self):
        # at interpreter exit the module's globals may already be gone
        if getattr(self, "h", None) and callable(globals().get("lib")):
            lib().orc_solver_free(self.h)
            self.h = None

    def run(self, epochs: int, within_reverse: bool = False, trace: bool = False):
        F = np.zeros(max(epochs, 1)) if trace else None
        lib().orc_run_epochs(self.h, epochs, int(within_reverse), _ptr(F))
        return F

    def step_unit(self, t: int) -> None:
        lib().orc_step_unit(self.h, t)

    def trace_epoch(self) -> np.ndarray:
        cap = self.lp.N + 1
        out = np.zeros(cap)
        k = lib().orc_trace_epoch(self.h, out, cap)
        return out[:k]

    @property
    def y(self) -> np.ndarray:
        out = np.zeros(self.lp.N)
        lib().orc_get_y(self.h, out)
        return out

    @y.setter
    def y(self, v):
        lib().orc_set_y(self.h, np.ascontiguousarray(v, dtype=np.float64))

    @property
    def x(self) -> np.ndarray:
        return self.y[: self.lp.n]

    @property
    def r(self) -> np.ndarray:
        out = np.zeros(self.lp.m)
        lib().orc_get_r(self.h, out)
        return out

    @property
    def epoch(self) -> int:
        return lib().orc_epoch(self.h)

    @epoch.setter
    def epoch(self, e: int):
        """Epoch counter (selects the class order of the next epoch)."""
        lib().orc_set_epoch(self.h, int(e))

    @property
    def lmax(self) -> float:
        return lib().orc_lmax(self.h)

    def penalty(self) -> float:
        return lib().orc_penalty(self.h)

    def metrics(self) -> dict:
        out = np.zeros(8)
        lib().orc_metrics(self.h, out)
        return dict(F=out[0], lp_value=out[1], linf=out[2], l2=out[3], max_viol=out[4],
                    dual_bound=out[5], gap=out[6])

    def multiplier_step(self, move_centre: bool = False, beta: float = 0.0) -> dict:
        """One augmented-Lagrangian update (Section 3.2): ubar -= beta (A y - b),
        ybar <- y with move_centre (prox on), then beta <- beta when > 0.
        Returns c^T x, ||A y - b||_inf, the LP dual bound D at the clipped new
        multiplier and the relative LP gap, all at the current y."""
        out = np.zeros(4)
        lib().orc_multiplier_step(self.h, int(move_centre), float(beta), out)
        return dict(lp_value=out[0], linf=out[1], lp_dual=out[2], lp_gap=out[3])

    @property
    def ubar(self) -> np.ndarray:
        out = np.zeros(self.lp.m)
        lib().orc_get_ubar(self.h, out)
        return out

    @property
    def ybar(self) -> np.ndarray:
        out = np.zeros(self.lp.N)
        lib().orc_get_ybar(self.h, out)
        return out

    @property
    def beta(self) -> float:
        return lib().orc_beta(self.h)
