"""CPU checks of libthetis: the library loads, exports every entry point its
header declares, and its host-side layout (validation, units, greedy colour
classes) agrees with the oracle's.  No call here touches a GPU."""
import os
import re

import numpy as np
import pytest

from oracle import oracle as O
from paper_1311_2661_amd import instances as I
from paper_1311_2661_amd import thetis as T

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    src = open(os.path.join(ROOT, "include", "thetis.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(thetis_[a-z_0-9]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    L = T.lib()
    names = declared_symbols()
    assert len(names) >= 20
    for name in names:
        assert hasattr(L, name), name
    assert set(names) == set(T.EXPORTED)


def test_params_default():
    p = T.thetis_params_default()
    assert p.beta == 10.0 and p.step_rule == T.STEP_PER_COORD and p.step_scale == 1.0
    assert p.schedule == T.SCHED_DET and p.precision == T.PREC_FP32 and p.refresh_every == 5


@pytest.mark.parametrize("maker", [
    lambda: I.vc_er(400, 1600, seed=3),
    lambda: I.vc_ba(3000, seed=1),
    lambda: I.mis_regular(500, 6, seed=2),
    lambda: I.mc_grid(side=12, k=4, seed=5),
])
def test_classes_match_oracle(maker):
    inst = maker()
    h = T.Instance(inst)
    nc, nu, cls = h.classes()
    lp = O.OracleLP(inst)
    kind, uid, colour = lp.units()
    assert nc == lp.nclasses
    assert nu == len(colour)
    assert np.array_equal(cls, colour)


def test_blocks_set_after_a_layout_use_the_callers_column_order():
    """Without blocks the layout renumbers the columns into plan order; blocks
    declared afterwards name columns in the caller's order, so the instance
    goes back to that order first and its classes equal the oracle's."""
    inst = I.mc_grid(side=10, k=4, seed=2)
    h = T.thetis_inst_create_csr(inst.m, inst.n, inst.nnz, inst.row_ptr, inst.col_idx, inst.val, inst.b,
                                 inst.c, inst.u, inst.sense)
    try:
        nc0, nu0, cls0 = T.thetis_inst_classes(h)      # layout without blocks
        assert nu0 > inst.n
        T.thetis_inst_set_simplex_blocks(h, len(inst.block_first_col), inst.block_k, inst.block_first_col,
                                         inst.fixed_label)
        nc, nu, cls = T.thetis_inst_classes(h)
        kind, uid, colour = O.OracleLP(inst).units()
        assert nc == O.OracleLP(inst).nclasses and nu == len(colour)
        assert np.array_equal(cls, colour)
    finally:
        T.thetis_inst_destroy(h)


def test_ba_colouring_is_small():
    # every new BA vertex has 3 earlier neighbours: greedy in vertex order
    # needs at most 4 colours, plus the slack class
    inst = I.vc_ba(20000, seed=0)
    nc, _, _ = T.Instance(inst).classes()
    assert nc <= 5


def _vc_arrays():
    inst = I.vc_lp(3, np.array([[0, 1], [1, 2]]), np.ones(3))
    return inst


@pytest.mark.parametrize("mutate,code", [
    (lambda a: a.__setitem__("col_idx", np.array([0, 1, 1, 5], np.int32)), T.EINVAL),
    (lambda a: a.__setitem__("col_idx", np.array([0, 0, 1, 2], np.int32)), T.EINVAL),
    (lambda a: a.__setitem__("c", np.array([1.0, np.nan, 1.0])), T.EINVAL),
    (lambda a: a.__setitem__("b", np.array([1.0, np.inf])), T.EINVAL),
    (lambda a: a.__setitem__("u", np.array([1.0, -1.0, 1.0])), T.EINVAL),
    (lambda a: a.__setitem__("sense", np.array([1, 2], np.int8)), T.EINVAL),
    (lambda a: a.__setitem__("row_ptr", np.array([0, 3, 2], np.int64)), T.EINVAL),
])
def test_invalid_instances_are_rejected(mutate, code):
    inst = _vc_arrays()
    a = dict(row_ptr=inst.row_ptr, col_idx=inst.col_idx, c=inst.c, b=inst.b, u=inst.u,
             sense=inst.sense)
    mutate(a)
    with pytest.raises(T.ThetisError) as ei:
        T.thetis_inst_create_csr(inst.m, inst.n, int(a["row_ptr"][-1]), a["row_ptr"], a["col_idx"],
                                 None, a["b"], a["c"], a["u"], a["sense"])
    assert ei.value.code == code
    assert T.thetis_last_error() != ""


def test_invalid_blocks_are_rejected():
    inst = I.mc_grid(side=4, k=3, seed=0)
    h = T.Instance.__new__(T.Instance)
    hh = T.thetis_inst_create_csr(inst.m, inst.n, inst.nnz, inst.row_ptr, inst.col_idx, inst.val,
                                  inst.b, inst.c, inst.u, inst.sense)
    with pytest.raises(T.ThetisError):
        T.thetis_inst_set_simplex_blocks(hh, 2, 3, np.array([0, 1]), None)   # overlap
    with pytest.raises(T.ThetisError):
        T.thetis_inst_set_simplex_blocks(hh, 1, 65, np.array([0]), None)      # k too large
    with pytest.raises(T.ThetisError):
        T.thetis_inst_set_simplex_blocks(hh, 1, 3, np.array([0]), np.array([3], np.int32))
    T.thetis_inst_destroy(hh)
    del h


def test_workspace_bytes_scale_with_precision():
    inst = I.vc_er(1000, 5000, seed=0)
    h = T.Instance(inst)
    p32 = T.thetis_params_default()
    p64 = T.thetis_params_default()
    p64.precision = T.PREC_FP64
    b32 = T.thetis_solver_workspace_bytes(h.h, p32)
    b64 = T.thetis_solver_workspace_bytes(h.h, p64)
    assert 0 < b32 < b64
    bad = T.thetis_params_default()
    bad.beta = -1.0
    with pytest.raises(T.ThetisError):
        T.thetis_solver_workspace_bytes(h.h, bad)
    bad = T.thetis_params_default()
    bad.refresh_every = 0
    with pytest.raises(T.ThetisError):
        T.thetis_solver_workspace_bytes(h.h, bad)


# ------------------------------------------------------------ general rounding shapes

def _rows_lp(rows, b, sense, n):
    row_ptr = [0]
    col, val = [], []
    for r in rows:
        for j in sorted(r):
            col.append(j)
            val.append(float(r[j]))
        row_ptr.append(len(col))
    m = len(rows)
    return I.LPInstance(m=m, n=n, row_ptr=np.array(row_ptr, np.int64), col_idx=np.array(col, np.int32),
                        val=np.array(val), b=np.array(b, float), c=np.ones(n), u=np.ones(n),
                        sense=np.full(m, sense, np.int8))


@pytest.mark.parametrize("seed", range(8))
def test_cover_q_and_shapes_match_the_oracle(seed):
    """q(P) from the library's bitset subset sums equals the oracle's
    subset-sum table, on random integer rows (right-hand sides up to 200)."""
    rng = np.random.default_rng(seed)
    n = 30
    rows = []
    for _ in range(25):
        cols = rng.choice(n, size=int(rng.integers(1, 9)), replace=False)
        rows.append({int(j): int(rng.integers(1, 70)) for j in cols})
    inst = _rows_lp(rows, [int(rng.integers(1, 200)) for _ in rows], 1, n)
    flags, q = T.Instance(inst).rounding_shape()
    assert flags == T.SHAPE_COVER
    assert q == O.OracleLP(inst).cover_q()


def test_rounding_shapes_of_the_workloads():
    sc = T.Instance(I.set_cover(200, 80, seed=1)).rounding_shape()
    assert sc == (T.SHAPE_COVER | T.SHAPE_SET_COVER, 1.0)
    vc = T.Instance(I.vc_er(50, 100, seed=1)).rounding_shape()
    assert vc == (T.SHAPE_COVER | T.SHAPE_SET_COVER, 1.0)
    mis = T.Instance(I.mis_regular(50, 3, seed=1)).rounding_shape()
    assert mis == (T.SHAPE_PACK, 0.0)
    pk = T.Instance(I.kcs_packing(60, 40, 3, seed=1)).rounding_shape()
    assert pk == (T.SHAPE_PACK, 0.0)
    mc = T.Instance(I.mc_grid(side=6, k=3, seed=1))
    assert mc.rounding_shape()[0] == 0
    mcov = I.multicover(80, 40, seed=2)
    fl, q = T.Instance(mcov).rounding_shape()
    assert fl == T.SHAPE_COVER and q == O.OracleLP(mcov).cover_q()


def test_blocks_whose_columns_share_a_row_are_rejected():
    """A simplex block with two columns in one row is refused (the block's
    curvature bound and its race-free scatter need every row to hold at most
    one column of each block)."""
    inst = I.LPInstance(m=2, n=3, row_ptr=np.array([0, 2, 4], np.int64),
                        col_idx=np.array([0, 2, 1, 2], np.int32), val=None,
                        b=np.ones(2), c=np.ones(3), u=np.ones(3), sense=np.ones(2, np.int8),
                        block_first_col=np.array([1], np.int64), block_k=2,
                        fixed_label=np.array([-1], np.int32))
    with pytest.raises(T.ThetisError, match="share a row"):
        T.Instance(inst)
    inst.block_first_col = np.array([0], np.int64)
    T.Instance(inst)
