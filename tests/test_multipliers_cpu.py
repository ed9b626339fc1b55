"""Pins of the oracle's multiplier step (augmented-Lagrangian framework,
Section 3.2) against what LP duality fixes, independent of the oracle:

  * the KKT pair of the LP (HiGHS primal and row duals) is a fixed point of
    the step and of the SCD epochs around it, and the LP dual function D at
    the LP duals equals LP* (strong duality);
  * D(u) <= LP* at every step from any start (weak duality);
  * the outer loop reaches LP* and a feasible point without beta -> inf
    (closed form for the triangle: x = 1/2, unique duals 1/2);
  * a beta change rescales every curvature: Lmax = beta * max_j ||A_j||^2 + rho.
"""
import numpy as np
import pytest
from scipy.optimize import linprog

from oracle import oracle as O
from paper_1311_2661_amd import instances as I

from test_oracle_pins import dense_aug, highs_lp, random_graph


def highs_lp_blocks(inst):
    """LP* and row duals of an instance with simplex blocks: the block rows
    sum x = 1 and the fixed labels become explicit constraints for HiGHS."""
    n = inst.n
    A = dense_aug(inst)[:, :n]
    sgn = inst.sense.astype(float)
    A_ub = -(sgn[:, None] * A)
    b_ub = -(sgn * inst.b)
    k = inst.block_k
    nb = len(inst.block_first_col)
    A_eq = np.zeros((nb, n))
    for t, f in enumerate(inst.block_first_col):
        A_eq[t, f:f + k] = 1.0
    bounds = [(0.0, u) for u in inst.u]
    for t, f in enumerate(inst.block_first_col):
        lab = inst.fixed_label[t]
        if lab >= 0:
            for i in range(k):
                v = 1.0 if i == lab else 0.0
                bounds[f + i] = (v, v)
    res = linprog(inst.c, A_ub=A_ub, b_ub=b_ub, A_eq=A_eq, b_eq=np.ones(nb), bounds=bounds,
                  method="highs")
    assert res.status == 0
    return res.fun, res.x, -res.ineqlin.marginals * sgn


def kkt_point(inst, x):
    """y = (x, s) with the slacks that make every inequality row exact."""
    A = dense_aug(inst)[:, : inst.n]
    s = np.where(inst.sense != 0, inst.sense * (A @ x - inst.b), 0.0)
    return np.concatenate([x, np.maximum(s, 0.0)])


def outer_loop(s, outer, inner=400, tol=1e-12, move_centre=False, beta=0.0):
    hist = []
    for _ in range(outer):
        for _ in range(40):
            s.run(inner)
            if s.metrics()["gap"] < tol:
                break
        hist.append(s.multiplier_step(move_centre=move_centre, beta=beta))
    return hist


def vc_instance(seed, n=14, p=0.3):
    rng = np.random.default_rng(seed)
    return I.vc_lp(n, random_graph(n, p, rng), rng.uniform(1, 10, n))


def mis_instance(seed, n=14, p=0.3):
    rng = np.random.default_rng(seed)
    return I.mis_lp(n, random_graph(n, p, rng), rng.uniform(1, 5, n))


# ---------------------------------------------------------------- fixed point

@pytest.mark.parametrize("maker,seed", [(vc_instance, 11), (vc_instance, 12), (mis_instance, 13)])
@pytest.mark.parametrize("prox", [False, True])
def test_lp_kkt_pair_is_a_fixed_point(maker, seed, prox):
    inst = maker(seed)
    lpstar, xstar, ustar = highs_lp(inst)
    ystar = kkt_point(inst, xstar)
    lp = O.OracleLP(inst)
    s = O.OracleSolver(lp, beta=10.0, prox=prox, ybar=ystar if prox else None, ubar=ustar)
    s.y = ystar
    st = s.multiplier_step(move_centre=prox)
    assert st["linf"] < 1e-9
    assert st["lp_value"] == pytest.approx(lpstar, abs=1e-9)
    # strong duality: the LP dual function at the LP duals is LP*
    assert st["lp_dual"] == pytest.approx(lpstar, abs=1e-8)
    assert np.abs(s.ubar - ustar).max() < 1e-8
    s.run(20)
    assert np.abs(s.y - ystar).max() < 1e-7


def test_lp_dual_function_of_a_wrong_sign_multiplier_is_clipped():
    """A covering row's multiplier below zero is clipped to zero before D is
    formed; D(0) of vertex cover is 0 (every reduced cost is c_j >= 0)."""
    inst = vc_instance(3)
    lp = O.OracleLP(inst)
    s = O.OracleSolver(lp, beta=10.0, ubar=np.full(inst.m, -5.0))
    s.y = np.concatenate([np.ones(inst.n), np.ones(inst.m)])    # every row exact: w = 0
    st = s.multiplier_step()
    assert st["linf"] == 0.0
    assert st["lp_dual"] == 0.0
    assert st["lp_value"] == pytest.approx(inst.c.sum(), rel=1e-15)
    assert np.all(s.ubar == -5.0)


# ---------------------------------------------------------------- weak duality, convergence

@pytest.mark.parametrize("maker,seed", [(vc_instance, 21), (mis_instance, 22)])
@pytest.mark.parametrize("prox", [False, True])
def test_outer_loop_reaches_lp_optimum(maker, seed, prox):
    inst = maker(seed)
    lpstar, _, _ = highs_lp(inst)
    lp = O.OracleLP(inst)
    s = O.OracleSolver(lp, beta=10.0, prox=prox, ybar=np.zeros(inst.n + inst.m) if prox else None,
                       ubar=np.zeros(inst.m), schedule=O.SCHED_PERM, seed=seed)
    hist = outer_loop(s, 12, move_centre=prox)
    for st in hist:
        assert st["lp_dual"] <= lpstar + 1e-9
    last = hist[-1]
    assert last["linf"] < 1e-8
    assert last["lp_value"] == pytest.approx(lpstar, abs=1e-7)
    assert last["lp_dual"] == pytest.approx(lpstar, abs=1e-7)
    assert last["lp_gap"] < 1e-8
    # penalty alone at the same beta stops short of LP*
    assert hist[0]["linf"] > 1e-3


def test_outer_loop_general_lp_with_equality_rows_and_bounds():
    rng = np.random.default_rng(31)
    m, n = 12, 16
    A = np.where(rng.random((m, n)) < 0.35, rng.uniform(0.5, 2.0, (m, n)), 0.0)
    for i in range(m):
        if not A[i].any():
            A[i, rng.integers(n)] = 1.0
    x0 = rng.uniform(0.2, 0.8, n)                 # a strictly feasible point
    sense = rng.choice([-1, 0, 1], size=m).astype(np.int8)
    b = A @ x0 - 0.3 * sense
    u = rng.uniform(1.0, 2.0, n)
    c = rng.uniform(-1.0, 2.0, n)
    rows = [np.nonzero(A[i])[0] for i in range(m)]
    row_ptr = np.concatenate([[0], np.cumsum([len(r) for r in rows])]).astype(np.int64)
    col = np.concatenate(rows).astype(np.int32)
    inst = I.LPInstance(m=m, n=n, row_ptr=row_ptr, col_idx=col,
                        val=np.concatenate([A[i, r] for i, r in enumerate(rows)]),
                        b=b, c=c, u=u, sense=sense)
    ub_rows = sense != 0
    res = linprog(c, A_ub=-(sense[ub_rows, None] * A[ub_rows]), b_ub=-(sense[ub_rows] * b[ub_rows]),
                  A_eq=A[~ub_rows], b_eq=b[~ub_rows], bounds=list(zip(np.zeros(n), u)), method="highs")
    assert res.status == 0
    # with prox the centre's weight 1/beta slows the outer iteration: a larger
    # beta there
    for prox, beta, outer in ((False, 5.0, 10), (True, 20.0, 30)):
        lp = O.OracleLP(inst)
        s = O.OracleSolver(lp, beta=beta, prox=prox, ybar=np.zeros(n + m) if prox else None,
                           ubar=np.zeros(m))
        hist = outer_loop(s, outer, move_centre=prox)
        for st in hist:
            assert st["lp_dual"] <= res.fun + 1e-9
        assert hist[-1]["linf"] < 1e-9
        assert hist[-1]["lp_value"] == pytest.approx(res.fun, abs=1e-8)
        assert hist[-1]["lp_dual"] == pytest.approx(res.fun, abs=1e-8)


@pytest.mark.parametrize("prox", [False, True])
def test_triangle_reaches_half_with_unique_duals(prox):
    # penalty alone at beta 10: x = 0.475; the LP: x = 1/2, LP* = 3/2, and the
    # only optimal dual gives every edge 1/2 (all three vertex rows tight)
    inst = I.vc_lp(3, np.array([[0, 1], [1, 2], [0, 2]]), np.ones(3))
    lp = O.OracleLP(inst)
    s = O.OracleSolver(lp, beta=10.0, prox=prox, ybar=np.zeros(6) if prox else None,
                       ubar=np.zeros(3))
    hist = outer_loop(s, 15, move_centre=prox)
    if not prox:
        assert hist[0]["lp_value"] == pytest.approx(3 * 0.475, abs=1e-12)
    assert np.allclose(s.x, 0.5, atol=1e-9)
    assert np.allclose(s.ubar, 0.5, atol=1e-9)
    assert hist[-1]["lp_dual"] == pytest.approx(1.5, abs=1e-9)


def test_multiway_cut_outer_loop_matches_highs():
    inst = I.mc_grid(side=5, k=3, seed=2)
    lpstar, _, _ = highs_lp_blocks(inst)
    lp = O.OracleLP(inst)
    s = O.OracleSolver(lp, beta=10.0, ubar=np.zeros(inst.m))
    hist = outer_loop(s, 20, inner=300)
    for st in hist:
        assert st["lp_dual"] <= lpstar + 1e-9
    assert hist[-1]["linf"] < 1e-7
    assert hist[-1]["lp_value"] == pytest.approx(lpstar, abs=1e-6)
    assert hist[-1]["lp_dual"] == pytest.approx(lpstar, abs=1e-6)


# ---------------------------------------------------------------- beta continuation

@pytest.mark.parametrize("prox", [False, True])
def test_beta_change_rescales_every_curvature(prox):
    inst = vc_instance(41, n=20, p=0.3)
    deg = np.bincount(inst.col_idx, minlength=inst.n)
    lp = O.OracleLP(inst)
    s = O.OracleSolver(lp, beta=10.0, prox=prox, ybar=np.zeros(inst.n + inst.m) if prox else None,
                       ubar=np.zeros(inst.m))
    assert s.lmax == pytest.approx(10.0 * max(deg.max(), 1) + (0.1 if prox else 0.0), rel=1e-15)
    s.run(3)
    s.multiplier_step(beta=40.0)
    assert s.beta == 40.0
    assert s.lmax == pytest.approx(40.0 * max(deg.max(), 1) + (1 / 40 if prox else 0.0), rel=1e-15)


def test_move_centre_copies_y_only_with_prox():
    inst = vc_instance(42)
    lp = O.OracleLP(inst)
    s = O.OracleSolver(lp, beta=10.0, prox=True, ybar=np.zeros(inst.n + inst.m), ubar=np.zeros(inst.m))
    s.run(5)
    s.multiplier_step(move_centre=True)
    assert np.array_equal(s.ybar, s.y)
    s2 = O.OracleSolver(lp, beta=10.0, ubar=np.zeros(inst.m))
    s2.run(5)
    s2.multiplier_step(move_centre=True)
    assert np.all(s2.ybar == 0.0)
