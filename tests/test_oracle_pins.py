"""Pins for the FP64 oracle against facts the paper and the mathematics fix.

None of these re-types the oracle's own formula: each compares it with a
closed form, an independent solver (HiGHS, L-BFGS-B, brute force), a
library routine (numpy's Philox) or an invariant stated in the paper.
"""
import itertools

import numpy as np
import pytest
from scipy.optimize import linprog, minimize

from oracle import oracle as O
from paper_1311_2661_amd import instances as I


# ---------------------------------------------------------------- helpers

def dense_aug(inst):
    """Dense [A | slack] matrix, built from the CSR by plain indexing."""
    A = np.zeros((inst.m, inst.n + inst.m))
    for i in range(inst.m):
        for e in range(inst.row_ptr[i], inst.row_ptr[i + 1]):
            A[i, inst.col_idx[e]] = 1.0 if inst.val is None else inst.val[e]
        A[i, inst.n + i] = -float(inst.sense[i])
    return A


def highs_lp(inst):
    """LP* and the row duals u* (sign convention of A x >= b rows) by HiGHS."""
    A = dense_aug(inst)[:, : inst.n]
    sgn = inst.sense.astype(float)
    ub_rows = sgn != 0
    A_ub = -(sgn[ub_rows, None] * A[ub_rows])
    b_ub = -(sgn[ub_rows] * inst.b[ub_rows])
    res = linprog(inst.c, A_ub=A_ub, b_ub=b_ub, bounds=list(zip(np.zeros(inst.n), inst.u)),
                  method="highs")
    assert res.status == 0
    u = np.zeros(inst.m)
    u[ub_rows] = -res.ineqlin.marginals * sgn[ub_rows]
    return res.fun, res.x, u


def converge(inst, beta=10.0, prox=False, ybar=None, tol=1e-12, max_rounds=400, seed=0,
             schedule=O.SCHED_DET):
    lp = O.OracleLP(inst)
    s = O.OracleSolver(lp, beta=beta, prox=prox, ybar=ybar, schedule=schedule, seed=seed)
    for _ in range(max_rounds):
        s.run(200)
        if s.metrics()["gap"] < tol:
            break
    return lp, s


def random_graph(n, p, rng):
    return np.array([(u, v) for u in range(n) for v in range(u + 1, n) if rng.random() < p],
                    dtype=np.int64).reshape(-1, 2)


# ---------------------------------------------------------------- Philox

@pytest.mark.parametrize("key", [(0, 0), (5, 7), (2**64 - 1, 123456789)])
def test_philox_matches_numpy(key):
    """Philox4x64-10 block c equals numpy's Philox stream started at c-1
    (numpy advances its counter before each block)."""
    k = np.array(key, dtype=np.uint64)
    for ctr in [(1, 0, 0, 0), (0, 3, 9, 0), (2**64 - 1, 0, 0, 0), (17, 2**63, 5, 1)]:
        c = np.array(ctr, dtype=np.uint64)
        prev = c.copy()
        # subtract one with borrow
        for w in range(4):
            if prev[w] != 0:
                prev[w] -= np.uint64(1)
                break
            prev[w] = np.uint64(2**64 - 1)
        g = np.random.Philox(key=k, counter=prev)
        assert np.array_equal(g.random_raw(4), O.philox(c, k))


# ---------------------------------------------------------------- closed forms

@pytest.mark.parametrize("beta", [2.0, 10.0, 100.0])
def test_single_edge_equal_weights(beta):
    # F(beta) = 1 - 1/(2 beta): x_u + x_v = 1 - 1/beta at the minimiser
    inst = I.vc_lp(2, np.array([[0, 1]]), np.array([1.0, 1.0]))
    _, s = converge(inst, beta)
    assert s.metrics()["F"] == pytest.approx(1 - 1 / (2 * beta), abs=1e-12)


@pytest.mark.parametrize("cu,cv", [(1.0, 3.0), (2.5, 4.0)])
def test_single_edge_unequal_weights(cu, cv):
    # cheaper endpoint carries the edge: F = c_u - c_u^2 / (2 beta)
    beta = 10.0
    inst = I.vc_lp(2, np.array([[0, 1]]), np.array([cu, cv]))
    _, s = converge(inst, beta)
    assert s.metrics()["F"] == pytest.approx(cu - cu * cu / (2 * beta), abs=1e-12)
    assert s.x[1] == pytest.approx(0.0, abs=1e-12)
    assert s.x[0] == pytest.approx(1 - cu / beta, abs=1e-12)


def test_triangle():
    # symmetric x = 1/2 - 1/(4 beta), F = 3/2 - 3/(8 beta); beta=10: 0.475, 1.4625
    inst = I.vc_lp(3, np.array([[0, 1], [1, 2], [0, 2]]), np.ones(3))
    _, s = converge(inst, 10.0)
    assert np.allclose(s.x, 0.475, atol=1e-12)
    assert s.metrics()["F"] == pytest.approx(1.4625, abs=1e-12)


@pytest.mark.parametrize("k", [2, 5, 9])
def test_star(k):
    # K_{1,k}, unit weights: centre 1 - 1/(beta k), leaves 0, F = 1 - 1/(2 beta k)
    beta = 10.0
    edges = np.array([[0, i] for i in range(1, k + 1)])
    inst = I.vc_lp(k + 1, edges, np.ones(k + 1))
    _, s = converge(inst, beta)
    assert s.metrics()["F"] == pytest.approx(1 - 1 / (2 * beta * k), abs=1e-12)
    assert s.x[0] == pytest.approx(1 - 1 / (beta * k), abs=1e-12)


# ---------------------------------------------------------------- independent solvers

def _penalty_and_grad(A, inst, beta):
    b = inst.b
    c = np.concatenate([inst.c, np.zeros(inst.m)])

    def f(y):
        w = A @ y - b
        return c @ y + 0.5 * beta * w @ w, c + beta * A.T @ w
    return f


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_converged_penalty_matches_lbfgsb(seed):
    """F* from SCD equals L-BFGS-B on the same box-constrained QP."""
    rng = np.random.default_rng(seed)
    n = 12
    edges = random_graph(n, 0.35, rng)
    inst = I.vc_lp(n, edges, rng.uniform(1, 10, n))
    _, s = converge(inst, 10.0)
    A = dense_aug(inst)
    f = _penalty_and_grad(A, inst, 10.0)
    bounds = [(0, 1)] * inst.n + [(0, None)] * inst.m
    res = minimize(f, np.full(A.shape[1], 0.5), jac=True, method="L-BFGS-B", bounds=bounds,
                   options=dict(maxiter=20000, ftol=1e-15, gtol=1e-12))
    assert s.metrics()["F"] == pytest.approx(res.fun, rel=1e-8, abs=1e-8)
    assert s.metrics()["F"] <= res.fun + 1e-10


@pytest.mark.parametrize("seed,prox", [(3, False), (4, False), (5, True), (6, True)])
def test_dual_bound_weak_and_strong_duality(seed, prox):
    """Phi(u) <= F(y) along the whole run and meets it at convergence, with
    the prox term too (then each column's minimum is the clipped minimiser
    of red y + rho/2 (y - ybar)^2)."""
    rng = np.random.default_rng(seed)
    n = 15
    inst = I.vc_lp(n, random_graph(n, 0.3, rng), rng.uniform(1, 10, n))
    yb = rng.uniform(0, 1, inst.n + inst.m) if prox else None
    lp = O.OracleLP(inst)
    s = O.OracleSolver(lp, beta=10.0, schedule=O.SCHED_PERM, seed=seed, prox=prox, ybar=yb)
    for _ in range(50):
        m = s.metrics()
        assert m["dual_bound"] <= m["F"] + 1e-12
        s.run(3)
    _, s2 = converge(inst, 10.0, prox=prox, ybar=yb)
    m = s2.metrics()
    assert m["F"] - m["dual_bound"] < 1e-9


def test_violation_of_equality_rows_is_absolute():
    """The original-row violation: b - A x on '>=' rows, A x - b on '<='
    rows, |A x - b| on equality rows (either side)."""
    inst = I.LPInstance(m=2, n=3, row_ptr=np.array([0, 2, 4], np.int64), col_idx=np.array([0, 1, 1, 2], np.int32),
                        val=None, b=np.array([1.0, 1.0]), c=np.ones(3), u=np.ones(3),
                        sense=np.array([0, 1], np.int8))
    lp = O.OracleLP(inst)
    s = O.OracleSolver(lp)
    for x, viol in (((0.8, 0.5, 0.9), 0.3), ((0.2, 0.6, 0.6), 0.2), ((0.5, 0.5, 0.2), 0.3)):
        s.y = np.array(list(x) + [0.0, 0.0])
        assert s.metrics()["max_viol"] == pytest.approx(viol, abs=1e-15)


@pytest.mark.parametrize("seed", [5, 6, 7])
def test_lp_bracket(seed):
    """LP* - ||u*||^2/(2 beta) <= F(beta) <= LP* for any dual solution u*."""
    rng = np.random.default_rng(seed)
    n = 14
    inst = I.vc_lp(n, random_graph(n, 0.3, rng), rng.uniform(1, 10, n))
    lpstar, _, ustar = highs_lp(inst)
    for beta in (10.0, 100.0):
        _, s = converge(inst, beta)
        F = s.metrics()["F"]
        assert F <= lpstar + 1e-9
        assert F >= lpstar - ustar @ ustar / (2 * beta) - 1e-9


def test_half_integrality_brute_force():
    """VC LP optimum is half-integral: min over {0,1/2,1}^n equals LP*."""
    rng = np.random.default_rng(11)
    for trial in range(4):
        n = 8
        edges = random_graph(n, 0.45, rng)
        if len(edges) == 0:
            continue
        w = rng.uniform(1, 10, n)
        inst = I.vc_lp(n, edges, w)
        lpstar, xstar, _ = highs_lp(inst)
        grid = np.array(list(itertools.product([0.0, 0.5, 1.0], repeat=n)))
        ok = np.all(grid[:, edges[:, 0]] + grid[:, edges[:, 1]] >= 1 - 1e-12, axis=1)
        best = (grid[ok] @ w).min()
        assert best == pytest.approx(lpstar, abs=1e-9)
        # HiGHS returns a vertex, which is half-integral
        assert np.allclose(xstar * 2, np.round(xstar * 2), atol=1e-9)
        # SCD at growing beta approaches LP* from below
        vals = []
        for beta in (10.0, 100.0, 1000.0):
            _, s = converge(inst, beta, max_rounds=2000)
            vals.append(s.metrics()["F"])
        assert vals[0] <= vals[1] + 1e-9 <= vals[2] + 2e-9
        assert lpstar - vals[2] < (lpstar - vals[0]) / 50 + 1e-9


def _max_matching_brute(n, edges):
    best = 0
    m = len(edges)
    # bitmask DP over edges in order: choose or skip while vertices free
    from functools import lru_cache

    @lru_cache(maxsize=None)
    def go(i, used):
        if i == m:
            return 0
        u, v = edges[i]
        r = go(i + 1, used)
        if not (used >> u) & 1 and not (used >> v) & 1:
            r = max(r, 1 + go(i + 1, used | (1 << u) | (1 << v)))
        return r
    best = go(0, 0)
    return best


def _min_vc_brute(n, edges, w):
    masks = np.arange(1 << n, dtype=np.int64)
    bits = (masks[:, None] >> np.arange(n)) & 1
    cover = np.all(bits[:, edges[:, 0]] | bits[:, edges[:, 1]], axis=1)
    return (bits[cover] @ w).min()


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_koenig_bipartite(seed):
    """Bipartite, unit weights: LP* = max matching = min vertex cover
    (Koenig), all by brute force on <= 20 vertices; SCD brackets it:
    nu - nu/(2 beta) <= F(beta) <= nu, since ||u*||^2 <= sum u* = nu."""
    rng = np.random.default_rng(100 + seed)
    a, b = 9, 9
    edges = np.array([(i, a + j) for i in range(a) for j in range(b) if rng.random() < 0.25],
                     dtype=np.int64)
    n = a + b
    nu = _max_matching_brute(n, tuple(map(tuple, edges.tolist())))
    assert nu == _min_vc_brute(n, edges, np.ones(n))
    inst = I.vc_lp(n, edges, np.ones(n))
    lpstar, _, _ = highs_lp(inst)
    assert lpstar == pytest.approx(nu, abs=1e-9)
    prev = -np.inf
    for beta in (10.0, 100.0, 1000.0):
        _, s = converge(inst, beta, max_rounds=3000)
        m = s.metrics()
        assert m["gap"] < 1e-9
        assert m["F"] <= nu + 1e-9
        assert m["F"] >= nu - nu / (2 * beta) - 1e-9
        assert m["F"] >= prev - 1e-12
        prev = m["F"]


def test_weighted_bipartite_total_unimodularity():
    """Weighted bipartite VC: LP* equals the brute-force integer optimum."""
    rng = np.random.default_rng(42)
    a, b = 8, 8
    edges = np.array([(i, a + j) for i in range(a) for j in range(b) if rng.random() < 0.3],
                     dtype=np.int64)
    w = rng.uniform(1, 10, a + b)
    inst = I.vc_lp(a + b, edges, w)
    lpstar, _, ustar = highs_lp(inst)
    assert lpstar == pytest.approx(_min_vc_brute(a + b, edges, w), abs=1e-9)
    _, s = converge(inst, 1000.0, max_rounds=3000)
    F = s.metrics()["F"]
    assert lpstar - ustar @ ustar / 2000.0 - 1e-9 <= F <= lpstar + 1e-9


# ---------------------------------------------------------------- the iteration itself

@pytest.mark.parametrize("schedule", [O.SCHED_DET, O.SCHED_PERM, O.SCHED_UNIFORM])
@pytest.mark.parametrize("step_rule", [O.STEP_PER_COORD, O.STEP_GLOBAL_LMAX])
@pytest.mark.parametrize("prox", [False, True])
def test_serial_monotone_descent(schedule, step_rule, prox):
    """Every single SCD step does not increase F (descent lemma for the
    1/L step of Algorithm 1; the exact minimiser for the per-coordinate L)."""
    rng = np.random.default_rng(9)
    n = 30
    inst = I.vc_lp(n, random_graph(n, 0.2, rng), rng.uniform(1, 10, n))
    lp = O.OracleLP(inst)
    yb = rng.uniform(0, 1, inst.n + inst.m) if prox else None
    s = O.OracleSolver(lp, beta=10.0, step_rule=step_rule, prox=prox, ybar=yb,
                       schedule=schedule, seed=3)
    prev = s.penalty()
    for _ in range(4):
        tr = s.trace_epoch()
        seq = np.concatenate([[prev], tr])
        assert np.all(np.diff(seq) <= 1e-13 * np.maximum(1.0, np.abs(seq[:-1])))
        prev = tr[-1]


def test_per_coordinate_step_is_exact_minimiser():
    """A per-coordinate step lands on the 1-D minimiser of F over [0, u_j],
    found independently by bounded scalar minimisation."""
    from scipy.optimize import minimize_scalar
    rng = np.random.default_rng(21)
    n = 20
    inst = I.vc_lp(n, random_graph(n, 0.25, rng), rng.uniform(1, 10, n))
    lp = O.OracleLP(inst)
    s = O.OracleSolver(lp, beta=10.0)
    kind, uid, _ = lp.units()
    y0 = np.concatenate([rng.uniform(0, 1, inst.n), rng.uniform(0, 0.5, inst.m)])
    for t in rng.choice(len(uid), 15, replace=False):
        s.y = y0
        j = uid[t]
        hi = 1.0 if j < inst.n else 5.0

        def fj(v):
            yy = y0.copy()
            yy[j] = v
            s.y = yy
            return s.penalty()
        ref = minimize_scalar(fj, bounds=(0.0, hi), method="bounded",
                              options=dict(xatol=1e-12)).x
        s.y = y0
        s.step_unit(t)
        assert s.y[j] == pytest.approx(ref, abs=1e-7)
        changed = np.nonzero(s.y != y0)[0]
        assert set(changed.tolist()) <= {j}


def test_det_classes_are_conflict_free_and_order_free():
    """Units inside one colour class share no row, so reversing the order
    inside every class gives bit-identical FP64 iterates."""
    inst = I.vc_er(300, 1500, seed=4)
    lp = O.OracleLP(inst)
    kind, uid, colour = lp.units()
    A = dense_aug(inst) != 0
    for cl in range(lp.nclasses):
        cols = uid[colour == cl]
        rows_hit = A[:, cols].sum(axis=1)
        assert rows_hit.max() <= 1
    s1 = O.OracleSolver(lp, beta=10.0, seed=7)
    s2 = O.OracleSolver(lp, beta=10.0, seed=7)
    s1.run(5)
    s2.run(5, within_reverse=True)
    assert np.array_equal(s1.y, s2.y)


def test_greedy_colouring_matches_definition():
    """Brute-force greedy colouring in vertex order on the vertex graph."""
    inst = I.vc_er(200, 900, seed=2)
    lp = O.OracleLP(inst)
    kind, uid, colour = lp.units()
    edges = inst.meta["edges"]
    adj = [[] for _ in range(inst.n)]
    for u, v in edges:
        adj[u].append(v)
        adj[v].append(u)
    col = [-1] * inst.n
    for v in range(inst.n):
        used = {col[w] for w in adj[v] if col[w] >= 0}
        c = 0
        while c in used:
            c += 1
        col[v] = c
    assert np.array_equal(colour[: inst.n], np.array(col))
    assert np.all(colour[inst.n:] == max(col) + 1)
    assert lp.nclasses == max(col) + 2


def test_class_order_is_a_permutation():
    inst = I.vc_er(100, 300, seed=0)
    lp = O.OracleLP(inst)
    for e in range(6):
        o = lp.class_order(5, e)
        assert sorted(o.tolist()) == list(range(lp.nclasses))


def numpy_philox_word(key, ctr):
    """First word of Philox4x64-10 block `ctr` under `key`, from numpy's
    generator (which advances its counter before each block)."""
    c = np.array(ctr, dtype=np.uint64)
    prev = c.copy()
    for w in range(4):
        if prev[w] != 0:
            prev[w] -= np.uint64(1)
            break
        prev[w] = np.uint64(2**64 - 1)
    return int(np.random.Philox(key=np.array(key, dtype=np.uint64), counter=prev).random_raw(1)[0])


def test_class_order_follows_the_philox_words():
    """Reading R13: in epoch e the classes run in increasing order of the
    Philox word of counter (e, class, 0, 0) under key (seed, 1), ties by
    class id; and a DET epoch is the serial steps of the units class by
    class in that order."""
    inst = I.vc_er(60, 150, seed=4)
    lp = O.OracleLP(inst)
    kind, uid, col = lp.units()
    nc = lp.nclasses
    for seed, epoch in [(3, 0), (3, 1), (11, 7)]:
        words = [numpy_philox_word((seed, 1), (epoch, c, 0, 0)) for c in range(nc)]
        want = sorted(range(nc), key=lambda c: (words[c], c))
        assert lp.class_order(seed, epoch).tolist() == want
    a = O.OracleSolver(lp, beta=5.0, seed=3)
    a.run(1)
    b = O.OracleSolver(lp, beta=5.0, seed=3)
    words = [numpy_philox_word((3, 1), (0, c, 0, 0)) for c in range(nc)]
    for c in sorted(range(nc), key=lambda c: (words[c], c)):
        for t in np.nonzero(col == c)[0]:
            b.step_unit(int(t))
    assert np.array_equal(a.y, b.y)


def test_mis_threshold_is_strict():
    """Reading R9: MIS_THRESH keeps v iff x_v > max(1/2, max_e fl(x_u+x_v)/2).
    At the all-1/2 point nothing is kept (keeping ties would take both ends
    of every edge); a vertex at 0.6 whose neighbours sit at 0.4 is the only
    one kept."""
    inst = I.mis_regular(40, 3, seed=1)
    lp = O.OracleLP(inst)
    sol, cost, aux = lp.round(np.full(inst.n, 0.5), O.RULE_MIS_THRESH)
    assert not sol.any() and cost == 0.0 and aux[0] == 0.5
    x = np.full(inst.n, 0.5)
    nbrs = [inst.col_idx[inst.row_ptr[i] + 1 - k] for i in range(inst.m) for k in (0, 1)
            if inst.col_idx[inst.row_ptr[i] + k] == 0]
    x[0], x[nbrs] = 0.6, 0.4
    sol, cost, aux = lp.round(x, O.RULE_MIS_THRESH)
    assert aux[0] == 0.5
    assert np.nonzero(sol)[0].tolist() == [0]


@pytest.mark.parametrize("schedule,stream", [(O.SCHED_PERM, 3), (O.SCHED_UNIFORM, 2)])
def test_perm_and_uniform_schedules_follow_their_philox_words(schedule, stream):
    """Reading R4/R13 for the oracle-only schedules: in epoch e, PERM visits
    every unit once, in increasing order of the Philox word of counter
    (e, unit, 0, 0) under key (seed, 3); UNIFORM draws unit floor(u U) with
    u the 53-bit uniform of counter (e, step, 0, 0) under key (seed, 2)
    (with replacement).  Two epochs equal the same steps made by hand."""
    inst = I.vc_er(30, 70, seed=2)
    lp = O.OracleLP(inst)
    U = len(lp.units()[0])
    seed = 7
    a = O.OracleSolver(lp, beta=5.0, schedule=schedule, seed=seed)
    a.run(2)
    b = O.OracleSolver(lp, beta=5.0, seed=seed)
    for e in range(2):
        words = [numpy_philox_word((seed, stream), (e, t, 0, 0)) for t in range(U)]
        if schedule == O.SCHED_PERM:
            seq = sorted(range(U), key=lambda t: (words[t], t))
        else:
            seq = [min(int(((w >> 11) * 2.0 ** -53) * U), U - 1) for w in words]
            assert len(set(seq)) < U                 # with replacement
        for t in seq:
            b.step_unit(t)
    assert np.array_equal(a.y, b.y)


def u53(w):
    return (w >> 11) * 2.0 ** -53


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_mis_random_rounding_follows_its_philox_draws(seed):
    """Readings R8/R9/R13: alpha = max_e (x_u + x_v - 1)_+, keep v iff the
    53-bit uniform of counter (rep, v, 0, 0) under key (seed, 4) is below
    x_v / (1 + alpha), then drop both ends of every edge kept twice."""
    inst = I.mis_regular(24, 3, seed=seed)
    lp = O.OracleLP(inst)
    x = np.random.default_rng(seed).uniform(0, 0.8, inst.n)
    ends = inst.col_idx.reshape(-1, 2)
    alpha = max(0.0, float(np.max(x[ends[:, 0]] + x[ends[:, 1]] - 1.0)))
    pick = np.array([u53(numpy_philox_word((seed, 4), (0, v, 0, 0))) < x[v] / (1.0 + alpha)
                     for v in range(inst.n)])
    drop = np.zeros(inst.n, bool)
    for a, b in ends:
        if pick[a] and pick[b]:
            drop[a] = drop[b] = True
    sol, cost, aux = lp.round(x, O.RULE_MIS_RAND, seed=seed, reps=1)
    assert aux[0] == pytest.approx(alpha, abs=1e-15)
    assert np.array_equal(sol.astype(bool), pick & ~drop)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_region_growing_follows_its_philox_draws(seed):
    """Readings R10/R13: radius = the uniform of counter (rep, 0, 1, 0), the
    labels ordered by the words of counters (rep, i, 2, 0) (ties by label);
    each block takes the first of the first k-1 labels in that order whose
    x is >= 1 - radius, else the last label."""
    inst = I.mc_grid(side=5, k=4, seed=seed)
    lp = O.OracleLP(inst)
    nb, k = len(inst.block_first_col), inst.block_k
    X = np.random.default_rng(seed).dirichlet(np.full(k, 0.4), nb)
    term = np.asarray(inst.meta["terminals"])
    X[term] = np.eye(k)[inst.fixed_label[term]]
    x = np.zeros(inst.n)
    for t, f in enumerate(inst.block_first_col):
        x[f: f + k] = X[t]
    rad = u53(numpy_philox_word((seed, 4), (0, 0, 1, 0)))
    words = [numpy_philox_word((seed, 4), (0, i, 2, 0)) for i in range(k)]
    order = sorted(range(k), key=lambda i: (words[i], i))
    want = []
    for t in range(nb):
        lab = order[k - 1]
        for i in order[: k - 1]:
            if X[t, i] >= 1.0 - rad:
                lab = i
                break
        want.append(lab)
    sol, cost, aux = lp.round(x, O.RULE_MC_CKR, seed=seed, reps=1)
    assert aux[0] == rad
    assert sol.tolist() == want


@pytest.mark.parametrize("gamma", [1.0, 0.5, 0.25])
def test_step_scale_scales_the_coordinate_step(gamma):
    """The scaled step y - gamma g / L (Algorithm 1 with a step factor):
    single edge, c = (1, 1), beta 10, from y = 0 the residual is -1, so the
    first vertex has g = 1 - 10 = -9 and L = 10: it moves to 0.9 gamma."""
    inst = I.vc_lp(2, np.array([[0, 1]]), np.array([1.0, 1.0]))
    lp = O.OracleLP(inst)
    s = O.OracleSolver(lp, beta=10.0, step_scale=gamma)
    kind, uid, col = lp.units()
    t = int(np.nonzero((kind == 0) & (uid == 0))[0][0])
    s.step_unit(t)
    assert s.y[0] == pytest.approx(0.9 * gamma, abs=1e-15)


def test_kkt_projected_gradient_vanishes():
    """At convergence the projected-gradient residual of the box QP is ~0
    (the monotone LCP of Appendix A)."""
    rng = np.random.default_rng(17)
    n = 25
    inst = I.vc_lp(n, random_graph(n, 0.2, rng), rng.uniform(1, 10, n))
    _, s = converge(inst, 10.0)
    A = dense_aug(inst)
    f = _penalty_and_grad(A, inst, 10.0)
    y = s.y
    _, g = f(y)
    hi = np.concatenate([inst.u, np.full(inst.m, np.inf)])
    res = y - np.clip(y - g, 0, hi)
    assert np.abs(res).max() < 1e-8


def test_lemma_xb_bound_prox():
    """With the proximal term, ||A x(beta) - b|| <= (1/beta)[||u*-ubar|| +
    sqrt(||u*-ubar||^2 + ||x*-xbar||^2)] for a primal-dual LP pair
    (Lemma xb, Appendix A), ubar = 0."""
    rng = np.random.default_rng(23)
    n = 16
    inst = I.vc_lp(n, random_graph(n, 0.3, rng), rng.uniform(1, 10, n))
    lpstar, xs, us = highs_lp(inst)
    ss = dense_aug(inst)[:, : inst.n] @ xs - inst.b
    xstar = np.concatenate([xs, ss])
    for beta in (5.0, 20.0):
        xbar = np.concatenate([rng.uniform(0, 1, inst.n), np.zeros(inst.m)])
        _, s = converge(inst, beta, prox=True, ybar=xbar)
        m = s.metrics()
        bound = (np.linalg.norm(us) + np.sqrt(us @ us + np.sum((xstar - xbar) ** 2))) / beta
        assert m["l2"] <= bound + 1e-9


def test_scd_linear_rate_theorem():
    """Theorem (scd): with the proximal term (l = 1/beta), uniform sampling
    and the 1/Lmax step, E||x_j - x*||^2 + (2/Lmax) E(f_j - f*) decays at
    least like (1 - l/(n(l+Lmax)))^j times its start.  Mean over 200 runs."""
    rng = np.random.default_rng(31)
    n = 8
    inst = I.vc_lp(n, random_graph(n, 0.45, rng), rng.uniform(1, 3, n))
    beta = 2.0
    yb = np.full(inst.n + inst.m, 0.25)
    _, ref = converge(inst, beta, prox=True, ybar=yb, tol=1e-15)
    ystar, fstar = ref.y, ref.penalty()
    lp = O.OracleLP(inst)
    E = 12
    vals = np.zeros(E + 1)
    R = 0.0
    runs = 200
    for sd in range(runs):
        s = O.OracleSolver(lp, beta=beta, step_rule=O.STEP_GLOBAL_LMAX, prox=True, ybar=yb,
                           schedule=O.SCHED_UNIFORM, seed=1000 + sd)
        Lmax = s.lmax
        y = s.y
        vals[0] += np.sum((y - ystar) ** 2) + 2 / Lmax * (s.penalty() - fstar)
        R = max(R, np.linalg.norm(y - ystar))
        for e in range(E):
            s.run(1)
            y = s.y
            R = max(R, np.linalg.norm(y - ystar))
            vals[e + 1] += np.sum((y - ystar) ** 2) + 2 / Lmax * (s.penalty() - fstar)
    vals /= runs
    U = inst.n + inst.m
    l = 1 / beta
    rate = 1 - l / (U * (l + Lmax))
    s0 = O.OracleSolver(lp, beta=beta, prox=True, ybar=yb)
    start = R ** 2 + 2 / Lmax * (s0.penalty() - fstar)
    for e in range(E + 1):
        assert vals[e] <= rate ** (e * U) * start + 1e-12
    assert vals[-1] < vals[0]


# ---------------------------------------------------------------- rounding

def test_vc_threshold_rounding_properties():
    """Section 2 rule with the scaling of Lemma (infeasible:rounded:vc):
    always a cover, and cost <= 2 c^T x~ with x~ = proj(x/(1-eps))."""
    rng = np.random.default_rng(3)
    for trial in range(60):
        n = int(rng.integers(5, 40))
        edges = random_graph(n, rng.uniform(0.05, 0.5), rng)
        if len(edges) == 0:
            continue
        w = rng.uniform(1, 10, n)
        inst = I.vc_lp(n, edges, w)
        lp = O.OracleLP(inst)
        x = rng.uniform(0, 1, n) ** rng.uniform(0.3, 3)
        sol, cost, aux = lp.round(x, O.RULE_VC_THRESH)
        feas, nv = lp.check(O.RULE_VC_THRESH, sol)
        assert feas and nv == 0
        eps = max(0.0, np.max(1 - x[edges[:, 0]] - x[edges[:, 1]]))
        assert aux[0] == pytest.approx(min(0.5, (1 - eps) / 2), abs=1e-15)
        if eps < 1:
            xt = np.clip(x / (1 - eps), 0, 1)
            assert np.all(xt[edges[:, 0]] + xt[edges[:, 1]] >= 1 - 1e-12)
            assert cost <= 2 * (w @ xt) + 1e-9
            assert w @ xt <= (w @ x) / (1 - eps) + 1e-9
        assert cost == pytest.approx(w @ sol)


def test_rounding_keeps_integral_feasible_points():
    rng = np.random.default_rng(8)
    n = 30
    edges = random_graph(n, 0.15, rng)
    w = rng.uniform(1, 10, n)
    inst = I.vc_lp(n, edges, w)
    lp = O.OracleLP(inst)
    x = np.zeros(n)
    x[np.unique(edges[:, 0])] = 1.0       # a cover
    sol, _, _ = lp.round(x, O.RULE_VC_THRESH)
    assert np.array_equal(sol, x.astype(np.int32))
    # independent set: greedy integral one
    mis = np.zeros(n)
    for v in range(n):
        if all(not mis[u] for e in edges for u in e if v in e and u != v):
            mis[v] = 1
    inst2 = I.mis_lp(n, edges, w)
    lp2 = O.OracleLP(inst2)
    for rule in (O.RULE_MIS_THRESH, O.RULE_MIS_RAND):
        sol, _, _ = lp2.round(mis, rule, seed=3, reps=4)
        assert np.array_equal(sol, mis.astype(np.int32))


def test_mis_roundings_are_independent_sets():
    rng = np.random.default_rng(12)
    for trial in range(40):
        n = int(rng.integers(5, 40))
        edges = random_graph(n, rng.uniform(0.05, 0.5), rng)
        if len(edges) == 0:
            continue
        w = rng.uniform(1, 5, n)
        inst = I.mis_lp(n, edges, w)
        lp = O.OracleLP(inst)
        x = rng.uniform(0, 1, n)
        for rule in (O.RULE_MIS_THRESH, O.RULE_MIS_RAND):
            sol, cost, aux = lp.round(x, rule, seed=trial, reps=10)
            feas, nv = lp.check(rule, sol)
            assert feas and nv == 0
            assert not np.any(sol[edges[:, 0]] & sol[edges[:, 1]])
            assert cost == pytest.approx(-(w @ sol))


def test_mis_random_best_of_reps_monotone():
    """Best of more repetitions is never worse (draws are per repetition)."""
    inst = I.mis_regular(200, 4, seed=1)
    lp = O.OracleLP(inst)
    x = np.full(inst.n, 0.5)
    costs = [lp.round(x, O.RULE_MIS_RAND, seed=9, reps=r)[1] for r in (1, 3, 10)]
    assert costs[0] >= costs[1] >= costs[2]


def test_check_counts_violations():
    edges = np.array([[0, 1], [1, 2], [2, 3]])
    inst = I.vc_lp(4, edges, np.ones(4))
    lp = O.OracleLP(inst)
    assert lp.check(O.RULE_VC_THRESH, np.array([0, 0, 0, 0])) == (False, 3)
    assert lp.check(O.RULE_VC_THRESH, np.array([0, 1, 0, 1])) == (True, 0)
    assert lp.check(O.RULE_VC_THRESH, np.array([1, 0, 0, 1])) == (False, 1)


# ---------------------------------------------------------------- multiway cut

def test_simplex_projection_matches_bisection():
    rng = np.random.default_rng(0)
    for _ in range(200):
        k = int(rng.integers(1, 12))
        v = rng.normal(0, 2, k)
        w = O.simplex_project(v)
        lo, hi = v.min() - 1, v.max()
        for _ in range(200):
            th = 0.5 * (lo + hi)
            if np.maximum(v - th, 0).sum() > 1:
                lo = th
            else:
                hi = th
        ref = np.maximum(v - 0.5 * (lo + hi), 0)
        assert np.allclose(w, ref, atol=1e-12)
        assert w.sum() == pytest.approx(1.0, abs=1e-12)


def test_multiway_cut_small_grid():
    inst = I.mc_grid(side=8, k=3, seed=1)
    lp = O.OracleLP(inst)
    s = O.OracleSolver(lp, beta=10.0)
    F = s.run(60, trace=True)
    assert np.all(np.diff(F) <= 1e-12 * np.abs(F[:-1]))
    x = s.x
    k = inst.block_k
    nv = inst.meta["n_vertices"]
    X = x[: nv * k].reshape(nv, k)
    assert np.allclose(X.sum(axis=1), 1.0, atol=1e-12)
    assert X.min() >= 0
    term = inst.meta["terminals"]
    assert np.array_equal(np.argmax(X[term], axis=1), np.arange(k))
    m = s.metrics()
    assert m["dual_bound"] <= m["F"] + 1e-12
    sol, cost, _ = lp.round(x, O.RULE_MC_CKR, seed=2, reps=10)
    assert lp.check(O.RULE_MC_CKR, sol) == (True, 0)
    assert np.array_equal(sol[term], np.arange(k))
    # cut cost recomputed from the edge list
    e = inst.meta["edges"]
    cut = inst.meta["edge_w"][sol[e[:, 0]] != sol[e[:, 1]]].sum()
    assert cost == pytest.approx(cut, rel=1e-12)
    # integral labelling is reproduced
    lab = sol.copy()
    Xi = np.zeros_like(X)
    Xi[np.arange(nv), lab] = 1
    xi = x.copy()
    xi[: nv * k] = Xi.reshape(-1)
    sol2, _, _ = lp.round(xi, O.RULE_MC_CKR, seed=5, reps=3)
    assert np.array_equal(sol2, lab)


def test_multiway_cut_two_terminals_is_min_cut():
    """k=2 on a path: the LP is integral; CKR recovers the cheapest edge."""
    n = 6
    edges = np.array([[i, i + 1] for i in range(n - 1)])
    w = np.array([5.0, 3.0, 0.5, 4.0, 6.0])
    inst = I.mc_grid_lp(n, edges, w, np.array([0, n - 1]))
    lp = O.OracleLP(inst)
    s = O.OracleSolver(lp, beta=100.0)
    for _ in range(50):
        s.run(200)
        if s.metrics()["gap"] < 1e-12:
            break
    sol, cost, _ = lp.round(s.x, O.RULE_MC_CKR, seed=0, reps=10)
    assert cost == pytest.approx(0.5)
    assert list(sol) == [0, 0, 0, 1, 1, 1]


# ---------------------------------------------------------------- generators

def test_er_generator():
    e = I.er_edges(1000, 5000, 0)
    assert e.shape == (5000, 2)
    assert np.all(e[:, 0] < e[:, 1])
    assert len({tuple(r) for r in e.tolist()}) == 5000
    assert np.array_equal(e, I.er_edges(1000, 5000, 0))


def test_ba_generator():
    n = 20000
    e = I.ba_edges(n, 3)
    assert e.shape[0] == 6 + 3 * (n - 4)
    deg = np.bincount(e.reshape(-1), minlength=n)
    assert deg.min() == 3
    s = np.sort(e, axis=1)
    assert np.all(s[:, 0] != s[:, 1])
    assert len(np.unique(s[:, 0] * n + s[:, 1])) == len(s)
    # every new vertex attaches to earlier vertices
    assert np.all(e[6:, 1] < e[6:, 0])
    # heavy tail: hubs far above the mean degree 6
    assert deg.max() > 100


@pytest.mark.parametrize("n,d", [(200, 3), (1000, 16), (501, 5)])
def test_regular_generator(n, d):
    inst = I.mis_regular(n, d, seed=7)
    e = inst.meta["edges"]
    deg = np.bincount(e.reshape(-1), minlength=inst.n)
    assert np.all(deg == d)
    assert np.all(e[:, 0] < e[:, 1])
    assert len(np.unique(e[:, 0] * inst.n + e[:, 1])) == len(e)


def test_grid_generator():
    e = I.grid_edges(1024)
    assert e.shape[0] == 2 * 1024 * 1023
    inst = I.mc_grid(side=16, k=8, seed=0)
    assert inst.n == 16 * 16 * 8 + 2 * 16 * 15 * 8
    assert inst.m == 2 * 2 * 16 * 15 * 8
    assert len(np.unique(inst.meta["terminals"])) == 8


def test_oracle_rejects_bad_indices():
    inst = I.vc_lp(3, np.array([[0, 1]]), np.ones(3))
    inst.col_idx = inst.col_idx.copy()
    inst.col_idx[1] = 7
    with pytest.raises(ValueError):
        O.OracleLP(inst)


def _shared_row_block_instance():
    """Rows x_0 + x_2 >= 1 and x_1 + x_2 >= 1; the block of columns 1, 2
    has both in the second row."""
    return I.LPInstance(m=2, n=3, row_ptr=np.array([0, 2, 4], np.int64),
                        col_idx=np.array([0, 2, 1, 2], np.int32), val=None,
                        b=np.ones(2), c=np.ones(3), u=np.ones(3), sense=np.ones(2, np.int8),
                        block_first_col=np.array([1], np.int64), block_k=2,
                        fixed_label=np.array([-1], np.int32))


def test_blocks_whose_columns_share_a_row_are_rejected():
    """The block minimiser of Appendix E is taken on a diagonal block of
    A^T A; a row holding two columns of one block breaks that form and the
    instance is refused."""
    with pytest.raises(ValueError):
        O.OracleLP(_shared_row_block_instance())
    ok = _shared_row_block_instance()
    ok.block_first_col = np.array([0], np.int64)    # columns 0, 1 never share a row
    O.OracleLP(ok)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_block_step_is_the_exact_block_minimiser(seed):
    """On the multiway-cut grid every column of a pixel block has the same
    norm, so the block step (projection onto the simplex of y - g/L_B,
    Appendix E) minimises F over the block exactly.  Checked against an
    SLSQP minimisation over the simplex of F written densely from the
    matrix (c^T x + beta/2 ||A y - b||^2)."""
    inst = I.mc_grid(side=5, k=3, seed=seed)
    lp = O.OracleLP(inst)
    s = O.OracleSolver(lp, beta=10.0, seed=seed)
    s.run(2)
    kind, uid, _ = lp.units()
    A, beta, k = dense_aug(inst), 10.0, inst.block_k

    def F(y):
        w = A @ y - inst.b
        return inst.c @ y[: inst.n] + 0.5 * beta * w @ w

    rng = np.random.default_rng(seed)
    for t in rng.choice(np.flatnonzero(kind == 1), 4, replace=False):
        y0 = s.y
        j0 = int(inst.block_first_col[uid[t]])
        s.step_unit(int(t))
        y1 = s.y

        def Fb(v):
            y = y0.copy()
            y[j0:j0 + k] = v
            return F(y)

        best = None
        for start in [y0[j0:j0 + k], np.full(k, 1.0 / k)]:
            res = minimize(Fb, start, method="SLSQP", bounds=[(0, 1)] * k,
                           constraints=[{"type": "eq", "fun": lambda v: v.sum() - 1.0}],
                           options={"ftol": 1e-15, "maxiter": 500})
            if best is None or res.fun < best.fun:
                best = res
        assert Fb(y1[j0:j0 + k]) <= best.fun + 1e-9 * max(1.0, abs(best.fun))
        assert np.allclose(y1[j0:j0 + k], best.x, atol=1e-6)
        other = np.ones(len(y0), bool)
        other[j0:j0 + k] = False
        assert np.array_equal(y1[other], y0[other])
