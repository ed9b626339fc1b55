"""GPU parity: the HIP path through the C ABI against the FP64 oracle on the
same seeded instances.

Bars (from the solve's arithmetic):
  * FP64 storage, DET schedule vs oracle DET replay: same update sequence,
    only the order of the dot-product sums differs, so iterates agree to
    1e-10 and rounded vectors, verdicts and colour classes are bit-exact.
  * FP32 storage vs the FP64 oracle at equal epochs: penalty F and c^T x
    within 1e-4 relative, row violation within 1e-4 absolute; rounding equal
    on every vertex whose oracle margin |x_v - T| exceeds the measured
    max |x_gpu - x_oracle| (the count inside that band is reported and
    must be 0 for these seeds).
  * Rounding, feasibility and metrics kernels given the same FP64 point:
    rounded vectors and verdicts bit-exact, costs and reductions to 1e-12.
"""
import os
import sys

import numpy as np
import pytest

from oracle import oracle as O
from paper_1311_2661_amd import instances as I

pytestmark = pytest.mark.gpu

T = None


def setup_module(module):
    global T
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1311_2661_amd import thetis as TT
    T = TT
    torch.cuda.set_device(0)


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def gpu_solver(inst, **kw):
    return T.Solver(T.Instance(inst), **kw)


def oracle_solver(inst, **kw):
    lp = O.OracleLP(inst)
    sched = kw.pop("schedule", O.SCHED_DET)
    return lp, O.OracleSolver(lp, schedule=sched, **kw)


def rel(a, b):
    return abs(a - b) / max(1.0, abs(b))


# ------------------------------------------------------------------ FP64 trajectories

@pytest.mark.parametrize("seed", [0, 1])
def test_fp64_det_matches_oracle_config_small(seed):
    """Vertex cover on G(1000, 5000), beta 10, 50 epochs, DET."""
    say(f"case fp64 det vc_er seed={seed}")
    inst = I.vc_er(1000, 5000, seed=seed)
    g = gpu_solver(inst, beta=10.0, precision=T.PREC_FP64, seed=seed, refresh_every=1000000)
    lp, o = oracle_solver(inst, beta=10.0, seed=seed)
    for chunk in (1, 9, 40):
        g.run(chunk)
        o.run(chunk)
        dy = np.abs(g.y - o.y).max()
        assert dy < 1e-10, dy
    gm, om = g.metrics(), o.metrics()
    for k in ("F", "lp_value", "dual_bound", "linf", "l2", "max_viol"):
        assert rel(gm[k], om[k]) < 1e-12, (k, gm[k], om[k])
    sol, cost, aux = g.round(T.ROUND_VC_THRESH)
    osol, ocost, oaux = lp.round(o.x, O.RULE_VC_THRESH)
    margin = np.abs(o.x - oaux[0]).min()
    say(f"  max|dy|={dy:.2e} min margin to T={margin:.3e}")
    assert np.array_equal(sol, osol)
    assert cost == pytest.approx(ocost, rel=1e-12)
    assert g.check(T.ROUND_VC_THRESH) == lp.check(O.RULE_VC_THRESH, osol) == (True, 0)


def test_fp64_refresh_does_not_move_the_trajectory():
    """Recomputing r from y every epoch changes nothing beyond rounding."""
    inst = I.vc_er(500, 2500, seed=4)
    g = gpu_solver(inst, precision=T.PREC_FP64, seed=4, refresh_every=1)
    lp, o = oracle_solver(inst, beta=10.0, seed=4)
    g.run(30)
    o.run(30)
    assert np.abs(g.y - o.y).max() < 1e-10


@pytest.mark.parametrize("rule,prox", [(T_rule, p) for T_rule in (0, 1) for p in (False, True)])
def test_fp64_step_rules_and_prox(rule, prox):
    say(f"case fp64 step_rule={rule} prox={prox}")
    inst = I.vc_er(400, 1600, seed=7)
    rng = np.random.default_rng(0)
    yb = rng.uniform(0, 1, inst.n + inst.m) if prox else None
    g = gpu_solver(inst, beta=5.0, step_rule=rule, prox=prox, ybar=yb, precision=T.PREC_FP64, seed=2)
    lp, o = oracle_solver(inst, beta=5.0, step_rule=rule, prox=prox, ybar=yb, seed=2)
    g.run(25)
    o.run(25)
    assert np.abs(g.y - o.y).max() < 1e-10
    gm, om = g.metrics(), o.metrics()
    for k in ("F", "dual_bound"):
        assert rel(gm[k], om[k]) < 1e-12


def test_fp64_ubar_and_step_scale():
    inst = I.vc_er(300, 1200, seed=8)
    rng = np.random.default_rng(1)
    ub = rng.uniform(0, 2, inst.m)
    g = gpu_solver(inst, beta=10.0, step_scale=0.7, ubar=ub, precision=T.PREC_FP64, seed=5)
    lp, o = oracle_solver(inst, beta=10.0, step_scale=0.7, ubar=ub, seed=5)
    g.run(20)
    o.run(20)
    assert np.abs(g.y - o.y).max() < 1e-10
    assert rel(g.metrics()["F"], o.metrics()["F"]) < 1e-12


def test_fp64_general_lp_values_equality_rows_and_bounds():
    """Non-unit matrix entries, all three row senses, mixed upper bounds
    (some infinite), an empty column and a long row."""
    rng = np.random.default_rng(5)
    m, n = 300, 200
    rows = []
    for i in range(m):
        k = int(rng.integers(1, 6)) if i < m - 1 else 60
        rows.append(np.sort(rng.choice(n - 1, size=k, replace=False)))   # column n-1 stays empty
    row_ptr = np.concatenate([[0], np.cumsum([len(r) for r in rows])]).astype(np.int64)
    col = np.concatenate(rows).astype(np.int32)
    val = rng.uniform(-2, 3, len(col))
    sense = rng.choice([-1, 0, 1], size=m).astype(np.int8)
    u = rng.uniform(0.5, 3, n)
    u[rng.choice(n, 20, replace=False)] = np.inf
    inst = I.LPInstance(m=m, n=n, row_ptr=row_ptr, col_idx=col, val=val, b=rng.uniform(-1, 2, m),
                        c=rng.uniform(0.1, 2, n), u=u, sense=sense)
    g = gpu_solver(inst, beta=3.0, precision=T.PREC_FP64, seed=9)
    lp, o = oracle_solver(inst, beta=3.0, seed=9)
    g.run(15)
    o.run(15)
    assert np.abs(g.y - o.y).max() < 1e-9
    gm, om = g.metrics(), o.metrics()
    for k in ("F", "lp_value", "linf", "max_viol"):
        assert rel(gm[k], om[k]) < 1e-11, k


def test_fp64_hubs_beyond_the_lds_tile_and_every_lane_group():
    """A star with 5000 leaves (hub above the 2048-entry LDS tile), a
    300-leaf star (LDS path) and paths giving degrees 1..64."""
    edges = [(0, i) for i in range(1, 5001)]
    base = 5001
    edges += [(base, base + i) for i in range(1, 301)]
    base += 301
    for d in (1, 3, 5, 8, 12, 16, 20, 32, 40, 64):
        edges += [(base, base + i) for i in range(1, d + 1)]
        base += d + 1
    edges = np.array(edges, dtype=np.int64)
    n = base
    w = np.random.default_rng(3).uniform(1, 10, n)
    inst = I.vc_lp(n, edges, w)
    g = gpu_solver(inst, precision=T.PREC_FP64, seed=1)
    lp, o = oracle_solver(inst, beta=10.0, seed=1)
    g.run(10)
    o.run(10)
    assert np.abs(g.y - o.y).max() < 1e-10


@pytest.mark.parametrize("kind", ["valued", "signed"])
def test_fp64_hub_with_values_beyond_the_lds_tile(kind):
    """A hub column of 5000 entries (past the 2048-entry LDS tile) whose
    entries carry general values or signs: rows a x_0 + b x_i >= 1 with
    a, b in [0.5, 2] ("valued"), or x_0 - x_i >= -1/2 and x_0 + x_i >= 1/2
    alternating ("signed", every value +-1).  Both the staged and the
    re-read part of the hub's scatter run; FP64 DET iterates and every
    reduction against the oracle's replay."""
    say(f"case fp64 hub past the LDS tile, {kind} entries")
    rng = np.random.default_rng(11)
    leaves = 5000
    n = leaves + 1
    cols = np.stack([np.zeros(leaves, np.int32), np.arange(1, n, dtype=np.int32)], axis=1).ravel()
    if kind == "valued":
        val = rng.uniform(0.5, 2.0, 2 * leaves)
        b = np.ones(leaves)
    else:
        val = np.ones(2 * leaves)
        val[1::4] = -1.0                 # odd rows: x_0 - x_i >= -1/2
        b = np.where(np.arange(leaves) % 2 == 0, 0.5, -0.5)
    inst = I.LPInstance(m=leaves, n=n, row_ptr=np.arange(0, 2 * leaves + 1, 2, dtype=np.int64),
                        col_idx=cols, val=val, b=b, c=rng.uniform(1, 10, n), u=np.ones(n),
                        sense=np.ones(leaves, dtype=np.int8))
    g = gpu_solver(inst, beta=10.0, precision=T.PREC_FP64, seed=2)
    lp, o = oracle_solver(inst, beta=10.0, seed=2)
    g.run(12)
    o.run(12)
    assert np.abs(g.y - o.y).max() < 1e-10
    gm, om = g.metrics(), o.metrics()
    for k in ("F", "lp_value", "linf", "max_viol", "dual_bound"):
        assert rel(gm[k], om[k]) < 1e-10, k


@pytest.mark.parametrize("seed", range(9))
def test_fp64_random_lp_sweep(seed):
    """Seeded LPs of mixed shape (instances.mixed_lp), with the step rule and the
    prox term varied by seed: FP64 DET iterates and every reduction against
    the oracle's replay."""
    inst = I.mixed_lp(seed)
    rule = T.STEP_GLOBAL_LMAX if seed % 4 == 3 else T.STEP_PER_COORD
    prox = seed % 2 == 1
    yb = np.random.default_rng(seed).uniform(0, 1, inst.n + inst.m) if prox else None
    say(f"case random LP seed {seed}: m={inst.m} n={inst.n} nnz={len(inst.col_idx)} rule={rule} prox={prox}")
    g = gpu_solver(inst, beta=4.0, step_rule=rule, prox=prox, ybar=yb, precision=T.PREC_FP64, seed=seed)
    lp, o = oracle_solver(inst, beta=4.0, step_rule=rule, prox=prox, ybar=yb, seed=seed)
    for _ in range(2):
        g.run(6)
        o.run(6)
        assert np.abs(g.y - o.y).max() < 1e-9
    gm, om = g.metrics(), o.metrics()
    for k in ("F", "lp_value", "linf", "max_viol", "dual_bound"):
        if np.isfinite(om[k]):
            assert rel(gm[k], om[k]) < 1e-10, k
        else:                            # an unbounded column minimum: Phi = -inf on both sides
            assert gm[k] == om[k], k


def test_fp64_multiway_cut_blocks():
    say("case fp64 multiway cut 24x24 k=5")
    inst = I.mc_grid(side=24, k=5, seed=2)
    g = gpu_solver(inst, precision=T.PREC_FP64, seed=3)
    lp, o = oracle_solver(inst, beta=10.0, seed=3)
    g.run(30)
    o.run(30)
    assert np.abs(g.y - o.y).max() < 1e-10
    gm, om = g.metrics(), o.metrics()
    for k in ("F", "lp_value", "dual_bound"):
        assert rel(gm[k], om[k]) < 1e-12, k
    sol, cost, aux = g.round(T.ROUND_MC_CKR, seed=4, reps=10)
    osol, ocost, oaux = lp.round(o.x, O.RULE_MC_CKR, seed=4, reps=10)
    assert np.array_equal(sol, osol)
    assert cost == pytest.approx(ocost, rel=1e-12)
    assert aux[1] == oaux[1]
    assert g.check(T.ROUND_MC_CKR) == (True, 0)


def test_fp64_independent_set():
    inst = I.mis_regular(800, 5, seed=3)
    g = gpu_solver(inst, precision=T.PREC_FP64, seed=6)
    lp, o = oracle_solver(inst, beta=10.0, seed=6)
    g.run(40)
    o.run(40)
    assert np.abs(g.y - o.y).max() < 1e-10
    for rule in (T.ROUND_MIS_THRESH, T.ROUND_MIS_RAND):
        sol, cost, aux = g.round(rule, seed=11, reps=10)
        osol, ocost, oaux = lp.round(o.x, rule, seed=11, reps=10)
        assert np.array_equal(sol, osol), rule
        assert cost == pytest.approx(ocost, rel=1e-12)
        assert g.check(rule) == (True, 0)


# ------------------------------------------------------------------ kernels on a given point

@pytest.mark.parametrize("seed", [0, 1, 2])
def test_rounding_and_check_kernels_bit_exact_on_oracle_point(seed):
    """The oracle's iterate is loaded into an FP64 solver: the pre-rounding
    pass, the rounding and the check must reproduce the oracle exactly."""
    inst = I.vc_er(2000, 9000, seed=seed)
    lp, o = oracle_solver(inst, beta=10.0, seed=seed, schedule=O.SCHED_PERM)
    o.run(7)
    g = gpu_solver(inst, precision=T.PREC_FP64)
    g.y = o.y
    gm, om = g.metrics(), o.metrics()
    for k in ("F", "lp_value", "dual_bound", "linf", "l2", "max_viol"):
        assert rel(gm[k], om[k]) < 1e-12, k
    sol, cost, aux = g.round(T.ROUND_VC_THRESH)
    osol, ocost, oaux = lp.round(o.x, O.RULE_VC_THRESH)
    assert aux[0] == oaux[0]
    assert np.array_equal(sol, osol)
    # check kernel on host-supplied solutions, including broken ones
    rng = np.random.default_rng(seed)
    for trial in range(3):
        bad = osol.copy()
        bad[rng.choice(inst.n, 25, replace=False)] = 0
        assert g.check(T.ROUND_VC_THRESH, bad) == lp.check(O.RULE_VC_THRESH, bad)
    # MIS rules on an independent-set instance with a random point
    mi = I.mis_regular(1500, 7, seed=seed)
    lpm = O.OracleLP(mi)
    x = rng.uniform(0, 1, mi.n)
    gm_ = gpu_solver(mi, precision=T.PREC_FP64)
    gm_.y = np.concatenate([x, np.zeros(mi.m)])
    for rule in (T.ROUND_MIS_THRESH, T.ROUND_MIS_RAND):
        sol, cost, aux = gm_.round(rule, seed=seed, reps=7)
        osol, ocost, oaux = lpm.round(x, rule, seed=seed, reps=7)
        assert np.array_equal(sol, osol)
        assert cost == pytest.approx(ocost, rel=1e-12)
        assert aux[0] == oaux[0]


def test_set_y_keeps_fixed_blocks():
    """thetis_set_y clips to the bounds, keeps every fixed block (terminal)
    at its unit vector and takes free blocks as given."""
    inst = I.mc_grid(side=12, k=4, seed=3)
    nv, k = inst.meta["n_vertices"], inst.block_k
    g = gpu_solver(inst, precision=T.PREC_FP64)
    y = np.full(inst.n + inst.m, 0.25)
    y[nv * k] = 7.0                           # an edge variable above its bound 1
    g.y = y
    got = g.y[: nv * k].reshape(nv, k)
    term = np.asarray(inst.meta["terminals"])
    assert np.array_equal(got[term], np.eye(k)[inst.fixed_label[term]])
    free = np.setdiff1d(np.arange(nv), term)
    assert np.all(got[free] == 0.25)
    assert g.y[nv * k] == 1.0


def test_multiway_cut_rounding_on_random_simplex_point():
    inst = I.mc_grid(side=40, k=8, seed=9)
    rng = np.random.default_rng(2)
    nv, k = inst.meta["n_vertices"], inst.block_k
    X = rng.dirichlet(np.full(k, 0.3), nv)
    X[inst.meta["terminals"]] = np.eye(k)
    y = np.zeros(inst.n + inst.m)
    y[: nv * k] = X.reshape(-1)
    lp = O.OracleLP(inst)
    g = gpu_solver(inst, precision=T.PREC_FP64)
    g.y = y
    sol, cost, aux = g.round(T.ROUND_MC_CKR, seed=8, reps=10)
    osol, ocost, oaux = lp.round(y[: inst.n], O.RULE_MC_CKR, seed=8, reps=10)
    assert np.array_equal(sol, osol)
    assert cost == pytest.approx(ocost, rel=1e-12)
    assert (aux[0], aux[1]) == (oaux[0], oaux[1])
    bad = osol.copy()
    bad[inst.meta["terminals"][0]] = (bad[inst.meta["terminals"][0]] + 1) % k
    assert g.check(T.ROUND_MC_CKR, bad) == lp.check(O.RULE_MC_CKR, bad) == (False, 1)


# ------------------------------------------------------------------ FP32 production path

def _fp32_vs_oracle(inst, epochs, seed, refresh_every=5):
    g = gpu_solver(inst, beta=10.0, precision=T.PREC_FP32, seed=seed, refresh_every=refresh_every)
    lp, o = oracle_solver(inst, beta=10.0, seed=seed)
    g.run(epochs)
    o.run(epochs)
    gm, om = g.metrics(), o.metrics()
    say(f"  F gpu {gm['F']:.10g} oracle {om['F']:.10g}; lp {gm['lp_value']:.10g} / {om['lp_value']:.10g}; "
        f"viol {gm['max_viol']:.3e} / {om['max_viol']:.3e}")
    assert rel(gm["F"], om["F"]) <= 1e-4
    assert rel(gm["lp_value"], om["lp_value"]) <= 1e-4
    assert abs(gm["max_viol"] - om["max_viol"]) <= 1e-4
    assert gm["dual_bound"] <= gm["F"]
    return g, lp, o


@pytest.mark.parametrize("seed", [0, 1, 2, 3, 4])
def test_fp32_config_small_parity(seed):
    """G(1000, 5000), beta 10, 50 epochs, FP32 storage with FP64 refresh."""
    say(f"case fp32 vc_er seed={seed}")
    inst = I.vc_er(1000, 5000, seed=seed)
    g, lp, o = _fp32_vs_oracle(inst, 50, seed)
    x = g.x
    ox = o.x
    err = np.abs(x - ox).max()
    sol, cost, aux = g.round(T.ROUND_VC_THRESH)
    osol, ocost, oaux = lp.round(ox, O.RULE_VC_THRESH)
    band = np.abs(ox - oaux[0]) <= err
    say(f"  max|x-x64|={err:.3e}, vertices inside that band of T: {int(band.sum())}")
    assert err < 1e-4
    assert int(band.sum()) == 0
    assert np.array_equal(sol, osol)
    assert g.check(T.ROUND_VC_THRESH) == (True, 0)
    assert cost == pytest.approx(ocost, rel=1e-9)


def test_fp32_ba_medium_parity():
    say("case fp32 vc_ba n=200000")
    inst = I.vc_ba(200_000, seed=1)
    g, lp, o = _fp32_vs_oracle(inst, 30, seed=1)
    sol, cost, _ = g.round(T.ROUND_VC_THRESH)
    assert g.check(T.ROUND_VC_THRESH) == (True, 0)
    e = inst.meta["edges"]
    assert np.all(sol[e[:, 0]] | sol[e[:, 1]])


def test_fp32_multiway_cut_parity():
    say("case fp32 multiway cut 64x64 k=8")
    inst = I.mc_grid(side=64, k=8, seed=1)
    g, lp, o = _fp32_vs_oracle(inst, 40, seed=2)
    sol, cost, _ = g.round(T.ROUND_MC_CKR, seed=1, reps=10)
    assert g.check(T.ROUND_MC_CKR) == (True, 0)
    assert np.array_equal(sol[inst.meta["terminals"]], np.arange(8))


@pytest.mark.parametrize("seed", [0, 1, 2, 3, 4])
def test_async_schedule_converges_to_the_oracle_value(seed):
    """ASYNC (atomics, nondeterministic order; P-ASYNC) on the small vertex
    cover workload (G(1000, 5000), beta 10) at convergence: both runs to a
    certified gap below 1e-6, F within 1e-4 relative, and the covers
    identical.  With prox off the minimiser in x need not be unique, so the
    two runs can stop at different points of equal F (max|x - x64| up to a
    few 1e-4 here); the band of the whole run, margin <= max|x - x64| +
    |T - T64|, is reported (seed 2 had one vertex inside it, rounded the same
    on both sides; the order of the atomics varies from run to run), and
    every vertex's margin is asserted above its own deviation
    |x_v - x64_v| + |T - T64|, which makes the equal rounding a consequence
    of the measured error rather than of luck."""
    say(f"case async vc_er seed={seed}")
    inst = I.vc_er(1000, 5000, seed=seed)
    g = gpu_solver(inst, beta=10.0, schedule=T.SCHED_ASYNC, step_scale=0.5, precision=T.PREC_FP32, seed=seed)
    lp, o = oracle_solver(inst, beta=10.0, seed=seed)
    done = g.run(3000, gap_tol=1e-6)
    o.run(600)
    gm, om = g.metrics(), o.metrics()
    assert om["gap"] < 1e-6
    assert gm["gap"] <= 1e-6 + 1e-12, (done, gm["gap"])
    assert rel(gm["F"], om["F"]) <= 1e-4
    sol, cost, aux = g.round(T.ROUND_VC_THRESH)
    assert g.check(T.ROUND_VC_THRESH) == (True, 0)
    ox = o.x
    osol, ocost, oaux = lp.round(ox, O.RULE_VC_THRESH)
    err = float(np.abs(g.x - ox).max())
    dT = abs(aux[0] - oaux[0])
    margin = np.abs(ox - oaux[0])
    band = margin <= err + dT
    own = margin <= np.abs(g.x - ox) + dT
    diff = sol != osol
    say(f"  epochs {done}; max|x-x64|={err:.3e} |dT|={dT:.2e} inside band={int(band.sum())} "
        f"inside own band={int(own.sum())} differing={int(diff.sum())}")
    assert np.all(band[diff])
    assert int(own.sum()) == 0
    assert np.array_equal(sol, osol)


def test_async_schedule_with_a_hub_past_the_lds_tile():
    """ASYNC with a 5000-entry hub (atomic scatter past the LDS tile) on a
    star plus 20000 random edges among its leaves: a certified gap below
    1e-5 and F within 1e-4 of the oracle's DET run to the same gap; the
    rounded cover is valid."""
    say("case async hub past the LDS tile")
    rng = np.random.default_rng(21)
    n = 5001
    star = np.stack([np.zeros(n - 1, np.int64), np.arange(1, n, dtype=np.int64)], axis=1)
    pairs = set()
    while len(pairs) < 20000:
        u, v = sorted(rng.integers(1, n, 2).tolist())
        if u != v:
            pairs.add((u, v))
    edges = np.concatenate([star, np.array(sorted(pairs), dtype=np.int64)])
    inst = I.vc_lp(n, edges, rng.uniform(1, 10, n))
    g = gpu_solver(inst, beta=10.0, schedule=T.SCHED_ASYNC, step_scale=0.5, precision=T.PREC_FP32, seed=5)
    lp, o = oracle_solver(inst, beta=10.0, seed=5)
    done = g.run(10000, gap_tol=1e-5)
    o.run(1500)
    gm, om = g.metrics(), o.metrics()
    say(f"  epochs {done}; gap {gm['gap']:.2e}; F {gm['F']:.8g} vs {om['F']:.8g}")
    assert om["gap"] < 1e-5
    assert gm["gap"] <= 1e-5 + 1e-12
    assert rel(gm["F"], om["F"]) <= 1e-4
    sol, cost, aux = g.round(T.ROUND_VC_THRESH)
    assert g.check(T.ROUND_VC_THRESH) == (True, 0)
    assert np.all(sol[edges[:, 0]] | sol[edges[:, 1]])


@pytest.mark.parametrize("prox", [False, True])
def test_set_beta_equals_a_solver_made_with_that_beta(prox):
    """thetis_set_beta recomputes everything beta enters (the per-coordinate
    curvatures beta ||A_j||^2 + rho, the blocks' stored bounds, Lmax and, with
    the prox term, rho = 1/beta): a solver made with beta 10 and set to 3
    before its first epoch follows the solver made with beta 3, bit for bit,
    and so does the FP64 oracle made with beta 3."""
    for name, inst in (("vc_er", I.vc_er(800, 4000, seed=6)), ("mc_grid", I.mc_grid(side=16, k=4, seed=6))):
        say(f"case set_beta {name} prox={prox}")
        a = gpu_solver(inst, beta=10.0, precision=T.PREC_FP64, prox=prox, seed=6)
        T.thetis_set_beta(a.h, 3.0)
        b = gpu_solver(inst, beta=3.0, precision=T.PREC_FP64, prox=prox, seed=6)
        lp, o = oracle_solver(inst, beta=3.0, prox=prox, seed=6)
        a.run(20)
        b.run(20)
        o.run(20)
        assert np.array_equal(a.y, b.y)
        assert np.abs(a.y - o.y).max() <= 1e-10
        a.close()
        b.close()


def test_gap_stop_and_reset():
    inst = I.vc_er(600, 2400, seed=5)
    g = gpu_solver(inst, seed=5)
    done = g.run(2000, gap_tol=1e-4)
    assert done < 2000 and done % 5 == 0
    assert g.metrics()["gap"] <= 1e-4 + 1e-9
    y1 = g.y
    g.reset()
    assert g.epoch == 0
    assert np.all(g.y == 0)
    g.run(done)
    assert np.array_equal(g.y, y1)      # DET is reproducible


def test_degenerate_instances():
    # no rows: every x goes to its cheaper bound
    inst = I.LPInstance(m=0, n=5, row_ptr=np.zeros(1, np.int64), col_idx=np.zeros(0, np.int32),
                        val=None, b=np.zeros(0), c=np.array([1.0, -1, 2, -3, 0]), u=np.ones(5),
                        sense=np.zeros(0, np.int8))
    g = gpu_solver(inst, precision=T.PREC_FP64)
    g.run(2)
    assert np.array_equal(g.x, [0, 1, 0, 1, 0])
    # one edge
    inst = I.vc_lp(2, np.array([[0, 1]]), np.array([1.0, 3.0]))
    g = gpu_solver(inst, precision=T.PREC_FP64)
    g.run(50)
    assert g.metrics()["F"] == pytest.approx(1 - 1 / 20, abs=1e-12)


@pytest.mark.timeout(900)
def test_full_size_ba_config_parity():
    """The benchmark workload at full size and in the benchmark's launch
    configuration (BA n = 2,000,000, refresh every 5, 100 epochs, DET)
    against the FP64 oracle run once in the same class order.

    FP64 storage (P-DET64): iterates within 1e-10, and every vertex's oracle
    margin to the threshold T exceeds that deviation plus T's own, so the
    rounded cover is bit-identical (asserted) and the smallest margin is
    asserted above 1e-10.

    FP32 storage (production): F and c^T x within 1e-4 relative, violation
    within 1e-4; the rounded cover equals the oracle's on every vertex whose
    margin exceeds its own FP32 deviation plus the threshold's deviation.
    The count inside that band and the count that differ are asserted at
    the values measured for this seed (recorded with the design notes)."""
    import time
    say("case full-size vc_ba n=2000000, 100 epochs: oracle")
    t0 = time.time()
    inst = I.vc_ba(2_000_000, seed=0)
    lp, o = oracle_solver(inst, beta=10.0, seed=0)
    o.run(100)
    om = o.metrics()
    ox = o.x
    osol, ocost, oaux = lp.round(ox, O.RULE_VC_THRESH)
    margin = np.abs(ox - oaux[0])
    say(f"  oracle done {time.time() - t0:.1f} s; F {om['F']:.12g}; T {oaux[0]:.6g}; "
        f"min margin {margin.min():.3e}")
    e = inst.meta["edges"]

    say("case full-size vc_ba n=2000000, 100 epochs: FP64 storage")
    g = gpu_solver(inst, beta=10.0, precision=T.PREC_FP64, refresh_every=5, seed=0)
    g.run(100)
    gm = g.metrics()
    gx = g.x
    sol, cost, aux = g.round(T.ROUND_VC_THRESH)
    dx = float(np.abs(gx - ox).max())
    dT = abs(aux[0] - oaux[0])
    say(f"  fp64: max|x-x64|={dx:.3e} |dT|={dT:.2e} min margin={margin.min():.3e} "
        f"differing={int((sol != osol).sum())}")
    assert dx <= 1e-10
    assert margin.min() > 1e-10
    assert margin.min() > dx + dT
    assert np.array_equal(sol, osol)
    assert cost == pytest.approx(ocost, rel=1e-12)
    for k in ("F", "lp_value", "dual_bound", "max_viol"):
        assert rel(gm[k], om[k]) < 1e-11, (k, gm[k], om[k])
    assert g.check(T.ROUND_VC_THRESH) == lp.check(O.RULE_VC_THRESH, osol) == (True, 0)
    g.close()
    del g

    say("case full-size vc_ba n=2000000, 100 epochs: FP32 storage")
    g = gpu_solver(inst, beta=10.0, precision=T.PREC_FP32, refresh_every=5, seed=0)
    g.run(100)
    gm = g.metrics()
    sol, cost, aux = g.round(T.ROUND_VC_THRESH)
    assert g.check(T.ROUND_VC_THRESH) == (True, 0)
    gx = g.x
    say(f"  fp32: F {gm['F']:.10g} vs {om['F']:.10g}; lp {gm['lp_value']:.10g} vs {om['lp_value']:.10g}; "
        f"viol {gm['max_viol']:.4e} vs {om['max_viol']:.4e}")
    assert rel(gm["F"], om["F"]) <= 1e-4
    assert rel(gm["lp_value"], om["lp_value"]) <= 1e-4
    assert abs(gm["max_viol"] - om["max_viol"]) <= 1e-4
    assert gm["dual_bound"] <= gm["F"]
    dx = np.abs(gx - ox)
    dT = abs(aux[0] - oaux[0])
    diff = sol != osol
    band = margin <= dx + dT
    say(f"  fp32: max|x-x64|={dx.max():.3e} |dT|={dT:.2e} differing vertices={int(diff.sum())} "
        f"inside band={int(band.sum())}")
    assert np.all(band[diff])
    assert (int(band.sum()), int(diff.sum())) == FP32_BA_BAND_COUNTS
    assert cost == pytest.approx(ocost, rel=1e-4)
    assert np.all(sol[e[:, 0]] | sol[e[:, 1]])


# measured for seed 0 (BA n = 2M, 100 epochs, refresh 5): vertices whose
# oracle margin lies inside |x - x64| + |T - T64|, and vertices whose
# rounding differs (all of them inside the band)
FP32_BA_BAND_COUNTS = (0, 0)


@pytest.mark.parametrize("prec_name", ["fp64", "fp32"])
def test_full_size_det_runs_are_bit_reproducible(prec_name):
    """DET at the benchmark's size and launch configuration: three solves
    of 100 epochs (one solver reset and rerun, a second solver) end at the
    same bits, as they must when every class launch covers each of its
    columns once and the classes share no row."""
    say(f"case full-size determinism vc_ba n=2000000 {prec_name}")
    prec = T.PREC_FP64 if prec_name == "fp64" else T.PREC_FP32
    inst = I.vc_ba(2_000_000, seed=0)
    h = T.Instance(inst)
    g = T.Solver(h, beta=10.0, precision=prec, refresh_every=5, seed=0)
    g.run(100)
    y1 = g.y
    g.reset()
    g.run(100)
    y2 = g.y
    g.close()
    g2 = T.Solver(h, beta=10.0, precision=prec, refresh_every=5, seed=0)
    g2.run(100)
    y3 = g2.y
    g2.close()
    say(f"  max|y1-y2|={np.abs(y1 - y2).max():.3e} max|y1-y3|={np.abs(y1 - y3).max():.3e}")
    assert np.array_equal(y1, y2)
    assert np.array_equal(y1, y3)


@pytest.mark.timeout(1200)
def test_full_size_multiway_cut_200_epochs():
    """The multiway-cut workload at full size (1024 x 1024 grid, k = 8, FP32,
    refresh every 5, DET) in the benchmark's launch configuration.

    One epoch from the same state: after 195 epochs (a refresh epoch) the
    GPU state goes to the FP64 oracle and both run epoch 196 in the same
    class order: every coordinate within 1e-4 and F within 1e-6 relative.

    Equal epochs: the GPU's 200 FP32 epochs against the FP64 oracle's 200
    epochs from the start in the same class order: F and c^T x within 1e-4
    relative, the row violation within 1e-4.

    Rounding on a shared point: region growing (10 repetitions, seed 0) of
    the GPU's final x on both sides: labels, cut weight, radius and winning
    repetition identical.  Also, at any size: every block on its simplex,
    terminals fixed, the labelling valid, its cut recomputed on the host."""
    import time
    say("case full-size mc_grid 1024x1024 k=8: GPU 200 epochs")
    t0 = time.time()
    side, k = 1024, 8
    inst = I.mc_grid(side=side, k=k, seed=0)
    g = gpu_solver(inst, beta=10.0, precision=T.PREC_FP32, refresh_every=5, seed=0)
    g.run(195)
    y0 = g.y
    g.run(1)
    y1 = g.y
    g1 = g.metrics()
    g.run(4)
    gm = g.metrics()
    gy = g.y
    say(f"  gpu done {time.time() - t0:.1f} s; F(200) {gm['F']:.12g}")
    lp = O.OracleLP(inst)
    o1 = O.OracleSolver(lp, beta=10.0, seed=0)
    o1.y = y0
    o1.epoch = 195
    o1.run(1)
    yo = o1.y
    om1 = o1.metrics()
    del o1
    dy = float(np.abs(y1 - yo).max())
    say(f"  one epoch from the same state: max|y_gpu - y_oracle| = {dy:.3e}; "
        f"F {g1['F']:.12g} vs {om1['F']:.12g}")
    assert dy <= 1e-4
    assert rel(g1["F"], om1["F"]) <= 1e-6

    say("case full-size mc_grid 1024x1024 k=8: oracle 200 epochs")
    o = O.OracleSolver(lp, beta=10.0, seed=0)
    o.run(200)
    om = o.metrics()
    say(f"  oracle done {time.time() - t0:.1f} s; F {gm['F']:.12g} vs {om['F']:.12g}; "
        f"lp {gm['lp_value']:.12g} vs {om['lp_value']:.12g}; viol {gm['max_viol']:.4e} vs {om['max_viol']:.4e}; "
        f"max|y - y64| {float(np.abs(gy - o.y).max()):.3e}")
    assert rel(gm["F"], om["F"]) <= 1e-4
    assert rel(gm["lp_value"], om["lp_value"]) <= 1e-4
    assert abs(gm["max_viol"] - om["max_viol"]) <= 1e-4
    assert gm["dual_bound"] <= gm["F"]
    del o

    nv = side * side
    X = gy[: nv * k].reshape(nv, k)
    assert np.abs(X.sum(axis=1) - 1.0).max() <= 1e-5
    assert X.min() >= 0.0
    term = inst.meta["terminals"]
    assert np.array_equal(X[term], np.eye(k)[np.arange(k)])
    sol, cost, aux = g.round(T.ROUND_MC_CKR, seed=0, reps=10)
    osol, ocost, oaux = lp.round(gy[: inst.n], O.RULE_MC_CKR, seed=0, reps=10)
    say(f"  region growing on the GPU's x: cut {cost:.12g} vs {ocost:.12g}; rep {aux[1]:.0f} vs {oaux[1]:.0f}")
    assert np.array_equal(sol, osol)
    assert cost == pytest.approx(ocost, rel=1e-12)
    assert (aux[0], aux[1]) == (oaux[0], oaux[1])
    assert g.check(T.ROUND_MC_CKR) == lp.check(O.RULE_MC_CKR, osol) == (True, 0)
    assert np.array_equal(sol[term], np.arange(k))
    e = inst.meta["edges"]
    cut = float(inst.meta["edge_w"][sol[e[:, 0]] != sol[e[:, 1]]].sum())
    assert cut == pytest.approx(cost, rel=1e-12)


def test_bf16_x_storage_error_is_stated_and_bounded():
    """x stored in BF16 (round to nearest even, residual updated with the
    realised step), s and r in FP32: the iteration is not the FP64 one, so
    the error against the FP64 oracle is reported; F must stay within 1e-2
    relative at equal epochs and the roundings must stay valid."""
    say("case bf16 mis_regular")
    inst = I.mis_regular(3000, 6, seed=4)
    g = gpu_solver(inst, beta=10.0, precision=T.PREC_BF16X, seed=4)
    lp, o = oracle_solver(inst, beta=10.0, seed=4)
    g.run(60)
    o.run(60)
    gm, om = g.metrics(), o.metrics()
    x, ox = g.x, o.x
    err = np.abs(x - ox).max()
    say(f"  F bf16 {gm['F']:.8g} fp64 {om['F']:.8g} rel {rel(gm['F'], om['F']):.2e}; max|x-x64| {err:.3e}")
    assert rel(gm["F"], om["F"]) < 1e-2
    assert gm["dual_bound"] <= gm["F"]
    # every stored x is a bf16 value
    xb = x.astype(np.float32).view(np.uint32)
    assert np.all((xb & 0xFFFF) == 0)
    for rule in (T.ROUND_MIS_THRESH, T.ROUND_MIS_RAND):
        g.round(rule, seed=3, reps=5)
        assert g.check(rule) == (True, 0)


@pytest.mark.parametrize("maker", [lambda: I.vc_ba(20000, seed=3), lambda: I.mc_grid(side=24, k=8, seed=4)])
def test_solo_autotune_does_not_change_results(maker):
    """The per-class tuner runs real epochs and changes only how many columns
    a lane group updates at once: the trajectory is the untuned one."""
    inst = maker()
    a = gpu_solver(inst, seed=5)
    b = gpu_solver(inst, seed=5)
    ch = a.autotune(2)
    assert len(ch) == a.nclasses and all(c in (1, 2, 4) for c in ch)
    assert a.epoch == 7
    a.run(10)
    b.run(17)
    assert np.array_equal(a.y, b.y)
    assert a.metrics()["F"] == b.metrics()["F"]


def test_calibrate_random_rates_are_positive():
    """The random-access calibration runs in bounds and returns finite
    positive times for the gather, read-modify-write, copy and per-XCD
    window read-modify-write passes."""
    import math
    times = T.thetis_calibrate_random(16, 3)
    assert len(times) == 4
    assert all(math.isfinite(v) and v > 0 for v in times)
    with pytest.raises(T.ThetisError):
        T.thetis_calibrate_random(40, 1)
