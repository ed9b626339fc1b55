"""Pins of the MAP-inference LP (local polytope of a pairwise factor graph)
and the oracle's node-based roundings against what the mathematics fixes:

  * on a chain the local polytope is tight: HiGHS's LP optimum equals the
    minimum energy found by the Viterbi recursion, the oracle's
    augmented-Lagrangian solve reaches it, and the argmax rounding returns
    the Viterbi labelling;
  * the one-hot point of any labelling is feasible and its LP objective is
    the energy the rounding reports;
  * on a loopy graph, LP* <= the brute-force minimum energy <= the energy
    of either rounding;
  * label frequencies of the sampling rounding follow the node marginals;
    evidence is kept; argmax ties go to the lower label.
"""
import itertools

import numpy as np
import pytest
from scipy.optimize import linprog
from scipy.sparse import csr_matrix

from oracle import oracle as O
from paper_1311_2661_amd import instances as I


def lp_star(inst):
    A = csr_matrix((inst.val, inst.col_idx, inst.row_ptr), shape=(inst.m, inst.n))
    nb, k = len(inst.block_first_col), inst.block_k
    rows, cols = [], []
    for t, f in enumerate(inst.block_first_col):
        rows += [t] * k
        cols += list(range(f, f + k))
    S = csr_matrix((np.ones(len(rows)), (rows, cols)), shape=(nb, inst.n))
    from scipy.sparse import vstack
    res = linprog(inst.c, A_eq=vstack([A, S]), b_eq=np.concatenate([inst.b, np.ones(nb)]),
                  bounds=(0, 1), method="highs")
    assert res.status == 0
    return res.fun


def energy(inst, lab):
    k = inst.block_k
    nx = len(inst.block_first_col) * k
    en = sum(inst.c[t * k + lab[t]] for t in range(len(lab)))
    for e, (i, j) in enumerate(inst.pair_ends):
        en += inst.c[inst.pair_first[e] + lab[i] * k + lab[j]]
    return en


def one_hot(inst, lab):
    k = inst.block_k
    x = np.zeros(inst.n)
    for t, l in enumerate(lab):
        x[t * k + l] = 1.0
    for e, (i, j) in enumerate(inst.pair_ends):
        x[inst.pair_first[e] + lab[i] * k + lab[j]] = 1.0
    return x


def viterbi(unary, trans):
    n, k = unary.shape
    cost = unary[0].copy()
    back = np.zeros((n, k), int)
    for i in range(1, n):
        tot = cost[:, None] + trans
        back[i] = np.argmin(tot, axis=0)
        cost = tot[back[i], np.arange(k)] + unary[i]
    lab = [int(np.argmin(cost))]
    for i in range(n - 1, 0, -1):
        lab.append(int(back[i][lab[-1]]))
    return float(cost.min()), lab[::-1]


def solve(inst, outer=30, inner=200, beta=10.0):
    lp = O.OracleLP(inst)
    s = O.OracleSolver(lp, beta=beta, ubar=np.zeros(inst.m))
    st = None
    for _ in range(outer):
        s.run(inner)
        st = s.multiplier_step()
        if st["linf"] < 1e-9 and abs(st["lp_gap"]) < 1e-9:
            break
    return lp, s, st


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_chain_lp_is_tight_and_argmax_gives_viterbi(seed):
    n, k = 10, 3
    inst = I.map_chain_window(n, k, n - 1, seed=seed)
    unary = inst.c[: n * k].reshape(n, k)
    trans = inst.c[n * k: n * k + k * k].reshape(k, k)
    e_min, lab = viterbi(unary, trans)
    assert lp_star(inst) == pytest.approx(e_min, abs=1e-9)
    lp, s, st = solve(inst)
    assert st["lp_value"] == pytest.approx(e_min, abs=1e-6)
    assert st["lp_dual"] <= e_min + 1e-9
    sol, cost, aux = lp.round(s.x, O.RULE_MAP_ARGMAX)
    assert list(sol) == lab
    assert cost == pytest.approx(e_min, abs=1e-9)
    assert lp.check(O.RULE_MAP_ARGMAX, sol) == (True, 0)


@pytest.mark.parametrize("seed", [3, 4])
def test_one_hot_point_is_feasible_and_its_objective_is_the_energy(seed):
    inst = I.map_chain_window(15, 4, 25, seed=seed)
    lp = O.OracleLP(inst)
    rng = np.random.default_rng(seed)
    A = csr_matrix((inst.val, inst.col_idx, inst.row_ptr), shape=(inst.m, inst.n))
    for _ in range(5):
        lab = rng.integers(0, 4, 15)
        x = one_hot(inst, lab)
        assert np.all(A @ x == 0.0)
        sol, cost, _ = lp.round(x, O.RULE_MAP_ARGMAX)
        assert np.array_equal(sol, lab)
        assert cost == pytest.approx(inst.c @ x, rel=1e-13)
        assert cost == pytest.approx(energy(inst, lab), rel=1e-13)
        sol2, cost2, _ = lp.round(x, O.RULE_MAP_SAMPLE, seed=5, reps=3)
        assert np.array_equal(sol2, lab) and cost2 == cost


def test_loopy_graph_bounds_by_enumeration():
    side, k = 3, 3
    rng = np.random.default_rng(7)
    ends = np.array(I.grid_edges(side), dtype=np.int32)
    unary = rng.standard_normal((side * side, k))
    pair = np.stack([-0.8 * np.eye(k) + 0.3 * rng.standard_normal((k, k)) for _ in range(len(ends))])
    inst = I.map_lp(side * side, k, ends, unary, pair)
    best = min(energy(inst, lab) for lab in itertools.product(range(k), repeat=side * side))
    star = lp_star(inst)
    assert star <= best + 1e-9
    # the coupled marginals make the inner problem stiff at beta 10; the outer
    # loop at beta 1 reaches LP* exactly within tens of steps
    lp, s, st = solve(inst, outer=60, beta=1.0)
    assert st["lp_value"] == pytest.approx(star, abs=1e-9)
    assert st["lp_dual"] == pytest.approx(star, abs=1e-9)
    for rule, reps in ((O.RULE_MAP_ARGMAX, 1), (O.RULE_MAP_SAMPLE, 20)):
        sol, cost, _ = lp.round(s.x, rule, seed=1, reps=reps)
        assert cost >= best - 1e-12
        assert cost == pytest.approx(energy(inst, sol), rel=1e-13)


def test_sampling_follows_the_marginals_and_keeps_evidence():
    n, k = 4, 5
    inst = I.map_chain_window(n, k, n - 1, seed=9)
    inst.fixed_label[2] = 3
    lp = O.OracleLP(inst)
    rng = np.random.default_rng(0)
    x = np.zeros(inst.n)
    mus = rng.dirichlet(np.ones(k), n)
    x[: n * k] = mus.reshape(-1)
    counts = np.zeros((n, k))
    trials = 3000
    for seed in range(trials):
        sol, _, _ = lp.round(x, O.RULE_MAP_SAMPLE, seed=seed, reps=1)
        counts[np.arange(n), sol] += 1
    assert np.all(counts[2] == np.eye(k)[3] * trials)
    for t in (0, 1, 3):
        assert np.abs(counts[t] / trials - mus[t]).max() < 0.035


def test_argmax_ties_go_to_the_lower_label():
    inst = I.map_chain_window(3, 3, 2, seed=1)
    lp = O.OracleLP(inst)
    x = np.zeros(inst.n)
    x[:9] = [0.4, 0.4, 0.2, 0.1, 0.45, 0.45, 1 / 3, 1 / 3, 1 / 3]
    sol, _, _ = lp.round(x, O.RULE_MAP_ARGMAX)
    assert list(sol) == [0, 1, 0]


def test_map_rules_need_pairwise_factors():
    lp = O.OracleLP(I.mc_grid(side=5, k=3, seed=1))
    with pytest.raises(ValueError):
        lp.round(np.zeros(lp.n), O.RULE_MAP_ARGMAX)
