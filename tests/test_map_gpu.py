"""GPU parity of the MAP-inference LP (local polytope of a pairwise factor
graph) through the C ABI: the solve against the FP64 oracle (DET, 1e-9),
the node-based roundings bit-exact on the GPU's own x (exact in FP64),
energies to 1e-12; on a chain the outer loop plus the argmax rounding
returns the Viterbi labelling; the TAC-KBP-shaped graph of the MAP
experiments (12,000 boolean variables, 17,000 factors) at full size.
"""
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


def same_labels(g, lp, rule, seed, reps):
    sol, cost, aux = g.round(rule, seed=seed, reps=reps)
    osol, ocost, oaux = lp.round(g.x, rule, seed=seed, reps=reps)
    assert np.array_equal(sol, osol)
    assert cost == pytest.approx(ocost, rel=1e-12, abs=1e-12)
    assert aux[1] == oaux[1]
    assert g.check(rule) == lp.check(rule, osol) == (True, 0)
    return sol, cost


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


def test_fp64_solve_matches_oracle():
    say("case fp64 MAP LP chain+window 300 vars k=5 450 factors")
    inst = I.map_chain_window(300, 5, 450, seed=2)
    g = T.Solver(T.Instance(inst), beta=2.0, ubar=np.zeros(inst.m), precision=T.PREC_FP64, seed=2)
    lp = O.OracleLP(inst)
    o = O.OracleSolver(lp, beta=2.0, ubar=np.zeros(inst.m), seed=2)
    for _ in range(2):
        g.run(15)
        o.run(15)
        assert np.abs(g.y - o.y).max() < 1e-9
        gs, os_ = g.multiplier_step(), o.multiplier_step()
        for k in ("lp_value", "lp_dual"):
            assert abs(gs[k] - os_[k]) <= 1e-12 * max(1.0, abs(os_[k]))
    for rule, reps in ((T.ROUND_MAP_ARGMAX, 1), (T.ROUND_MAP_SAMPLE, 8)):
        same_labels(g, lp, rule, seed=3, reps=reps)


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_roundings_bit_exact_with_evidence(precision):
    inst = I.map_chain_window(2000, 7, 3500, seed=4)
    inst.fixed_label[::50] = 2
    prec = T.PREC_FP64 if precision == "fp64" else T.PREC_FP32
    g = T.Solver(T.Instance(inst), beta=2.0, precision=prec, seed=4)
    g.run(10)
    lp = O.OracleLP(inst)
    for rule, reps in ((T.ROUND_MAP_ARGMAX, 1), (T.ROUND_MAP_SAMPLE, 6)):
        sol, _ = same_labels(g, lp, rule, seed=9, reps=reps)
        assert np.all(sol[::50] == 2)


def test_chain_outer_loop_and_argmax_give_viterbi():
    n, k = 400, 6
    inst = I.map_chain_window(n, k, n - 1, seed=5)
    unary = inst.c[: n * k].reshape(n, k)
    trans = inst.c[n * k: n * k + k * k].reshape(k, k)
    e_min, lab = viterbi(unary, trans)
    g = T.Solver(T.Instance(inst), beta=2.0, ubar=np.zeros(inst.m), precision=T.PREC_FP64, seed=5)
    outer, epochs, st = g.run_multipliers(200, 100, feas_tol=1e-9, lp_gap_tol=1e-10)
    say(f"  chain: {outer} steps {epochs} epochs, LP {st['lp_value']:.12g} vs Viterbi {e_min:.12g}")
    assert st["lp_dual"] <= e_min + 1e-9
    sol, cost, _ = g.round(T.ROUND_MAP_ARGMAX)
    assert list(sol) == lab
    assert cost == pytest.approx(e_min, rel=1e-12)


def test_map_rules_need_pairwise_factors():
    g = T.Solver(T.Instance(I.mc_grid(side=8, k=3, seed=1)))
    with pytest.raises(T.ThetisError) as e:
        g.round(T.ROUND_MAP_ARGMAX)
    assert e.value.code == T.EINVAL


@pytest.mark.timeout(600)
def test_full_size_boolean_entity_linking_shape():
    """12,000 boolean variables and 17,000 factors (the entity-linking graph's
    size), FP32, outer loop, both roundings bit-exact against the oracle."""
    say("case full-size MAP 12000 boolean vars, 17000 factors")
    inst = I.map_chain_window(12000, 2, 17000, seed=0, window=40)
    g = T.Solver(T.Instance(inst), beta=2.0, ubar=np.zeros(inst.m), precision=T.PREC_FP32, seed=0)
    outer, epochs, st = g.run_multipliers(20, 50)
    lp = O.OracleLP(inst)
    for rule, reps in ((T.ROUND_MAP_ARGMAX, 1), (T.ROUND_MAP_SAMPLE, 10)):
        sol, cost = same_labels(g, lp, rule, seed=1, reps=reps)
        assert cost >= st["lp_dual"] - 1e-9 * abs(st["lp_dual"])
        say(f"  rule {rule}: energy {cost:.10g}, LP bound {st['lp_dual']:.10g}")
