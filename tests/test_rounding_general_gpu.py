"""GPU parity of the general covering/packing roundings (Appendix B and C)
through the C ABI.  The rounding is a function of the stored x, which is
exact in FP64, so the oracle rounds the GPU's own x: rounded vectors,
thresholds, alphas and winning repetitions bit-exact, costs to 1e-12.
Then the solve itself on these instances against the oracle (FP64 DET to
1e-10), and the benchmark's full-size set-cover and packing instances.
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


RULES = {5: "COVER_THRESH", 6: "COVER_RAND", 7: "PACK_RAND"}


def same_rounding(g, lp, rule, seed, reps):
    sol, cost, aux = g.round(rule, seed=seed, reps=reps)
    osol, ocost, oaux = lp.round(g.x, rule, seed=seed, reps=reps)
    assert np.array_equal(sol, osol), RULES[rule]
    assert cost == pytest.approx(ocost, rel=1e-12, abs=1e-12)
    assert aux[0] == oaux[0] and aux[1] == oaux[1]
    assert g.check(rule) == lp.check(rule, osol) == (True, 0)
    return sol, cost, aux


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("epochs", [3, 40])
def test_set_cover_roundings_bit_exact(precision, epochs):
    say(f"case set cover 3000x1200 {precision} {epochs} epochs")
    inst = I.set_cover(3000, 1200, seed=5, mean_size=6.0)
    prec = T.PREC_FP64 if precision == "fp64" else T.PREC_FP32
    g = T.Solver(T.Instance(inst), precision=prec, seed=5)
    g.run(epochs)
    lp = O.OracleLP(inst)
    for rule, reps in ((T.ROUND_COVER_THRESH, 1), (T.ROUND_COVER_RAND, 5)):
        same_rounding(g, lp, rule, seed=7, reps=reps)


@pytest.mark.parametrize("epochs", [2, 30])
def test_integer_covering_random_rounding_bit_exact(epochs):
    """Non-unit integer entries and demands up to 4: q(P) from the host's
    subset sums, the scaling, the completion of short rows."""
    say(f"case multicover 2500x1000 {epochs} epochs")
    inst = I.multicover(2500, 1000, seed=6, mean_size=7.0)
    g = T.Solver(T.Instance(inst), precision=T.PREC_FP32, seed=6)
    g.run(epochs)
    lp = O.OracleLP(inst)
    same_rounding(g, lp, T.ROUND_COVER_RAND, seed=11, reps=6)


@pytest.mark.parametrize("epochs", [2, 30])
def test_weighted_packing_alteration_bit_exact(epochs):
    say(f"case kcs packing 3000 sets k=4 {epochs} epochs")
    inst = I.kcs_packing(3000, 1500, 4, seed=8)
    g = T.Solver(T.Instance(inst), precision=T.PREC_FP32, seed=8)
    g.run(epochs)
    lp = O.OracleLP(inst)
    same_rounding(g, lp, T.ROUND_PACK_RAND, seed=13, reps=6)


def test_general_rules_reduce_to_graph_rules_on_the_gpu():
    inst = I.vc_er(2000, 8000, seed=2)
    g = T.Solver(T.Instance(inst), seed=2)
    g.run(20)
    a = g.round(T.ROUND_VC_THRESH)
    b = g.round(T.ROUND_COVER_THRESH)
    assert np.array_equal(a[0], b[0]) and a[1] == b[1] and a[2][0] == b[2][0]
    inst = I.mis_regular(2000, 5, seed=3)
    g = T.Solver(T.Instance(inst), seed=3)
    g.run(20)
    a = g.round(T.ROUND_MIS_RAND, seed=4, reps=5)
    b = g.round(T.ROUND_PACK_RAND, seed=4, reps=5)
    assert np.array_equal(a[0], b[0]) and a[1] == b[1] and list(a[2]) == list(b[2])


def test_general_rules_reject_other_shapes():
    g = T.Solver(T.Instance(I.vc_er(100, 300, seed=1)))
    with pytest.raises(T.ThetisError) as e:
        g.round(T.ROUND_PACK_RAND)
    assert e.value.code == T.EINVAL
    g = T.Solver(T.Instance(I.multicover(100, 50, seed=1)))
    with pytest.raises(T.ThetisError) as e:
        g.round(T.ROUND_COVER_THRESH)
    assert e.value.code == T.EINVAL


def test_fp64_solve_on_set_cover_and_packing_matches_oracle():
    for inst in (I.set_cover(1500, 600, seed=9, mean_size=5.0), I.kcs_packing(1200, 700, 3, seed=9),
                 I.multicover(1000, 500, seed=9)):
        g = T.Solver(T.Instance(inst), precision=T.PREC_FP64, seed=9)
        lp = O.OracleLP(inst)
        o = O.OracleSolver(lp, beta=10.0, seed=9)
        g.run(25)
        o.run(25)
        assert np.abs(g.y - o.y).max() < 1e-10


# ------------------------------------------------------------------ full size

@pytest.mark.timeout(600)
def test_full_size_set_cover_roundings():
    """The set-cover workload (4,000,000 elements, 1,000,000 sets, FP32): the
    oracle rounds the GPU's x and agrees bit for bit."""
    import time
    say("case full-size set cover 4M x 1M")
    t0 = time.time()
    inst = I.set_cover(4_000_000, 1_000_000, seed=0)
    g = T.Solver(T.Instance(inst), precision=T.PREC_FP32, seed=0)
    g.run(50)
    say(f"  solve done {time.time() - t0:.1f} s")
    lp = O.OracleLP(inst)
    for rule, reps in ((T.ROUND_COVER_THRESH, 1), (T.ROUND_COVER_RAND, 3)):
        sol, cost, aux = same_rounding(g, lp, rule, seed=1, reps=reps)
        say(f"  {RULES[rule]}: cost {cost:.10g} aux {aux[0]:.6g} ({time.time() - t0:.1f} s)")


@pytest.mark.timeout(600)
def test_full_size_packing_rounding():
    import time
    say("case full-size k-column-sparse packing 2M sets, 1M elements, k = 4")
    t0 = time.time()
    inst = I.kcs_packing(2_000_000, 1_000_000, 4, seed=0)
    g = T.Solver(T.Instance(inst), precision=T.PREC_FP32, seed=0)
    g.run(50)
    lp = O.OracleLP(inst)
    sol, cost, aux = same_rounding(g, lp, T.ROUND_PACK_RAND, seed=1, reps=3)
    say(f"  PACK_RAND: profit {-cost:.10g} alpha {aux[0]:.6g} ({time.time() - t0:.1f} s)")
