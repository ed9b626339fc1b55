"""Pins of the oracle's general covering/packing roundings (Appendix B and
C) against what the paper and plain mathematics fix:

  * q(P) of the covering lemma against brute-force enumeration of binary x
    and hand-computed rows;
  * the set-cover threshold rule reduces to the vertex-cover rule on graphs
    (f = 2) and keeps, on any point, a cover within f/(1-eps) of c^T x;
  * the covering scaling gives a feasible fractional point (the lemma) and
    the randomized rule always returns a cover, reproducing integral
    feasible points;
  * the packing alteration reduces to the independent-set rule on graphs,
    always returns a feasible packing, and matches a hand-worked row.
"""
import itertools

import numpy as np
import pytest

from oracle import oracle as O
from paper_1311_2661_amd import instances as I


def lp_from_rows(rows, b, c, sense):
    """Instance from a list of {column: value} rows."""
    n = len(c)
    row_ptr = [0]
    col, val = [], []
    for r in rows:
        for j in sorted(r):
            col.append(j)
            val.append(float(r[j]))
        row_ptr.append(len(col))
    m = len(rows)
    return I.LPInstance(m=m, n=n, row_ptr=np.array(row_ptr, np.int64), col_idx=np.array(col, np.int32),
                        val=np.array(val), b=np.array(b, float), c=np.array(c, float), u=np.ones(n),
                        sense=np.full(m, sense, np.int8))


def dense(inst):
    A = np.zeros((inst.m, inst.n))
    for i in range(inst.m):
        for e in range(inst.row_ptr[i], inst.row_ptr[i + 1]):
            A[i, inst.col_idx[e]] = 1.0 if inst.val is None else inst.val[e]
    return A


def brute_q(inst):
    A = dense(inst)
    q = np.inf
    for i in range(inst.m):
        if inst.b[i] <= 0:
            continue
        cols = np.nonzero(A[i])[0]
        for k in range(len(cols) + 1):
            for sub in itertools.combinations(cols, k):
                s = A[i, list(sub)].sum()
                if s < inst.b[i]:
                    q = min(q, inst.b[i] - s)
    return q


# ---------------------------------------------------------------- q(P)

@pytest.mark.parametrize("row,b,q", [({0: 2, 1: 2}, 3, 1.0), ({0: 3, 1: 3}, 5, 2.0), ({0: 4}, 3, 3.0),
                                     ({0: 2, 1: 4}, 5, 1.0), ({0: 1, 1: 1, 2: 1}, 2, 1.0),
                                     ({0: 5, 1: 7}, 11, 4.0), ({0: 6, 1: 10}, 15, 5.0)])
def test_cover_q_hand_rows(row, b, q):
    inst = lp_from_rows([row], [b], np.ones(max(row) + 1), 1)
    assert O.OracleLP(inst).cover_q() == q


@pytest.mark.parametrize("seed", range(6))
def test_cover_q_matches_enumeration(seed):
    rng = np.random.default_rng(seed)
    n, m = 9, 6
    rows = []
    for _ in range(m):
        cols = rng.choice(n, size=int(rng.integers(1, 7)), replace=False)
        rows.append({int(j): int(rng.integers(1, 9)) for j in cols})
    b = [int(rng.integers(1, 25)) for _ in range(m)]
    inst = lp_from_rows(rows, b, np.ones(n), 1)
    assert O.OracleLP(inst).cover_q() == brute_q(inst)


def test_cover_q_rejects_non_covering():
    inst = lp_from_rows([{0: 1.5, 1: 1}], [2], [1, 1], 1)
    assert O.OracleLP(inst).cover_q() == -1.0
    inst = lp_from_rows([{0: 1, 1: 1}], [1], [1, 1], -1)
    assert O.OracleLP(inst).cover_q() == -1.0


# ---------------------------------------------------------------- set cover threshold

@pytest.mark.parametrize("seed", range(4))
def test_cover_threshold_reduces_to_vertex_cover_rule(seed):
    rng = np.random.default_rng(seed)
    inst = I.vc_er(60, 200, seed=seed)
    lp = O.OracleLP(inst)
    x = rng.uniform(0, 1, inst.n)
    s1, c1, a1 = lp.round(x, O.RULE_VC_THRESH)
    s2, c2, a2 = lp.round(x, O.RULE_COVER_THRESH)
    assert np.array_equal(s1, s2) and c1 == c2 and a1[0] == a2[0]


@pytest.mark.parametrize("seed", range(5))
def test_cover_threshold_keeps_a_cover_within_f_over_one_minus_eps(seed):
    rng = np.random.default_rng(seed)
    inst = I.set_cover(300, 120, seed=seed, mean_size=5.0)
    lp = O.OracleLP(inst)
    A = dense(inst)
    f = int(np.diff(inst.row_ptr).max())
    for trial in range(5):
        x = rng.uniform(0, 1, inst.n) * rng.uniform(0.2, 1.0)
        sol, cost, aux = lp.round(x, O.RULE_COVER_THRESH)
        assert np.all(A @ sol >= 1.0)
        assert lp.check(O.RULE_COVER_THRESH, sol) == (True, 0)
        eps = max(0.0, float(np.max(1.0 - A @ x)))
        if eps < 1.0:
            assert cost <= f / (1.0 - eps) * inst.c @ x * (1 + 1e-12)
            assert aux[0] == pytest.approx((1.0 - eps) / f, rel=1e-12)


def test_cover_threshold_on_a_feasible_point_is_hochbaums_rule():
    # every element in at most f sets: keeping x_s >= 1/f covers (x feasible)
    inst = lp_from_rows([{0: 1, 1: 1, 2: 1}, {2: 1, 3: 1}, {0: 1, 3: 1}], [1, 1, 1], [3, 1, 2, 1], 1)
    lp = O.OracleLP(inst)
    x = np.array([0.3, 0.5, 0.3, 0.7])
    sol, cost, aux = lp.round(x, O.RULE_COVER_THRESH)
    assert aux[0] == pytest.approx(1 / 3)
    assert list(sol) == [0, 1, 0, 1] and cost == 2.0


# ---------------------------------------------------------------- randomized covering

@pytest.mark.parametrize("maker", [lambda s: I.set_cover(250, 100, seed=s, mean_size=4.0),
                                   lambda s: I.multicover(200, 90, seed=s, mean_size=6.0)])
@pytest.mark.parametrize("seed", range(3))
def test_cover_random_always_covers_and_scaling_is_feasible(maker, seed):
    rng = np.random.default_rng(seed + 10)
    inst = maker(seed)
    lp = O.OracleLP(inst)
    A = dense(inst)
    q = lp.cover_q()
    assert q >= 1.0
    for trial in range(4):
        x = rng.uniform(0, 1, inst.n) * rng.uniform(0.5, 1.0)
        sol, cost, aux = lp.round(x, O.RULE_COVER_RAND, seed=trial, reps=3)
        assert np.all(A @ sol >= inst.b)
        assert cost == pytest.approx(inst.c @ sol, rel=1e-12)
        eps = max(0.0, float(np.max(inst.b - A @ x)))
        assert aux[0] == pytest.approx(eps / q, rel=1e-12)
        if aux[0] < 1.0:
            # covering lemma: the scaled point is feasible, cost within 1/(1-alpha)
            xt = np.minimum(1.0, x / (1.0 - aux[0]))
            assert np.all(A @ xt >= inst.b - 1e-9)
            assert inst.c @ xt <= inst.c @ x / (1.0 - aux[0]) * (1 + 1e-12)


def test_cover_random_reproduces_integral_feasible_points():
    inst = I.multicover(150, 60, seed=4, mean_size=6.0)
    lp = O.OracleLP(inst)
    x = np.ones(inst.n)
    A = dense(inst)
    rng = np.random.default_rng(0)
    # drop sets while the point stays feasible
    for j in rng.permutation(inst.n):
        x[j] = 0.0
        if np.any(A @ x < inst.b):
            x[j] = 1.0
    sol, cost, aux = lp.round(x, O.RULE_COVER_RAND, seed=3, reps=2)
    assert aux[0] == 0.0
    assert np.array_equal(sol, x.astype(np.int32))


def test_cover_random_completes_short_rows_by_decreasing_x():
    # one row, b = 2, entries 1, 1, 1, 1, x = (1, 0.3, 0.3, 0.4): feasible, so
    # alpha = 0 and one round (ceil(ln 2)); set 0 is always drawn.  When the
    # draws leave the row short, completion takes the largest remaining x,
    # ties by entry order: set 3, else set 1.
    inst = lp_from_rows([{0: 1, 1: 1, 2: 1, 3: 1}], [2], [1, 1, 1, 1], 1)
    lp = O.OracleLP(inst)
    x = np.array([1.0, 0.3, 0.3, 0.4])
    seen = set()
    for seed in range(40):
        w = [O.philox(np.array([0, j, 16, 0], np.uint64), np.array([seed, 4], np.uint64))[0] for j in range(4)]
        drawn = {j for j in range(4) if (int(w[j]) >> 11) * 2.0 ** -53 < x[j]}
        want = set(drawn)
        if len(drawn) < 2:
            want.add(3 if 3 not in drawn else 1)
        sol, cost, aux = lp.round(x, O.RULE_COVER_RAND, seed=seed, reps=1)
        assert aux[0] == 0.0
        assert set(np.nonzero(sol)[0]) == want
        seen.add(len(drawn))
    assert 1 in seen and 2 in seen


@pytest.mark.parametrize("x,alpha", [((0.75, 0.75), 0.5), ((0.6, 0.9), 0.5), ((0.9, 0.95), 0.15)])
def test_cover_random_scales_by_eps_over_q(x, alpha):
    """The covering lemma's alpha = eps / q(P): the row 2 x0 + 2 x1 >= 4 has
    q = 4 - 2 = 2 (its subset sums are 0, 2, 4), so a violation eps gives
    alpha = eps / 2."""
    inst = lp_from_rows([{0: 2, 1: 2}], [4], [1, 1], 1)
    lp = O.OracleLP(inst)
    assert lp.cover_q() == 2.0
    sol, cost, aux = lp.round(np.array(x), O.RULE_COVER_RAND, seed=0, reps=1)
    assert aux[0] == pytest.approx(alpha, abs=1e-15)


def test_cover_random_takes_the_union_of_ceil_ln_2m_rounds():
    """Four rows of two sets each (b = 1, x = 0.3 everywhere): the union is
    over t = ceil(ln 8) = 3 rounds of draws (reading R23: each row then stays
    short with probability at most 1/(2m)); a row the draws leave uncovered
    takes its larger scaled x, ties to the first entry.  Reproduced from
    explicit Philox draws for 30 seeds."""
    m = 4
    inst = lp_from_rows([{2 * i: 1, 2 * i + 1: 1} for i in range(m)], [1] * m, [1] * (2 * m), 1)
    lp = O.OracleLP(inst)
    x = np.full(2 * m, 0.3)
    t = int(np.ceil(np.log(2.0 * m)))
    assert t == 3
    for seed in range(30):
        sol, cost, aux = lp.round(x, O.RULE_COVER_RAND, seed=seed, reps=1)
        assert aux[0] == pytest.approx(0.4, abs=1e-15)
        xt = np.minimum(1.0, x / (1.0 - aux[0]))
        drawn = set()
        for j in range(2 * m):
            for r in range(t):
                w = O.philox(np.array([0, j, 16 + r, 0], np.uint64), np.array([seed, 4], np.uint64))[0]
                if (int(w) >> 11) * 2.0 ** -53 < xt[j]:
                    drawn.add(j)
        want = set(drawn)
        for i in range(m):
            if 2 * i not in drawn and 2 * i + 1 not in drawn:
                want.add(2 * i)
        assert set(np.nonzero(sol)[0]) == want, seed


# ---------------------------------------------------------------- packing alteration

@pytest.mark.parametrize("seed", range(4))
def test_pack_rule_reduces_to_independent_set_rule(seed):
    rng = np.random.default_rng(seed)
    inst = I.mis_regular(80, 4, seed=seed)
    lp = O.OracleLP(inst)
    x = rng.uniform(0, 1, inst.n)
    s1, c1, a1 = lp.round(x, O.RULE_MIS_RAND, seed=seed, reps=5)
    s2, c2, a2 = lp.round(x, O.RULE_PACK_RAND, seed=seed, reps=5)
    assert np.array_equal(s1, s2) and c1 == c2 and a1[0] == a2[0] and a1[1] == a2[1]


@pytest.mark.parametrize("seed", range(4))
def test_pack_rule_always_feasible(seed):
    rng = np.random.default_rng(seed)
    inst = I.kcs_packing(150, 60, 3, seed=seed)
    lp = O.OracleLP(inst)
    A = dense(inst)
    for trial in range(4):
        x = rng.uniform(0, 1, inst.n)
        sol, cost, aux = lp.round(x, O.RULE_PACK_RAND, seed=trial, reps=4)
        assert np.all(A @ sol <= inst.b)
        assert cost == pytest.approx(inst.c @ sol, rel=1e-12)
        assert aux[0] == pytest.approx(max(0.0, float(np.max((A @ x - inst.b) / inst.b))), rel=1e-12)
        assert lp.check(O.RULE_PACK_RAND, sol) == (True, 0)


def test_pack_alteration_hand_worked_row():
    # one row, weights 5, 6, 3 against capacity 10 (w = 0.5, 0.6, 0.3); x = 1
    # gives alpha = 0.4.  Kept sets by hand for every chosen set C:
    expected = {(): (), (0,): (0,), (1,): (1,), (2,): (2,), (0, 1): (1,), (0, 2): (0, 2),
                (1, 2): (1, 2), (0, 1, 2): (1,)}
    inst = lp_from_rows([{0: 5, 1: 6, 2: 3}], [10], [-1, -1, -1], -1)
    lp = O.OracleLP(inst)
    x = np.ones(3)
    seen = set()
    for seed in range(40):
        w = [O.philox(np.array([0, j, 0, 0], np.uint64), np.array([seed, 4], np.uint64))[0] for j in range(3)]
        chosen = tuple(j for j in range(3) if (int(w[j]) >> 11) * 2.0 ** -53 < 1.0 / 1.4)
        sol, cost, aux = lp.round(x, O.RULE_PACK_RAND, seed=seed, reps=1)
        assert aux[0] == pytest.approx(0.4)
        assert tuple(np.nonzero(sol)[0]) == expected[chosen]
        seen.add(chosen)
    assert (0, 1, 2) in seen and (0, 1) in seen


def test_general_rules_reject_other_shapes():
    lp = O.OracleLP(I.vc_er(30, 60, seed=1))
    x = np.full(30, 0.5)
    with pytest.raises(ValueError):
        lp.round(x, O.RULE_PACK_RAND)
    lp = O.OracleLP(I.multicover(40, 20, seed=1))
    with pytest.raises(ValueError):
        lp.round(np.full(20, 0.5), O.RULE_COVER_THRESH)
