"""Property-based checks (hypothesis) of the oracle's roundings against the
rounding lemmas: any graph, any weights, any point in the box.

* Vertex cover (Section 2 rule with the scaling lemma of Appendix C): the
  threshold rounding always returns a cover, T = min(1/2, (1 - eps)/2), and
  when eps < 1 the scaled point x/(1 - eps) (clipped) satisfies every edge
  row and the cover costs at most twice its cost.
* Independent set (Appendix B, threshold and randomized alteration): always
  an independent set, whatever the point, and the reported cost is minus the
  kept weight.
* Set cover (Hochbaum's f-threshold on the covering scaling): always a cover,
  and with a feasible point the cost is at most f c^T x.
Shrinking reports the smallest failing instance if one of them breaks."""
import numpy as np
import pytest
from hypothesis import HealthCheck, given, settings
from hypothesis import strategies as st

from oracle import oracle as O
from paper_1311_2661_amd import instances as I

SETTINGS = settings(max_examples=150, deadline=None, derandomize=True, database=None,
                    suppress_health_check=[HealthCheck.too_slow])


@st.composite
def graphs(draw, max_n=12):
    n = draw(st.integers(2, max_n))
    pairs = [(u, v) for u in range(n) for v in range(u + 1, n)]
    chosen = draw(st.lists(st.sampled_from(pairs), min_size=1, max_size=len(pairs), unique=True))
    edges = np.array(sorted(chosen), dtype=np.int64)
    w = np.array(draw(st.lists(st.floats(0.5, 10.0), min_size=n, max_size=n)))
    x = np.array(draw(st.lists(st.floats(0.0, 1.0), min_size=n, max_size=n)))
    return n, edges, w, x


@SETTINGS
@given(graphs())
def test_vertex_cover_threshold_lemma(g):
    n, edges, w, x = g
    lp = O.OracleLP(I.vc_lp(n, edges, w))
    sol, cost, aux = lp.round(x, O.RULE_VC_THRESH)
    assert lp.check(O.RULE_VC_THRESH, sol) == (True, 0)
    assert np.all(sol[edges[:, 0]] | sol[edges[:, 1]])
    eps = max(0.0, float(np.max(1 - x[edges[:, 0]] - x[edges[:, 1]])))
    assert aux[0] == pytest.approx(min(0.5, (1 - eps) / 2), abs=1e-15)
    assert cost == pytest.approx(float(w @ sol))
    if eps < 1:
        # 1 - eps carries the rounding of eps (about one ulp of 1), which the
        # division magnifies by 1/(1 - eps) when every edge is nearly empty
        rel_err = 1e-12 + 4 * np.finfo(np.float64).eps / (1 - eps)
        xt = np.clip(x / (1 - eps), 0, 1)
        assert np.all(xt[edges[:, 0]] + xt[edges[:, 1]] >= 1 - rel_err)
        assert cost <= 2 * float(w @ xt) * (1 + rel_err) + 1e-9


@SETTINGS
@given(graphs(), st.integers(0, 2**31 - 1))
def test_independent_set_roundings_are_independent(g, seed):
    n, edges, w, x = g
    lp = O.OracleLP(I.mis_lp(n, edges, w))
    for rule in (O.RULE_MIS_THRESH, O.RULE_MIS_RAND):
        sol, cost, _ = lp.round(x, rule, seed=seed, reps=3)
        assert lp.check(rule, sol) == (True, 0)
        assert not np.any(sol[edges[:, 0]] & sol[edges[:, 1]])
        assert cost == pytest.approx(-float(w @ sol))


@st.composite
def set_systems(draw):
    n_sets = draw(st.integers(1, 8))
    n_elem = draw(st.integers(1, 10))
    rows = []
    for _ in range(n_elem):
        rows.append(sorted(draw(st.lists(st.integers(0, n_sets - 1), min_size=1, max_size=n_sets, unique=True))))
    c = np.array(draw(st.lists(st.floats(0.5, 10.0), min_size=n_sets, max_size=n_sets)))
    x = np.array(draw(st.lists(st.floats(0.0, 1.0), min_size=n_sets, max_size=n_sets)))
    return n_sets, rows, c, x


@SETTINGS
@given(set_systems())
def test_set_cover_threshold_covers_and_is_f_approximate_on_feasible_points(sys_):
    n_sets, rows, c, x = sys_
    row_ptr = np.zeros(len(rows) + 1, np.int64)
    row_ptr[1:] = np.cumsum([len(r) for r in rows])
    col_idx = np.array([j for r in rows for j in r], np.int32)
    inst = I.LPInstance(m=len(rows), n=n_sets, row_ptr=row_ptr, col_idx=col_idx, val=None,
                        b=np.ones(len(rows)), c=c, u=np.ones(n_sets), sense=np.ones(len(rows), np.int8))
    lp = O.OracleLP(inst)
    sol, cost, _ = lp.round(x, O.RULE_COVER_THRESH)
    assert lp.check(O.RULE_COVER_THRESH, sol) == (True, 0)
    for r in rows:
        assert any(sol[j] for j in r)
    f = max(len(r) for r in rows)
    if all(x[r].sum() >= 1.0 for r in map(np.array, rows)):
        assert cost <= f * float(c @ x) + 1e-9


def test_vertex_cover_threshold_when_every_edge_is_nearly_empty():
    """eps close to 1 (both ends of the edge near 0): the threshold rule still
    returns a cover (T is formed from fl(x_u + x_v)/2 directly), while the
    scaled point x/(1 - eps) meets its edge row only up to the rounding of
    1 - eps magnified by 1/(1 - eps)."""
    edges = np.array([[0, 1]])
    x = np.array([1e-9, 1e-9 + 3e-17])
    lp = O.OracleLP(I.vc_lp(2, edges, np.array([1.0, 2.0])))
    sol, cost, aux = lp.round(x, O.RULE_VC_THRESH)
    assert lp.check(O.RULE_VC_THRESH, sol) == (True, 0)
    assert aux[0] == pytest.approx((x[0] + x[1]) / 2, rel=1e-15)
    eps = 1 - x[0] - x[1]
    xt = np.clip(x / (1 - eps), 0, 1)
    assert abs(xt.sum() - 1) <= 4 * np.finfo(np.float64).eps / (1 - eps)
