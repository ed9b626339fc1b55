"""The figures the benchmark's roofline is built from.

The library reports, per kernel group, the launch count, the summed device
time and the algorithmic bytes of the launches of the timed epochs.  The
byte counts here are written out from the instance itself with the
per-column and per-slack costs of a coordinate update (Algorithm 1 applied
to one column: its row indices, the residual entries read and written, x
read and written, its cost; a slack reads and writes itself and its row's
residual), so the numerator of the reported bandwidth is checked against an
independent count, not against the library's own arithmetic."""
import numpy as np
import pytest

from paper_1311_2661_amd import instances as I
from paper_1311_2661_amd import thetis as T

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)


@pytest.mark.parametrize("prec", [T.PREC_FP32, T.PREC_FP64])
def test_vertex_cover_sweep_bytes_and_launch_counts(prec):
    say(f"case measurement vc_ba n=50000 prec={prec}")
    inst = I.vc_ba(50_000, seed=4)
    n, m = inst.n, inst.m
    entries = 2 * m                   # every edge row holds its two endpoints
    R = 8 if prec == T.PREC_FP64 else 4
    X = R
    # per column: schedule entry 4, packed entry pointers 8, x read and
    # written, the FP64 cost 8; per entry: row index 4, residual read and
    # written; per slack: s and r read and written
    per_col = 4 + 8 + 2 * X + 8
    per_entry = 4 + 2 * R
    per_slack = 4 * R
    g = T.Solver(T.Instance(inst), beta=10.0, precision=prec, refresh_every=5, seed=4)
    try:
        tr = g.traffic()
        assert tr["updates_per_epoch"] == n + m
        assert tr["sweep_bytes"] == per_col * n + per_entry * entries + per_slack * m

        epochs = 5
        g.set_timing(1)
        g.run(epochs)
        t = g.timing()
        g.set_timing(0)
        cols, slack, ref = t["k_sweep"], t["k_sweep_slack"], t["refresh (k_rows+k_dual+k_finalize)"]
        say(f"  k_sweep {cols}; slack {slack}; refresh {ref}")
        # one launch per colour class of vertex columns, one for the slack class
        assert g.nclasses >= 2
        assert cols["launches"] == epochs * (g.nclasses - 1)
        assert slack["launches"] == epochs
        assert cols["alg_bytes"] == epochs * (per_col * n + per_entry * entries)
        assert slack["alg_bytes"] == epochs * per_slack * m
        assert t["k_sweep_block"]["launches"] == 0
        assert ref["launches"] >= 1
        for k in (cols, slack, ref):
            assert k["ms"] > 0.0
    finally:
        g.close()
