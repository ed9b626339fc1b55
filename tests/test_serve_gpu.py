"""Serving: continuous batching with admission by device-memory budget.
Every served result must be exactly what the same solve gives alone."""
import sys
import time

import numpy as np
import pytest

from paper_1311_2661_amd import instances as I

pytestmark = pytest.mark.gpu
T = S = None


def setup_module(module):
    global T, S
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1311_2661_amd import serve as SS
    from paper_1311_2661_amd import thetis as TT
    T, S = TT, SS
    torch.cuda.set_device(0)


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def mix():
    return [("vc", I.vc_er(400, 2000, seed=1)), ("mis", I.mis_regular(900, 6, seed=2)),
            ("mc", I.mc_grid(side=10, k=4, seed=3)), ("vc", I.vc_ba(6000, seed=4)),
            ("mis", I.mis_regular(300, 3, seed=5)), ("mc", I.mc_grid(side=6, k=8, seed=6)),
            ("vc", I.vc_er(80, 300, seed=7)), ("mis", I.mis_regular(2500, 11, seed=8))]


def test_served_results_equal_solve_alone():
    say("case serve mix vs alone")
    reqs = mix()
    srv = S.Server(hbm_budget=8 << 30, epoch_cap=100, slots=16)
    futs = []
    for k, (kind, lp) in enumerate(reqs):
        futs.append(srv.submit(lp, kind, seed=k))
        time.sleep(0.002 * (k % 3))          # staggered arrivals: later ones join running batches
    res = [f.result(timeout=120) for f in futs]
    srv.close()
    for k, ((kind, lp), r) in enumerate(zip(reqs, res)):
        a = S.solve_alone(lp, kind, seed=k, epoch_cap=100)
        say(f"  {kind}: epochs {r.epochs}/{a['epochs']} gap {r.gap:.2e} feasible {r.feasible}")
        assert r.epochs == a["epochs"]
        assert r.F == a["F"]
        assert np.array_equal(r.sol, a["sol"])
        assert r.cost == a["cost"]
        assert r.feasible and a["feasible"]
        assert r.latency > 0


def test_budget_forces_waits_but_serves_everything():
    say("case serve tight budget")
    reqs = mix()
    p = T.thetis_params_default()
    p.refresh_every = 5
    insts = [T.Instance(lp) for _, lp in reqs]       # keep the handles alive while sizing
    sizes = [T.thetis_solver_workspace_bytes(h.h, p) for h in insts]
    del insts
    budget = int(max(sizes) * 1.2)           # roughly one request at a time
    srv = S.Server(hbm_budget=budget, epoch_cap=50, slots=16)
    futs = [srv.submit(lp, kind, seed=k) for k, (kind, lp) in enumerate(reqs)]
    res = [f.result(timeout=120) for f in futs]
    srv.close()
    assert all(r.feasible for r in res)
    assert srv.peak_used <= budget
    assert srv.used == 0
    # some request had to wait for memory
    assert max(r.t_admitted - r.t_arrival for r in res) > 0


def test_oversize_request_fails_loudly():
    srv = S.Server(hbm_budget=1 << 20, epoch_cap=10, slots=4)
    f = srv.submit(I.vc_ba(50000, seed=1), "vc")
    with pytest.raises(T.ThetisError):
        f.result(timeout=60)
    ok = srv.submit(I.vc_er(30, 60, seed=2), "vc")
    assert ok.result(timeout=60).feasible
    srv.close()


def test_failed_batch_call_fails_its_requests_and_serving_continues():
    """A batch call that raises (forced from the host: the Python call is
    replaced once) ends the requests it held with that error; the server
    keeps serving."""
    srv = S.Server(hbm_budget=8 << 30, epoch_cap=20, slots=4)
    b = srv.groups["ones"]["batch"]
    real = b.run
    state = {"armed": True}

    def run_once_failing(*args, **kw):
        if state["armed"]:
            state["armed"] = False
            raise T.ThetisError(T.EDEVICE, "batch call failed (forced from the host)")
        return real(*args, **kw)

    b.run = run_once_failing
    f = srv.submit(I.vc_er(200, 600, seed=1), "vc", seed=1)
    with pytest.raises(T.ThetisError) as e:
        f.result(timeout=60)
    assert e.value.code == T.EDEVICE
    ok = srv.submit(I.vc_er(150, 400, seed=2), "vc", seed=2)
    assert ok.result(timeout=60).feasible
    srv.close()


def test_deadlines_and_the_per_solve_log(tmp_path):
    """A request past its deadline on the device is finished from its current
    point (reason "deadline", rounded and checked); one whose deadline passes
    while it waits for memory fails with DeadlineExceeded; every finished or
    failed request leaves one JSON line in the log."""
    import json
    say("case serve deadlines + JSONL log")
    log = tmp_path / "serve.jsonl"
    big = I.mc_grid(side=40, k=8, seed=9)       # far from the gap at the cap
    p = T.thetis_params_default()
    h = T.Instance(big)
    need = T.thetis_solver_workspace_bytes(h.h, p)
    h.close()
    # room for one such request: the second waits for memory
    srv = S.Server(hbm_budget=int(need * 1.5), epoch_cap=100000, slots=4, log_path=str(log))
    f1 = srv.submit(big, "mc", seed=1, deadline_s=0.5)
    time.sleep(0.05)
    f2 = srv.submit(I.mc_grid(side=40, k=8, seed=10), "mc", seed=2, deadline_s=0.2)
    f3 = srv.submit(I.vc_er(300, 1200, seed=3), "vc", seed=3)     # no deadline: reaches the gap
    r1 = f1.result(timeout=120)
    with pytest.raises(S.DeadlineExceeded):
        f2.result(timeout=120)
    r3 = f3.result(timeout=120)
    srv.close()
    assert r1.reason == "deadline" and not r1.reached_gap and r1.feasible
    assert 0 < r1.epochs < 100000
    assert r1.latency >= 0.5
    assert r3.reason == "gap" and r3.reached_gap
    lines = [json.loads(x) for x in log.read_text().splitlines()]
    assert sorted(x["id"] for x in lines) == [0, 1, 2]
    by = {x["id"]: x for x in lines}
    assert by[0]["reason"] == "deadline" and by[0]["epochs"] == r1.epochs and by[0]["feasible"]
    assert by[1]["reason"] == "error" and "DeadlineExceeded" in by[1]["error"]
    assert by[2]["reason"] == "gap" and by[2]["gap"] <= 1e-4
