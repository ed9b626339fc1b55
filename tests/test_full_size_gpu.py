"""The batched and served workloads at their full sizes, in the launch
configuration bench.py times, run as bench.py itself runs them (a child
process), checked on sampled outputs:

  * 4,096 independent-set LPs (n ~ U[200, 50000], random d-regular graphs,
    d ~ U{3..16}), FP32, window of 256 (the benchmark default), stop at the
    1e-4 certified gap or 200 epochs: every sampled instance at the gap,
    every sampled rounding an independent set, every sampled batched solve
    bit-identical to the same solve alone, and the FP64 oracle run for the
    same epochs on a stratified sample agrees (F, c^T x within 1e-4 relative, violation within 1e-4).
  * Poisson arrivals at 200/s of mixed requests (1e3..1e6 edges) for one
    second: nothing fails, every result is feasible, every sampled served
    result equals the same request solved alone, and the FP64 oracle run for
    the served epochs on a stratified sample agrees (F, c^T x within 1e-4
    relative).
"""
import json
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def setup_module(module):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def run_bench(*args, timeout):
    print("case bench.py " + " ".join(args), flush=True)
    res = subprocess.run([sys.executable, "-u", os.path.join(ROOT, "bench.py"), *args], cwd=ROOT,
                         capture_output=True, text=True, timeout=timeout)
    assert res.returncode == 0, res.stderr[-3000:]
    line = [ln for ln in res.stdout.splitlines() if ln.startswith("{")][-1]
    return json.loads(line)


@pytest.mark.timeout(900)
def test_mis_batch_4096_full_size():
    d = run_bench("--workload", "mis_batch", "--instances", "4096", "--precision", "fp32",
                  "--baseline-sample", "32", "--cpu-baseline-seconds", "15", timeout=850)
    print(json.dumps({k: d[k] for k in ("value", "epochs", "gap_reached_sampled", "feasible_sampled",
                                        "batched_equals_alone_sampled", "cpu_baseline")}), flush=True)
    assert d["config"]["instances"] == 4096
    n, m = d["gap_reached_sampled"].split("/")
    assert n == m
    n, m = d["feasible_sampled"].split("/")
    assert n == m
    n, m = d["batched_equals_alone_sampled"].split("/")
    assert n == m and int(m) == 32
    n, m = d["cpu_baseline"]["agrees_with_gpu"].split(" ")[0].split("/")
    assert n == m and int(m) >= 2


@pytest.mark.timeout(900)
def test_serving_at_full_rate():
    d = run_bench("--workload", "serve", "--duration", "1", "--baseline-sample", "16", timeout=850)
    print(json.dumps({k: d[k] for k in ("value", "latency_s", "per_kind", "served_equals_alone_sampled")}),
          flush=True)
    assert d["failed"] == 0
    for kind, v in d["per_kind"].items():
        n, m = v["feasible"].split("/")
        assert n == m, kind
    n, m = d["served_equals_alone_sampled"].split("/")
    assert n == m and int(m) == 16
    # the FP64 oracle, run for the served epochs on a size-stratified sample
    n, m = d["cpu_baseline"]["agrees_with_gpu"].split(" ")[0].split("/")
    assert n == m and int(m) >= 2
