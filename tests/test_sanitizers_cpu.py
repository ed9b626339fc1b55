"""Host code under the address and undefined-behaviour sanitizers: the
oracle (every entry point: schedules, prox, multiplier steps, all rounding
rules and checks) and the library's host layout code (instance creation,
blocks, pairwise factors, colouring and plans, rounding shapes, rejected
inputs), each built with gcc/g++ and driven over instances of every
workload kind.  Any sanitizer report aborts the driver."""
import os
import shutil
import subprocess

import numpy as np
import pytest

from paper_1311_2661_amd import instances as I

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HOST = os.path.join(ROOT, "tests", "host")
SAN = ["-g", "-O1", "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]


def write_inst(path, inst, x):
    nb = 0 if inst.block_first_col is None else len(inst.block_first_col)
    npw = 0 if inst.pair_ends is None else len(inst.pair_first)
    val = np.ones(inst.nnz) if inst.val is None else inst.val
    fixed = np.full(nb, -1, np.int32) if inst.fixed_label is None else inst.fixed_label
    with open(path, "wb") as f:
        np.array([inst.m, inst.n, inst.nnz, nb, inst.block_k, npw], np.int64).tofile(f)
        np.asarray(inst.row_ptr, np.int64).tofile(f)
        np.asarray(inst.col_idx, np.int32).tofile(f)
        np.asarray(val, np.float64).tofile(f)
        np.asarray(inst.b, np.float64).tofile(f)
        np.asarray(inst.c, np.float64).tofile(f)
        np.asarray(inst.u, np.float64).tofile(f)
        np.asarray(inst.sense, np.int8).tofile(f)
        if nb:
            np.asarray(inst.block_first_col, np.int64).tofile(f)
            np.asarray(fixed, np.int32).tofile(f)
        if npw:
            np.asarray(inst.pair_ends, np.int32).reshape(-1).tofile(f)
            np.asarray(inst.pair_first, np.int64).tofile(f)
        np.asarray(x, np.float64).tofile(f)


@pytest.fixture(scope="module")
def inst_files(tmp_path_factory):
    d = tmp_path_factory.mktemp("san")
    rng = np.random.default_rng(0)
    insts = [I.vc_er(60, 200, seed=1), I.mis_regular(40, 3, seed=1), I.set_cover(80, 40, seed=1, mean_size=4.0),
             I.multicover(60, 30, seed=1), I.kcs_packing(50, 40, 3, seed=1), I.mc_grid(side=5, k=3, seed=1),
             I.map_chain_window(12, 3, 16, seed=1), I.vc_lp(1, np.zeros((0, 2), np.int64), np.ones(1))]
    paths = []
    for q, inst in enumerate(insts):
        x = rng.uniform(0, 1, inst.n)
        if inst.block_first_col is not None:
            for f in inst.block_first_col:
                x[f:f + inst.block_k] = 1.0 / inst.block_k
        p = str(d / f"inst{q}.bin")
        write_inst(p, inst, x)
        paths.append(p)
    return d, paths


def build_and_run(cmd, exe, paths):
    res = subprocess.run(cmd, capture_output=True, text=True)
    assert res.returncode == 0, res.stderr[-3000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    env.pop("LD_PRELOAD", None)
    res = subprocess.run([exe] + paths, capture_output=True, text=True, env=env, timeout=600)
    assert res.returncode == 0, (res.stdout[-2000:], res.stderr[-4000:])
    return res.stdout


@pytest.mark.skipif(shutil.which("gcc") is None, reason="no gcc")
def test_oracle_under_sanitizers(inst_files):
    d, paths = inst_files
    exe = str(d / "orc_san")
    cmd = ["gcc"] + SAN + ["-ffp-contract=off", "-I", HOST, os.path.join(ROOT, "oracle", "thetis_oracle.c"),
                           os.path.join(HOST, "oracle_driver.c"), "-lm", "-o", exe]
    assert "oracle driver ok" in build_and_run(cmd, exe, paths)


@pytest.mark.skipif(shutil.which("g++") is None, reason="no g++")
def test_host_layout_under_sanitizers(inst_files):
    d, paths = inst_files
    exe = str(d / "lay_san")
    cmd = ["g++", "-std=c++17"] + SAN + ["-I", HOST, os.path.join(ROOT, "paper_1311_2661_amd", "csrc", "layout.cpp"),
                                         os.path.join(HOST, "layout_driver.cpp"), "-pthread", "-o", exe]
    assert "layout driver ok" in build_and_run(cmd, exe, paths)
