#!/usr/bin/env python3
"""Throughput of the SCD hot path on one MI355X.

Workload: the vertex-cover LP of a Barabasi-Albert graph (n = 2,000,000
vertices, 3 edges per new vertex, 5,999,994 edges, weights uniform[1,10],
seeded), slack form with one slack per edge, beta = 10, x/s/r stored in
FP32 with an FP64 residual refresh every 5 epochs, DET colour-class
schedule, 100 epochs.  One step = one whole solve: reset to y = 0, 100
epochs, the FP64 pre-rounding pass, threshold rounding and the feasibility
check.  Inputs are resident in HBM before the timed region.

Prints one JSON line on stdout; progress goes to stderr.
"""
import argparse
import hashlib
import numpy as np
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "coord updates/s + HBM GB/s; batched solves/s and p99 latency at 1e-4 LP gap"
HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_k_sweep_vc_ba2m.json")
KERNEL_SRC = [os.path.join(ROOT, "paper_1311_2661_amd", "csrc", f) for f in ("thetis.hip", "layout.cpp")]


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def kernel_hash() -> str:
    """Hash of the sources that decide the kernel and the layout it walks."""
    h = hashlib.sha256()
    for p in KERNEL_SRC:
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def counter_traffic(workload: str):
    """HBM bytes per launch of the dominant kernel from the committed
    rocprofv3 counter summary, if it was taken on the current kernel source."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_source_sha256_16") != kernel_hash() or t.get("workload") != workload:
        return None
    return t.get("hbm_bytes_per_launch")


def summarize_counters(fetch_csv: str, write_csv: str, workload: str, copy_mib: int, command: str):
    """Writes the traffic summary of the dominant kernel from two rocprofv3
    counter runs of this script (FETCH_SIZE, then WRITE_SIZE, KiB per
    dispatch), each scaled by what the same counter reads for the plain
    device copy of `copy_mib` MiB the runs also perform."""
    import csv
    import statistics

    def per_kernel(path, counter):
        rows = [r for r in csv.DictReader(open(path)) if r["Counter_Name"] == counter]
        sweep = [float(r["Counter_Value"]) for r in rows
                 if "k_sweep<" in r["Kernel_Name"] and "k_sweep_" not in r["Kernel_Name"]]
        copies = sorted(float(r["Counter_Value"]) for r in rows if "copyBuffer" in r["Kernel_Name"]
                        or "elementwise" in r["Kernel_Name"])
        return sweep, copies

    expect_kib = copy_mib * 1024.0
    f_sweep, f_copy = per_kernel(fetch_csv, "FETCH_SIZE")
    w_sweep, w_copy = per_kernel(write_csv, "WRITE_SIZE")
    # the calibration copies are the dispatches that read (write) about copy_mib
    f_cal = [v for v in f_copy if 0.5 * expect_kib < v < 2.0 * expect_kib]
    w_cal = [v for v in w_copy if 0.5 * expect_kib < v < 2.0 * expect_kib]
    kf = expect_kib / statistics.median(f_cal)
    kw = expect_kib / statistics.median(w_cal)
    fetch = statistics.mean(f_sweep) * kf
    write = statistics.mean(w_sweep) * kw
    out = dict(kernel="k_sweep", workload=workload, kernel_source_sha256_16=kernel_hash(),
               fetch_kib_per_launch=statistics.mean(f_sweep), write_kib_per_launch=statistics.mean(w_sweep),
               launches=len(f_sweep), fetch_scale=kf, write_scale=kw,
               hbm_bytes_per_launch=1024.0 * (fetch + write), command=command)
    with open(TRAFFIC_FILE, "w") as fh:
        json.dump(out, fh, indent=1)
    print(json.dumps(out, indent=1))


def access_split(inst, unit_class):
    """Entries of the structural columns per colour class, split into those
    whose row the class owns (the row's first-scheduled column is in it: its
    residual sits in the column's own contiguous run) and the rest (the row
    belongs to an earlier class: a random residual access)."""
    import numpy as np
    rp = inst.row_ptr
    cls = unit_class[: inst.n]
    ent_cls = cls[inst.col_idx]
    lens = np.diff(rp)
    nz = lens > 0
    row_min = np.full(inst.m, np.iinfo(np.int32).max, np.int64)
    row_min[nz] = np.minimum.reduceat(ent_cls, rp[:-1][nz])
    owned = ent_cls == np.repeat(row_min, lens)
    nc = int(cls.max()) + 1
    return (np.bincount(ent_cls[owned], minlength=nc).astype(np.int64),
            np.bincount(ent_cls[~owned], minlength=nc).astype(np.int64),
            np.bincount(cls, minlength=nc).astype(np.int64))


def random_access_model(T, words: int, owned, foreign, ncols, sweep_ms_per_epoch: float):
    """Prices one epoch of plain-column sweeps with rates timed live on this
    GPU.  Sequential bytes (row index 4 B per entry, residual read + write
    8 B per owned entry, 20 B per column) go at the copy rate in both
    models.  Foreign entries (rows an earlier class owns) cost one random
    4-byte read-modify-write each: in `model_us_per_epoch` at the rate of a
    buffer the size of the residual touched anywhere (the row order without
    XCD windows), in `window_model_us_per_epoch` at the rate of random
    read-modify-writes that stay inside each XCD's eighth of a buffer whose
    eighths are the size of a class's per-XCD window (the row layout's
    windows)."""
    import math
    k = max(13, min(28, int(round(math.log2(max(words, 8192))))))
    g_ms, rmw_ms, cp_ms, _ = T.thetis_calibrate_random(k, 10)
    w = float(1 << k)
    rmw_rate, gather_rate, copy_gbs = w / (rmw_ms * 1e-3), w / (g_ms * 1e-3), 8 * w / (cp_ms * 1e-3) / 1e9
    F, O, N = float(sum(foreign)), float(sum(owned)), float(sum(ncols))
    # a class's foreign rows split over the 8 XCD windows: the buffer's eighths
    per_class = max(foreign) if len(foreign) else 0
    kw = max(13, min(28, int(round(math.log2(max(per_class, 8192))))))
    xcd_ms = T.thetis_calibrate_random(kw, 10)[3]
    xcd_rate = float(1 << kw) / (xcd_ms * 1e-3)
    seq_bytes = 4 * (F + O) + 8 * O + 20 * N
    seq_us = 1e6 * seq_bytes / (copy_gbs * 1e9)
    model_us = 1e6 * (F / rmw_rate) + seq_us
    wmodel_us = 1e6 * (F / xcd_rate) + seq_us
    meas_us = 1e3 * sweep_ms_per_epoch
    return {"buffer_words": int(w), "random_rmw_per_s": rmw_rate, "random_gather_per_s": gather_rate,
            "copy_gbs": copy_gbs, "owned_entries_per_epoch": int(O), "foreign_entries_per_epoch": int(F),
            "model_us_per_epoch": model_us, "window_buffer_words": 1 << kw, "xcd_window_rmw_per_s": xcd_rate,
            "window_model_us_per_epoch": wmodel_us, "measured_us_per_epoch": meas_us,
            "frac_of_model": model_us / meas_us if meas_us > 0 else None,
            "frac_of_window_model": wmodel_us / meas_us if meas_us > 0 else None}


def cpu_baseline(inst, epochs_cap: int, budget_s: float, seed: int):
    """The FP64 oracle (serial C, one thread) in the same DET order on the
    same instance; a bounded number of epochs, timed without its setup."""
    from oracle import oracle as O
    lp = O.OracleLP(inst)
    o = O.OracleSolver(lp, beta=10.0, schedule=O.SCHED_DET, seed=seed)
    upd = inst.n + int((inst.sense != 0).sum())
    t0 = time.perf_counter()
    o.run(1)
    t1 = time.perf_counter() - t0
    more = int(max(0, min(epochs_cap - 1, budget_s / max(t1, 1e-9) - 1)))
    t0 = time.perf_counter()
    if more:
        o.run(more)
    t2 = time.perf_counter() - t0
    ep = 1 + more
    total = t1 + t2
    return dict(value=ep * upd / total, unit="coord updates/s", cores=1, kind="oracle",
                sample=f"{ep} of the 100 epochs of the same instance, DET class order, serial FP64 C, "
                       f"{total:.1f} s, setup excluded")


def _mis_spec(k, seed):
    from paper_1311_2661_amd import instances as I
    rng = I.rng_for(seed, 1000 + k)
    n = int(rng.integers(200, 50001))
    d = int(rng.integers(3, 17))
    return n, d


def _mis_make(args):
    k, seed = args
    from paper_1311_2661_amd import instances as I
    n, d = _mis_spec(k, seed)
    inst = I.mis_regular(n, d, seed=seed * 100003 + k)
    return inst.n, inst.meta["edges"].astype(np.int32), -inst.c


def mis_batch(args):
    """Batched workload: independent-set LPs on random d-regular graphs,
    n uniform in [200, 50000], d uniform in {3..16}, weights uniform[1,5];
    all instances solved in one batch to a 1e-4 certified gap (cap 200
    epochs).  Baseline: the same solver run one instance per launch
    sequence, timed on a stratified sample and extrapolated."""
    import multiprocessing as mp
    from paper_1311_2661_amd import instances as I
    t0 = time.perf_counter()
    count = args.instances
    workers = max(1, min(16, (os.cpu_count() or 1)))
    with mp.get_context("fork").Pool(workers) as pool:      # before the GPU is touched
        made = pool.map(_mis_make, [(k, args.seed) for k in range(count)], chunksize=8)
    nv = np.array([m[0] for m in made])
    ne = np.array([len(m[1]) for m in made])
    log(f"{count} instances: {nv.sum()} vertices, {ne.sum()} edges, generated in {time.perf_counter() - t0:.1f} s "
        f"({workers} workers)")
    import torch
    from paper_1311_2661_amd import thetis as T
    T.lib()
    torch.cuda.set_device(0)
    prec = {"bf16": T.PREC_BF16X, "fp32": T.PREC_FP32}[args.precision]

    def solver_of(k):
        n, e, w = made[k]
        inst = I.mis_lp(n, e.astype(np.int64), w)
        h = T.Instance(inst)
        s = T.Solver(h, beta=10.0, precision=prec, refresh_every=5, seed=k)
        s.instance = None
        h.close()
        return s

    t0 = time.perf_counter()
    solvers = [solver_of(k) for k in range(count)]
    torch.cuda.synchronize()
    log(f"layout + upload of {count} solvers: {time.perf_counter() - t0:.1f} s")
    b = T.Batch(solvers)
    if args.window:
        b.set_window(args.window)
    choice = b.autotune(epochs_per_candidate=2)
    log(f"autotuned: widen {choice[0]}, grid x{choice[1]}, strided {choice[2]}, columns per group {choice[3]}")
    upd_total = []
    for w in range(args.warmup):
        for s in solvers:
            s.reset()
        b.run(args.cap, gap_tol=args.gap)
    for s in solvers:
        s.reset()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    done = b.run(args.cap, gap_tol=args.gap)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    reached = 0
    for s in solvers[:: max(1, count // 64)]:
        m = s.metrics()
        reached += m["gap"] <= args.gap
    sample_n = len(solvers[:: max(1, count // 64)])
    log(f"batch: {count} solves in {elapsed:.3f} s; epochs median {int(np.median(done))} max {int(done.max())}; "
        f"gap reached in {reached}/{sample_n} sampled")
    # per-instance updates: n + m coordinates per epoch
    upd = float(np.sum((nv + ne) * done))
    # one instance per launch sequence: stratified sample by size
    order = np.argsort(nv)
    strata = np.array_split(order, args.baseline_sample)
    pick = [int(st[len(st) // 2]) for st in strata if len(st)]
    times, same = [], 0
    for k in pick:
        s = solver_of(k)
        torch.cuda.synchronize()
        ta = time.perf_counter()
        e_alone = s.run(args.cap, gap_tol=args.gap)
        s.round(T.ROUND_MIS_THRESH)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - ta)
        # the batched solve must be the solve alone, bit for bit
        sb = solvers[k]
        ma, mb = s.metrics(), sb.metrics()
        same += int(e_alone == int(done[k]) and np.array_equal(s.y, sb.y) and ma["F"] == mb["F"])
        s.close()
    log(f"batched == alone on {same}/{len(pick)} sampled instances")
    per_solve = float(np.mean(times))
    base = 1.0 / per_solve
    value = count / elapsed
    # validity of the batched answers on a sample
    feas = 0
    for s in solvers[:: max(1, count // 32)]:
        s.round(T.ROUND_MIS_THRESH)
        feas += s.check(T.ROUND_MIS_THRESH)[0]
    out = {
        "metric": METRIC, "value": value, "unit": "solves/s", "n_gpus": 1, "steps": 1,
        "warmup": args.warmup, "ms_per_step": 1e3 * elapsed, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": args.precision, "data": "synthetic",
        "config": {"workload": f"mis_batch_{count}_n200-50000_d3-16_{args.precision}_gap{args.gap:g}_cap{args.cap}",
                   "instances": count, "vertices": int(nv.sum()), "edges": int(ne.sum()),
                   "gap_tol": args.gap, "epoch_cap": args.cap, "autotune": list(choice),
                   "window": args.window, "seed": args.seed},
        "coord_updates_per_s": upd / elapsed,
        "epochs": {"median": float(np.median(done)), "max": int(done.max()), "min": int(done.min())},
        "gap_reached_sampled": f"{reached}/{sample_n}",
        "feasible_sampled": f"{feas}/{len(solvers[:: max(1, count // 32)])}",
        "one_per_launch": {"solves_per_s": base, "sample": f"{len(pick)} instances stratified by size, solved alone, "
                           f"mean {1e3 * per_solve:.2f} ms per solve (extrapolated to the population)"},
        "speedup_vs_one_per_launch": value / base,
        "batched_equals_alone_sampled": f"{same}/{len(pick)}",
    }
    if args.cpu_baseline_seconds > 0:
        log("cpu baseline (oracle) ...")
        out["cpu_baseline"] = mis_cpu_baseline(made, pick, done, solvers, args)
        log(f"cpu baseline: {out['cpu_baseline']}")
    print(json.dumps(out), flush=True)


def mis_cpu_baseline(made, pick, done, solvers, args):
    """The FP64 oracle (serial C, one thread) solves the stratified sample
    (in stratum order until the time budget is spent), each for as many
    epochs as its batched solve ran; solves/s = 1 / the mean time over the
    strata solved.  Each oracle solve is also compared with the batched FP32
    solve at that epoch: F and c^T x within 1e-4 relative, the row violation
    within 1e-4."""
    from oracle import oracle as O
    from paper_1311_2661_amd import instances as I
    times, agree, n_done = [], 0, 0
    order = list(range(len(pick)))
    # interleave small and large strata so a short budget still spans sizes
    order = [order[i // 2] if i % 2 == 0 else order[-(i // 2) - 1] for i in range(len(order))]
    seen = set()
    spent = 0.0
    for q in order:
        if q in seen:
            continue
        seen.add(q)
        if spent > args.cpu_baseline_seconds and n_done >= 2:
            break
        k = pick[q]
        n, e, w = made[k]
        inst = I.mis_lp(n, e.astype(np.int64), w)
        lp = O.OracleLP(inst)
        o = O.OracleSolver(lp, beta=10.0, schedule=O.SCHED_DET, seed=k)
        ta = time.perf_counter()
        o.run(int(done[k]))
        dt = time.perf_counter() - ta
        spent += dt
        times.append(dt)
        om, gm = o.metrics(), solvers[k].metrics()
        rel = lambda a, b: abs(a - b) / max(1.0, abs(b))
        agree += int(rel(gm["F"], om["F"]) <= 1e-4 and rel(gm["lp_value"], om["lp_value"]) <= 1e-4
                     and abs(gm["max_viol"] - om["max_viol"]) <= 1e-4)
        n_done += 1
    return dict(value=1.0 / float(np.mean(times)), unit="solves/s", cores=1, kind="oracle",
                sample=f"{n_done} of the {len(pick)} size strata, each solved by the serial FP64 oracle for "
                       f"the epochs its batched solve ran ({spent:.1f} s, setup excluded); population mean "
                       f"estimated from the strata",
                agrees_with_gpu=f"{agree}/{n_done} (F and c^T x within 1e-4 relative, violation within 1e-4)")


def mc_grid(args):
    """Multiway cut on the 1024 x 1024 4-connected grid, k = 8 terminals at
    seeded random pixels, edge weights exp(-d^2), d ~ N(0,1); x blocks on the
    simplex (block coordinate steps), z and slacks as plain coordinates;
    FP32, 200 epochs, region-growing rounding (10 repetitions, fixed seed)."""
    import torch
    from paper_1311_2661_amd import instances as I
    from paper_1311_2661_amd import thetis as T
    T.lib()
    torch.cuda.set_device(0)
    t0 = time.perf_counter()
    side = args.side
    inst = I.mc_grid(side=side, k=8, seed=args.seed)
    log(f"grid {side}x{side}: {inst.n} columns, {inst.m} rows, {inst.nnz} entries ({time.perf_counter() - t0:.1f} s)")
    t0 = time.perf_counter()
    h = T.Instance(inst)
    s = T.Solver(h, beta=10.0, precision=T.PREC_FP32, refresh_every=5, seed=args.seed)
    log(f"layout + upload: {time.perf_counter() - t0:.1f} s, {h.classes()[0]} colour classes")
    tuned = s.autotune(4)                  # real epochs; every step resets
    log(f"columns per lane group by class: {tuned}")
    tr = s.traffic()
    ep = args.epochs

    def step():
        s.reset()
        s.run(ep)
        sol, cost, aux = s.round(T.ROUND_MC_CKR, seed=args.seed, reps=10)
        return sol, cost, s.check(T.ROUND_MC_CKR)

    for _ in range(args.warmup):
        step()
    s.set_timing(10)
    acc = {k: dict(ms=0.0, launches=0, alg_bytes=0.0) for k in T.KERNEL_NAMES.values()}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        sol, cost, chk = step()
        for name, v in s.timing().items():
            for f in ("ms", "launches", "alg_bytes"):
                acc[name][f] += v[f]
        log(f"step {k} done")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    s.set_timing(0)
    m = s.metrics()
    # properties at full size: blocks on the simplex, terminals fixed, the
    # labelling valid, and its cut weight recomputed from the edge list
    x = s.x
    nv = side * side
    X = x[: nv * 8].reshape(nv, 8)
    e = inst.meta["edges"]
    cut = float(inst.meta["edge_w"][sol[e[:, 0]] != sol[e[:, 1]]].sum())
    props = dict(simplex_err=float(np.abs(X.sum(axis=1) - 1).max()), min_x=float(X.min()),
                 terminals_ok=bool(np.array_equal(np.argmax(X[inst.meta["terminals"]], axis=1), np.arange(8))),
                 labels_feasible=bool(chk[0]), cut_recomputed=cut, cut_reported=cost,
                 dual_below_F=bool(m["dual_bound"] <= m["F"]))
    log(f"properties: {props}")
    g = acc["k_sweep_block"]
    avg_ms = g["ms"] / max(g["launches"], 1)
    avg_bytes = g["alg_bytes"] / max(g["launches"], 1)
    achieved = avg_bytes / (avg_ms * 1e-3) / 1e9 if avg_ms > 0 else 0.0
    upd = tr["updates_per_epoch"]
    out = {
        "metric": METRIC, "value": args.steps * ep * upd / elapsed, "unit": "coord updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"mc_grid_{side}x{side}_k8_beta10_fp32_refresh5_{ep}ep_det", "columns": inst.n,
                   "rows": inst.m, "entries": inst.nnz, "coordinates_per_epoch": upd,
                   "group_cols_by_class": tuned, "seed": args.seed},
        "roofline": {"bound": "hbm", "kernel": "k_sweep_block", "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "alg_bytes_per_launch": avg_bytes, "avg_launch_us": 1e3 * avg_ms},
        "kernels": {name: dict(ms_total=round(v["ms"], 4), launches=v["launches"],
                               avg_us=round(1e3 * v["ms"] / max(v["launches"], 1), 3),
                               alg_gbs=round(v["alg_bytes"] / max(v["ms"], 1e-9) / 1e6, 1))
                    for name, v in acc.items() if v["launches"]},
        "solution": {"F": m["F"], "lp_value": m["lp_value"], "gap": m["gap"], "cut": cost, **props},
    }
    if args.cpu_baseline_seconds > 0:
        from oracle import oracle as O
        lp = O.OracleLP(inst)
        o = O.OracleSolver(lp, beta=10.0, seed=args.seed)
        t0 = time.perf_counter()
        o.run(1)
        t1 = time.perf_counter() - t0
        more = int(max(0, min(ep - 1, args.cpu_baseline_seconds / max(t1, 1e-9) - 1)))
        t0 = time.perf_counter()
        if more:
            o.run(more)
        tt = t1 + time.perf_counter() - t0
        out["cpu_baseline"] = dict(value=(1 + more) * upd / tt, unit="coord updates/s", cores=1, kind="oracle",
                                   sample=f"{1 + more} of the {ep} epochs of the same instance, DET class order, "
                                          f"serial FP64 C, {tt:.1f} s, setup excluded")
    print(json.dumps(out), flush=True)


# augmented-Lagrangian workloads: rounding rules with their repetitions, and
# the workload name's prefix
# beta and epochs between multiplier steps are the fastest to the tolerances
# among beta in {3, 10} (also 1 and 30 for packing, 1 for the MAP LP) and
# 10, 20, 30 or 50 epochs, measured on these instances
AL_WORKLOADS = {
    "al_ba": dict(rules=[(1, 1)], name="vc_ba_n{n}_m3", gap=1e-4, feas=5e-2, beta=3.0, inner=10),
    "setcover": dict(rules=[(5, 1), (6, 10)], name="set_cover_4000000x1000000_mean8", gap=1e-4, feas=5e-2,
                     beta=10.0, inner=10),
    # the packing LP's gap closes slowly under the outer loop: its stop is a
    # 1e-3 gap
    "packing": dict(rules=[(7, 10)], name="kcs_packing_2000000x1000000_k4", gap=1e-3, feas=5e-2, beta=3.0,
                    inner=10),
    # the text-chunking shape of the MAP experiments (47,000 variables of
    # domain 23, 100,000 factors)
    "map": dict(rules=[(8, 1), (9, 10)], name="map_chain_window_47000x23_100000factors", gap=3e-4, feas=1e-2,
                beta=3.0, inner=10),
}


def _al_instance(args):
    from paper_1311_2661_amd import instances as I
    if args.workload == "al_ba":
        return I.vc_ba(args.n, seed=args.seed)
    if args.workload == "setcover":
        return I.set_cover(4_000_000, 1_000_000, seed=args.seed)
    if args.workload == "map":
        return I.map_chain_window(47_000, 23, 100_000, seed=args.seed)
    return I.kcs_packing(2_000_000, 1_000_000, 4, seed=args.seed)


def al_workload(args):
    """Augmented-Lagrangian outer loop on one LP, then its roundings.
    al_ba: vertex cover on the BA graph (n = 2,000,000); setcover: weighted
    set cover, 4,000,000 elements, 1,000,000 sets of mean size 8; packing:
    k-column-sparse packing, 2,000,000 sets of 4 elements over 1,000,000
    elements, integer weights and capacities; map: the local-polytope LP of
    a pairwise factor graph shaped like text chunking (47,000 variables of
    domain 23, a chain plus agreement factors, 100,000 factors).  FP32
    storage, the workload's beta, refresh every 5 epochs, DET: from
    ubar = 0, blocks of `inner` epochs alternate
    with multiplier steps until ||A y - b||_inf <= feas_tol and the LP gap
    certified by the dual function <= lp_gap_tol (at most `outer` steps);
    then the workload's roundings and the check.  Every step re-solves from
    the start."""
    import torch
    from paper_1311_2661_amd import thetis as T
    T.lib()
    torch.cuda.set_device(0)
    wl = AL_WORKLOADS[args.workload]
    rules, wname, beta = wl["rules"], wl["name"], wl["beta"]
    if args.lp_gap_tol is None:
        args.lp_gap_tol = wl["gap"]
    if args.feas_tol is None:
        args.feas_tol = wl["feas"]
    if args.inner is None:
        args.inner = wl["inner"]
    t0 = time.perf_counter()
    inst = _al_instance(args)
    log(f"instance: {inst.m} rows, {inst.n} columns, {inst.nnz} entries ({time.perf_counter() - t0:.1f} s)")
    h = T.Instance(inst)
    s = T.Solver(h, beta=beta, ubar=np.zeros(inst.m), precision=T.PREC_FP32, refresh_every=5, seed=args.seed)
    tuned = s.autotune(4)
    log(f"columns per lane group by class: {tuned}")
    upd = s.traffic()["updates_per_epoch"]
    maximise = args.workload == "packing"

    def step():
        s.reset()
        outer, epochs, st = s.run_multipliers(args.outer, args.inner, feas_tol=args.feas_tol,
                                              lp_gap_tol=args.lp_gap_tol)
        rounded = []
        for rule, reps in rules:
            sol, cost, aux = s.round(rule, seed=args.seed, reps=reps)
            feas, nviol = s.check(rule)
            rounded.append((rule, reps, cost, aux, feas, sol))
        return outer, epochs, st, rounded

    for w in range(args.warmup):
        r = step()
        log(f"warmup {w}: outer {r[0]} epochs {r[1]} linf {r[2]['linf']:.3e} gap {r[2]['lp_gap']:.3e}")
    s.set_timing(10)
    acc = {k: dict(ms=0.0, launches=0, alg_bytes=0.0) for k in T.KERNEL_NAMES.values()}
    mul_ms, mul_bytes, results = [], [], []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        r = step()
        results.append(r)
        mul_ms.append(r[2]["device_ms"])
        mul_bytes.append(r[2]["alg_bytes"])
        for name, v in s.timing().items():
            for f in ("ms", "launches", "alg_bytes"):
                acc[name][f] += v[f]
        log(f"step {k} done: outer {r[0]} epochs {r[1]}")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    s.set_timing(0)
    assert all(all(x[4] for x in r[3]) for r in results), "a rounded solution is infeasible"
    # a property at any size: the reported cost recomputed on the host from
    # the instance and the returned solution
    for rule, reps, cost, aux, feas, sol in results[-1][3]:
        if rule in (8, 9):
            k = inst.block_k
            e = inst.pair_ends
            host = float(inst.c[inst.block_first_col + sol].sum() +
                         inst.c[inst.pair_first + sol[e[:, 0]].astype(np.int64) * k + sol[e[:, 1]]].sum())
        else:
            host = float(inst.c @ sol)
        assert abs(host - cost) <= 1e-9 * max(1.0, abs(cost)), (rule, host, cost)
    outer, epochs, st, rounded = results[-1]
    # time of the roundings alone (outside the timed steps, same state)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for rule, reps in rules:
        s.round(rule, seed=args.seed, reps=reps)
    torch.cuda.synchronize()
    round_ms = 1e3 * (time.perf_counter() - t1)
    g = acc["k_sweep"]
    avg_ms = g["ms"] / max(g["launches"], 1)
    avg_bytes = g["alg_bytes"] / max(g["launches"], 1)
    achieved = avg_bytes / (avg_ms * 1e-3) / 1e9 if avg_ms > 0 else 0.0
    mms = float(np.mean(mul_ms))
    mgbs = float(np.mean(mul_bytes)) / (mms * 1e-3) / 1e9
    names = {1: "vc_threshold", 5: "set_cover_threshold", 6: "cover_randomized", 7: "packing_alteration",
             8: "map_argmax", 9: "map_sampling"}
    lp_bound = st["lp_dual"]
    sol_out = {"outer_steps": outer, "epochs": epochs, "lp_value": st["lp_value"], "lp_dual": lp_bound,
               "lp_gap": st["lp_gap"], "linf": st["linf"]}
    for rule, reps, cost, aux, feas, _ in rounded:
        key = names[rule]
        if maximise:
            sol_out[key] = {"profit": -cost, "reps": reps, "alpha": aux[0], "feasible": bool(feas),
                            "ratio_to_lp_upper_bound": (-cost) / (-lp_bound)}
        else:
            sol_out[key] = {"cost": cost, "reps": reps, "aux": aux[0], "feasible": bool(feas),
                            "rel_gap_to_lp_bound": (cost - lp_bound) / abs(lp_bound),
                            "host_recomputed": True}
    workload = (f"{wname.format(n=args.n)}_augmented_lagrangian_beta{beta:g}_fp32_refresh5_{args.inner}ep_per_step_"
                f"to_linf{args.feas_tol:g}_gap{args.lp_gap_tol:g}_det")
    out = {
        "metric": METRIC, "value": sum(r[1] for r in results) * upd / elapsed, "unit": "coord updates/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": workload, "rows": inst.m, "columns": inst.n, "entries": inst.nnz,
                   "coordinates_per_epoch": upd, "beta": beta, "epochs_per_outer_step": args.inner,
                   "max_outer_steps": args.outer, "feas_tol": args.feas_tol, "lp_gap_tol": args.lp_gap_tol,
                   "roundings": [[names[r], reps] for r, reps in rules], "group_cols_by_class": tuned,
                   "seed": args.seed},
        "roofline": {"bound": "hbm", "kernel": "k_sweep", "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "alg_bytes_per_launch": avg_bytes, "avg_launch_us": 1e3 * avg_ms},
        "multiplier_step": {"device_ms": mms, "alg_bytes": float(np.mean(mul_bytes)), "alg_gbs": mgbs,
                            "frac_of_hbm_peak": mgbs / HBM_PEAK_GBS,
                            "kernels": "k_mul_rows + k_mul_cols + k_mul_final"},
        "roundings_ms": round_ms,
        "solution": sol_out,
    }
    log(f"solve: {outer} outer steps, {epochs} epochs, c^T x {st['lp_value']:.10g} D {lp_bound:.10g} "
        f"linf {st['linf']:.3e}; roundings {json.dumps({k: v for k, v in sol_out.items() if isinstance(v, dict)})}")
    if args.cpu_baseline_seconds > 0:
        from oracle import oracle as O
        lp = O.OracleLP(inst)
        o = O.OracleSolver(lp, beta=beta, ubar=np.zeros(inst.m), seed=args.seed)
        t0 = time.perf_counter()
        o.run(1)
        t_ep = time.perf_counter() - t0
        more = int(max(0, min(args.inner - 1, args.cpu_baseline_seconds / max(t_ep, 1e-9) - 2)))
        t0 = time.perf_counter()
        if more:
            o.run(more)
        t_more = time.perf_counter() - t0
        t0 = time.perf_counter()
        o.multiplier_step()
        t_mul = time.perf_counter() - t0
        ne = 1 + more
        # one multiplier step per `inner` epochs, as in the GPU solve
        tt = t_ep + t_more + t_mul * ne / args.inner
        out["cpu_baseline"] = dict(value=ne * upd / tt, unit="coord updates/s", cores=1, kind="oracle",
                                   sample=f"{ne} epochs of the same instance from ubar = 0 (DET class order) and "
                                          f"one multiplier step ({t_mul:.2f} s) charged at one per {args.inner} "
                                          f"epochs; serial FP64 C, setup excluded")
    print(json.dumps(out), flush=True)


def _serve_compact(req):
    from paper_1311_2661_amd import instances as I
    return I.serving_compact(req)


def serve(args):
    """Serving workload: Poisson arrivals of mixed vertex-cover /
    independent-set / multiway-cut requests (edges log-uniform in [1e3, 1e6])
    replayed against the continuous-batching server; each request stops at
    the certified gap or the epoch cap.  Latency = arrival to result on the
    host, including expanding the request's LP rows and building its layout.
    Baseline: the same solves one instance at a time (stratified sample)."""
    import multiprocessing as mp
    from paper_1311_2661_amd import instances as I
    n_req = int(args.rate * args.duration)
    trace = I.serving_trace(n_req, args.rate, args.seed)
    t0 = time.perf_counter()
    workers = max(1, min(16, (os.cpu_count() or 1)))
    with mp.get_context("fork").Pool(workers) as pool:      # before the GPU is touched
        compact = pool.map(_serve_compact, trace, chunksize=4)
    edges = np.array([r["edges"] for r in trace])
    kinds = [r["kind"] for r in trace]
    log(f"{n_req} requests over {trace[-1]['t_arrival']:.1f} s; edges median {int(np.median(edges))}, "
        f"kinds vc/mis/mc {kinds.count('vc')}/{kinds.count('mis')}/{kinds.count('mc')}; "
        f"compact forms in {time.perf_counter() - t0:.1f} s")
    import threading
    import torch
    from paper_1311_2661_amd import serve as SV
    from paper_1311_2661_amd import thetis as T
    T.lib()
    torch.cuda.set_device(0)
    free, total = torch.cuda.mem_get_info()
    budget = int(args.budget_gb * (1 << 30)) if args.budget_gb > 0 else int(0.5 * free)
    srv = SV.Server(hbm_budget=budget, gap_tol=args.gap, epoch_cap=args.cap, slots=args.slots,
                    precision=T.PREC_FP32, builders=args.builders, log_path=args.serve_log or None)
    # warm-up: one small request of each kind (kernels load, graphs capture)
    warm = [srv.submit(I.serving_expand(I.serving_compact(dict(kind=k, edges=2000, seed=10**6 + j))), k, seed=j)
            for j, k in enumerate(["vc", "mis", "mc"])]
    for f in warm:
        f.result()
    futs = [None] * n_req
    tstart = time.perf_counter()

    def client():
        for k, r in enumerate(trace):
            dt = tstart + r["t_arrival"] - time.perf_counter()
            if dt > 0:
                time.sleep(dt)
            c = compact[k]
            futs[k] = srv.submit(lambda c=c: I.serving_expand(c), r["kind"], seed=r["seed"] % (1 << 31),
                                 t_arrival=time.perf_counter())
    th = threading.Thread(target=client)
    th.start()
    th.join()
    log(f"all {n_req} submitted after {time.perf_counter() - tstart:.1f} s")
    res, errs = [], 0
    for k, f in enumerate(futs):
        try:
            res.append(f.result())
        except Exception as e:
            errs += 1
            log(f"request {k} failed: {e}")
        if k % max(1, n_req // 10) == 0:
            log(f"collected {k + 1}/{n_req}")
    srv.close()
    tend = max(r.t_done for r in res)
    makespan = tend - tstart
    lat = np.array([r.latency for r in res])
    per_kind = {}
    for kd in ("vc", "mis", "mc"):
        rk = [r for r in res if r.kind == kd]
        if rk:
            per_kind[kd] = dict(n=len(rk), p50_s=float(np.median([r.latency for r in rk])),
                                p99_s=float(np.quantile([r.latency for r in rk], 0.99)),
                                epochs_median=float(np.median([r.epochs for r in rk])),
                                gap_reached=f"{sum(r.reached_gap for r in rk)}/{len(rk)}",
                                gap_median=float(np.median([r.gap for r in rk])),
                                feasible=f"{sum(r.feasible for r in rk)}/{len(rk)}")
    # solves at the gap are the metric; requests stopped by the epoch cap
    # (the grid multiway cuts) are served and reported, not counted
    at_gap = [r for r in res if r.reached_gap]
    capped = [r for r in res if not r.reached_gap]
    value = len(at_gap) / makespan
    lat_gap = np.array([r.latency for r in at_gap]) if at_gap else np.zeros(1)
    # one request at a time, same solves: stratified sample by size
    order = np.argsort(edges)
    pick = [int(st[len(st) // 2]) for st in np.array_split(order, args.baseline_sample) if len(st)]
    times, same, pick_gap = [], 0, 0
    for k in pick:
        lp = I.serving_expand(compact[k])
        torch.cuda.synchronize()
        ta = time.perf_counter()
        ref = SV.solve_alone(lp, trace[k]["kind"], seed=trace[k]["seed"] % (1 << 31), gap_tol=args.gap,
                             epoch_cap=args.cap)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - ta)
        pick_gap += int(ref["gap"] <= args.gap)
        # the served result must be the solve alone
        r = futs[k].result()
        same += int(r.epochs == ref["epochs"] and r.F == ref["F"] and r.cost == ref["cost"]
                    and np.array_equal(r.sol, ref["sol"]))
    log(f"served == alone on {same}/{len(pick)} sampled requests")
    # one at a time, the same requests in sequence: solves at the gap per
    # second of the stratified sample (its capped solves take their time too)
    alone = pick_gap / float(np.sum(times))
    if alone <= 0.0:
        raise RuntimeError("no sampled request reached the gap alone: the one-at-a-time rate is undefined")
    cpu = None
    if args.cpu_baseline_seconds > 0:
        cpu = serve_cpu_baseline(compact, trace, futs, pick, args)
        log(f"cpu baseline: {cpu}")
    out = {
        "metric": METRIC, "value": value, "unit": "solves/s", "n_gpus": 1, "steps": 1, "warmup": 3,
        "ms_per_step": 1e3 * makespan, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"serve_poisson{args.rate:g}_{args.duration:g}s_edges1e3-1e6_gap{args.gap:g}_cap{args.cap}",
                   "requests": n_req, "rate_per_s": args.rate, "budget_bytes": budget, "slots_per_kind": args.slots,
                   "epochs_per_tick": 5, "seed": args.seed},
        "latency_s": {"p50": float(np.median(lat_gap)), "p99": float(np.quantile(lat_gap, 0.99)),
                      "max": float(lat_gap.max()), "of": "solves at the gap"},
        "latency_all_s": {"p50": float(np.median(lat)), "p99": float(np.quantile(lat, 0.99)), "max": float(lat.max())},
        "solves_at_gap": len(at_gap),
        "capped": {"n": len(capped), "kinds": {kd: sum(r.kind == kd for r in capped) for kd in ("vc", "mis", "mc")},
                   "solves_per_s": len(capped) / makespan,
                   "gap_median": float(np.median([r.gap for r in capped])) if capped else None,
                   "note": "stopped by the epoch cap before the gap; served, rounded, checked, not counted in value"},
        "per_kind": per_kind, "failed": errs, "peak_budget_used_bytes": srv.peak_used,
        "one_at_a_time": {"solves_per_s": alone, "sample": f"{len(pick)} requests stratified by size, solved alone "
                          f"in sequence ({pick_gap} reached the gap), mean {1e3 * float(np.mean(times)):.1f} ms"},
        "speedup_vs_one_at_a_time": value / alone,
        "served_equals_alone_sampled": f"{same}/{len(pick)}",
    }
    if cpu is not None:
        out["cpu_baseline"] = cpu
    print(json.dumps(out), flush=True)


def serve_cpu_baseline(compact, trace, futs, pick, args):
    """The FP64 oracle (serial C, one thread) solves the size-stratified
    sample of requests (small and large strata interleaved, until the time
    budget is spent), each for as many epochs as its served solve ran, in the
    same class order.  Its rate in entry updates per second (epochs x
    (matrix entries + columns + rows)) over those solves prices every
    stratum's served work; solves/s = 1 / the mean priced time over all
    strata.  Each oracle solve is compared with the served FP32 solve: F and
    c^T x within 1e-4 relative."""
    from oracle import oracle as O
    from paper_1311_2661_amd import instances as I
    work = []
    for k in pick:
        lp = I.serving_expand(compact[k])
        work.append(float(futs[k].result().epochs) * (len(lp.col_idx) + lp.n + lp.m))
    order = list(range(len(pick)))
    order = [order[i // 2] if i % 2 == 0 else order[-(i // 2) - 1] for i in range(len(order))]
    done_work, agree, seen, spent, n_done = 0.0, 0, set(), 0.0, 0
    for q in order:
        if q in seen:
            continue
        seen.add(q)
        if spent > args.cpu_baseline_seconds and n_done >= 2:
            break
        k = pick[q]
        r = futs[k].result()
        lp = O.OracleLP(I.serving_expand(compact[k]))
        o = O.OracleSolver(lp, beta=10.0, schedule=O.SCHED_DET, seed=trace[k]["seed"] % (1 << 31))
        ta = time.perf_counter()
        o.run(int(r.epochs))
        spent += time.perf_counter() - ta
        done_work += work[q]
        n_done += 1
        om = o.metrics()
        rel = lambda a, b: abs(a - b) / max(1.0, abs(b))
        agree += int(rel(r.F, om["F"]) <= 1e-4 and rel(r.lp_value, om["lp_value"]) <= 1e-4)
    rate = done_work / spent
    return dict(value=rate / float(np.mean(work)), unit="solves/s", cores=1, kind="oracle",
                sample=f"{n_done} of the {len(pick)} size strata solved by the serial FP64 oracle for the epochs "
                       f"their served solves ran ({spent:.1f} s, setup excluded, {rate:.3g} entry updates/s); "
                       f"every stratum's served work priced at that rate",
                agrees_with_gpu=f"{agree}/{n_done} (F and c^T x within 1e-4 relative)")


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--epochs", type=int, default=100)
    ap.add_argument("--n", type=int, default=2_000_000)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--schedule", choices=["det", "async"], default="det")
    ap.add_argument("--cpu-baseline-seconds", type=float, default=15.0,
                    help="time budget of the oracle baseline (0 skips it)")
    ap.add_argument("--copy-calibration-mb", type=int, default=0,
                    help="also run a plain device copy of this size (counter calibration)")
    ap.add_argument("--summarize-counters", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="write the k_sweep traffic summary from two rocprofv3 counter runs and exit")
    ap.add_argument("--workload", choices=["vc_ba", "mc_grid", "mis_batch", "serve", "al_ba", "setcover", "packing",
                                           "map"],
                    default="vc_ba")
    ap.add_argument("--outer", type=int, default=200, help="al_ba / setcover / packing: most multiplier steps")
    ap.add_argument("--inner", type=int, default=None, help="al_ba / setcover / packing: epochs between multiplier steps")
    ap.add_argument("--feas-tol", type=float, default=None, help="al_ba / setcover / packing: ||A y - b||_inf to stop at")
    ap.add_argument("--lp-gap-tol", type=float, default=None, help="al_ba / setcover / packing: certified LP gap to stop at")
    ap.add_argument("--side", type=int, default=1024, help="mc_grid: grid side")
    ap.add_argument("--rate", type=float, default=200.0, help="serve: arrivals per second")
    ap.add_argument("--duration", type=float, default=10.0, help="serve: seconds of arrivals")
    ap.add_argument("--budget-gb", type=float, default=0.0, help="serve: device-memory budget (0: half of free)")
    ap.add_argument("--slots", type=int, default=256, help="serve: slots per batch kind")
    ap.add_argument("--builders", type=int, default=12, help="serve: host layout threads")
    ap.add_argument("--serve-log", default="", help="serve: append one JSON line per request to this file")
    ap.add_argument("--instances", type=int, default=4096, help="mis_batch: instance count")
    ap.add_argument("--precision", choices=["bf16", "fp32"], default="fp32", help="mis_batch: x storage")
    ap.add_argument("--gap", type=float, default=1e-4, help="mis_batch: certified gap to stop at")
    ap.add_argument("--cap", type=int, default=200, help="mis_batch: epoch cap")
    ap.add_argument("--baseline-sample", type=int, default=32, help="mis_batch: instances solved alone")
    ap.add_argument("--window", type=int, default=256,
                    help="mis_batch: most instances running at once (0: all); the rest start as they retire")
    args = ap.parse_args()

    if args.summarize_counters:
        wl = f"vc_ba_n{args.n}_m3_beta10_fp32_refresh5_{args.epochs}ep_{args.schedule}"
        cmd = ("cd /tmp && rocprofv3 --pmc FETCH_SIZE (then WRITE_SIZE) --output-format csv -d <out> -o run -- "
               f"python3 <repo>/bench.py --steps 1 --warmup 0 --epochs {args.epochs} --cpu-baseline-seconds 0 "
               f"--copy-calibration-mb {args.copy_calibration_mb or 256}")
        return summarize_counters(*args.summarize_counters, wl, args.copy_calibration_mb or 256, cmd)

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: the solve is sized for one MI355X and the library "
              "has no multi-GPU path (run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    if args.workload == "mis_batch":
        return mis_batch(args)
    if args.workload == "serve":
        return serve(args)
    if args.workload in AL_WORKLOADS:
        return al_workload(args)
    if args.workload == "mc_grid":
        if args.epochs == 100:
            args.epochs = 200
        return mc_grid(args)

    import numpy as np
    import torch
    from paper_1311_2661_amd import instances as I
    from paper_1311_2661_amd import thetis as T

    T.lib()
    assert torch.cuda.is_available(), "bench needs a GPU"
    torch.cuda.set_device(0)
    t0 = time.perf_counter()
    inst = I.vc_ba(args.n, seed=args.seed)
    log(f"instance: BA n={inst.n} edges={inst.m} ({time.perf_counter() - t0:.1f} s)")
    t0 = time.perf_counter()
    sched = T.SCHED_DET if args.schedule == "det" else T.SCHED_ASYNC
    h = T.Instance(inst)
    s = T.Solver(h, beta=10.0, precision=T.PREC_FP32, refresh_every=5, schedule=sched,
                 step_scale=1.0 if sched == T.SCHED_DET else 0.5, seed=args.seed)
    nclasses = h.classes()[0]
    log(f"layout + upload: {time.perf_counter() - t0:.1f} s, {nclasses} colour classes")
    tuned = s.autotune(4) if sched == T.SCHED_DET else []      # real epochs; every step resets
    log(f"columns per lane group by class: {tuned}")
    traffic = s.traffic()
    upd_per_epoch = traffic["updates_per_epoch"]

    if args.copy_calibration_mb:
        a = torch.empty(args.copy_calibration_mb * 1024 * 1024 // 4, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        a.fill_(1.0)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        log(f"copy calibration: {args.copy_calibration_mb} MiB read + written 3 times")

    def step():
        s.reset()
        s.run(args.epochs)
        sol, cost, aux = s.round(T.ROUND_VC_THRESH)
        feas, nv = s.check(T.ROUND_VC_THRESH)
        return cost, feas, nv

    for w in range(args.warmup):
        cost, feas, nv = step()
        log(f"warmup {w}: cover cost {cost:.6g} feasible {feas}")

    s.set_timing(10)            # events around the launches of every 10th epoch
    acc = {k: dict(ms=0.0, launches=0, alg_bytes=0.0) for k in T.KERNEL_NAMES.values()}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    results = []
    for k in range(args.steps):
        results.append(step())
        tm = s.timing()
        for name, v in tm.items():
            for f in ("ms", "launches", "alg_bytes"):
                acc[name][f] += v[f]
        log(f"step {k} done")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    s.set_timing(0)
    m = s.metrics()
    log(f"final: F={m['F']:.10g} lp={m['lp_value']:.10g} gap={m['gap']:.3e} viol={m['max_viol']:.3e}")
    assert all(r[1] for r in results), "rounded solution infeasible"

    total_updates = args.steps * args.epochs * upd_per_epoch
    value = total_updates / elapsed
    g = acc["k_sweep"]
    avg_ms = g["ms"] / max(g["launches"], 1)
    avg_bytes = g["alg_bytes"] / max(g["launches"], 1)
    achieved = avg_bytes / (avg_ms * 1e-3) / 1e9 if avg_ms > 0 else 0.0
    workload = f"vc_ba_n{args.n}_m3_beta10_fp32_refresh5_{args.epochs}ep_{args.schedule}"
    tr = counter_traffic(workload)
    step_bytes = args.epochs * traffic["sweep_bytes"] + (args.epochs // 5) * traffic["refresh_bytes"]
    kernels = {name: dict(ms_total=round(v["ms"], 4), launches=v["launches"],
                          avg_us=round(1e3 * v["ms"] / max(v["launches"], 1), 3),
                          alg_gbs=round(v["alg_bytes"] / max(v["ms"], 1e-9) / 1e6, 1))
               for name, v in acc.items() if v["launches"]}
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "coord updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": workload, "graph": "barabasi_albert", "n_vertices": inst.n,
                   "edges": inst.m, "coordinates_per_epoch": upd_per_epoch, "epochs": args.epochs,
                   "beta": 10.0, "refresh_every": 5, "schedule": args.schedule,
                   "colour_classes": nclasses, "group_cols_by_class": tuned, "seed": args.seed},
        "hbm_gbs_algorithmic_step": step_bytes / (elapsed / args.steps) / 1e9,
        "roofline": {"bound": "hbm", "kernel": "k_sweep", "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": tr, "alg_bytes_per_launch": avg_bytes, "avg_launch_us": 1e3 * avg_ms},
        "kernels": kernels,
        "solution": {"F": m["F"], "lp_value": m["lp_value"], "gap": m["gap"],
                     "max_row_violation": m["max_viol"], "cover_cost": results[-1][0],
                     "feasible": bool(results[-1][1])},
    }
    if sched == T.SCHED_DET:
        owned, foreign, ncols = access_split(inst, h.classes()[2])
        sweep_ms_epoch = g["ms"] / max(g["launches"], 1) * (nclasses - 1)
        out["random_access"] = random_access_model(T, inst.m, owned, foreign, ncols, sweep_ms_epoch)
        log(f"random access: {out['random_access']}")
    if args.cpu_baseline_seconds > 0:
        log("cpu baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline(inst, args.epochs, args.cpu_baseline_seconds, args.seed)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
