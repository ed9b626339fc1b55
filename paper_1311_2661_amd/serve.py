"""Continuous-batching LP-rounding server on one GPU.

Requests (an LP relaxation of vertex cover, independent set or multiway cut)
arrive at any time.  A pool of builder threads makes each request's host
layout (the library call releases the GIL).  Admission is by device-memory
budget: a built request takes a slot as soon as its workspace fits in the
budget and its batch has a free slot; otherwise it waits (first fit in
arrival order, never dropped).  An admitted request's device state is
allocated and uploaded by an uploader thread on its own stream, so the
batch keeps running meanwhile; it joins the batch at the next tick.  Each batch kind -- all-ones matrices (vertex
cover, independent set) and +-1 matrices (multiway cut) -- has one worker
thread and one stream, so their epochs overlap on the device.  A worker
admits waiting requests into free slots, runs `epochs_per_tick` epochs of
every slot in one batched launch sequence, and hands back every solve that
reached the certified gap (or its epoch cap): rounding, feasibility check,
result, slot and memory released.  Each solve computes exactly what it
would compute alone (the batch guarantees it), so results do not depend on
what else is being served.

A request may carry a deadline (seconds after its arrival): one still
waiting or being built when it passes fails with DeadlineExceeded; one
already on the device is finished at the next tick from its current point
(rounded and checked like any other, with reason "deadline").  Every
finished or failed request can be appended as one JSON line to a log.
Builders stop building while many built requests wait for a slot, so a
backlog holds compact requests, not layouts.
"""
from __future__ import annotations

import concurrent.futures as cf
import json
import threading
import time
from dataclasses import dataclass, field
from typing import Optional

import numpy as np

from . import thetis as T

RULES = {"vc": T.ROUND_VC_THRESH, "mis": T.ROUND_MIS_RAND, "mc": T.ROUND_MC_CKR}
GROUP = {"vc": "ones", "mis": "ones", "mc": "signed"}


@dataclass
class Result:
    kind: str
    sol: np.ndarray
    cost: float
    feasible: bool
    n_violated: int
    epochs: int
    F: float
    lp_value: float
    gap: float
    reached_gap: bool
    t_arrival: float
    t_admitted: float
    t_done: float
    reason: str = "gap"          # why it stopped: "gap", "cap", "deadline" or "diverged"

    @property
    def latency(self) -> float:
        return self.t_done - self.t_arrival


class DeadlineExceeded(RuntimeError):
    """The request's deadline passed before it reached the device."""


@dataclass
class _Req:
    rid: int
    kind: str
    lp: object
    seed: int
    t_arrival: float
    future: cf.Future
    deadline: Optional[float] = None      # absolute (perf_counter) time, or None
    instance: Optional[T.Instance] = None
    ws_bytes: int = 0
    solver: Optional[T.Solver] = None
    slot: int = -1
    epochs: int = 0
    t_admitted: float = 0.0
    workspace: object = None
    upload: Optional[cf.Future] = None


def admit(waiting, free_bytes: int, free_slots: dict, hold_from: int = -1) -> list:
    """First fit in arrival order: the indices of `waiting` (objects with
    ``ws_bytes`` and ``kind``) that can start now.  `free_slots` maps a
    batch group to its free slot count and is decremented.  With
    ``hold_from >= 0`` nothing at or after that position is admitted (an
    older request has waited too long for memory and goes first)."""
    picked = []
    for k, r in enumerate(waiting):
        if 0 <= hold_from <= k:
            break
        g = GROUP[r.kind]
        if r.ws_bytes <= free_bytes and free_slots.get(g, 0) > 0:
            picked.append(k)
            free_bytes -= r.ws_bytes
            free_slots[g] -= 1
    return picked


class Server:
    AGING_S = 0.5

    def __init__(self, hbm_budget: int, gap_tol: float = 1e-4, epoch_cap: int = 200,
                 epochs_per_tick: int = 5, slots: int = 256, precision: int = T.PREC_FP32,
                 builders: int = 4, beta: float = 10.0, reps: int = 10,
                 deadline_s: Optional[float] = None, log_path: Optional[str] = None,
                 max_built_waiting: Optional[int] = None):
        import torch
        if epoch_cap % epochs_per_tick:
            raise ValueError("epoch_cap must be a multiple of epochs_per_tick")
        self.deadline_s = deadline_s
        self.log = open(log_path, "a") if log_path else None
        self.log_lock = threading.Lock()
        # built requests allowed to wait for a slot before builders pause
        self.max_built = max_built_waiting if max_built_waiting else 2 * slots
        self.budget = int(hbm_budget)
        self.gap_tol, self.cap, self.tick = gap_tol, epoch_cap, epochs_per_tick
        self.precision, self.beta, self.reps = precision, beta, reps
        self.lock = threading.Lock()
        self.cv = threading.Condition(self.lock)
        self.used = 0
        self.peak_used = 0
        self.waiting = []               # built, not admitted
        self.pending_builds = 0
        self.closed = False
        self.next_id = 0
        self.builders = cf.ThreadPoolExecutor(max_workers=builders)
        self.uploaders = cf.ThreadPoolExecutor(max_workers=2)
        self._local = threading.local()
        self.device = torch.device("cuda", torch.cuda.current_device())
        self.groups = {}
        for g in ("ones", "signed"):
            stream = torch.cuda.Stream(device=self.device)
            batch = T.Batch(capacity=slots, precision=precision, unit_values=(g == "ones"), stream=stream)
            self.groups[g] = dict(stream=stream, batch=batch, slots=[None] * slots, thread=None, uploading=[])
        for g in self.groups:
            t = threading.Thread(target=self._worker, args=(g,), daemon=True, name=f"thetis-serve-{g}")
            self.groups[g]["thread"] = t
            t.start()

    # -------------------------------------------------------------- client side
    def submit(self, lp, kind: str, seed: int = 0, t_arrival: Optional[float] = None,
               deadline_s: Optional[float] = None) -> cf.Future:
        """Queues one request; `deadline_s` (else the server's default) is
        counted from its arrival."""
        if kind not in RULES:
            raise ValueError(f"unknown request kind {kind}")
        fut = cf.Future()
        with self.lock:
            if self.closed:
                raise RuntimeError("server closed")
            rid = self.next_id
            self.next_id += 1
            self.pending_builds += 1
        t0 = time.perf_counter() if t_arrival is None else t_arrival
        dl = deadline_s if deadline_s is not None else self.deadline_s
        req = _Req(rid, kind, lp, seed, t0, fut, None if dl is None else t0 + dl)
        self.builders.submit(self._build, req)
        return fut

    def _expired(self, r: _Req, now: float) -> bool:
        return r.deadline is not None and now > r.deadline

    def _record(self, r: _Req, res: Optional[Result], err: Optional[BaseException]):
        """One JSON line per finished or failed request."""
        if self.log is None:
            return
        rec = dict(id=r.rid, kind=r.kind, seed=r.seed, ws_bytes=r.ws_bytes, epochs=r.epochs,
                   t_arrival=r.t_arrival, t_admitted=r.t_admitted or None)
        if res is not None:
            rec.update(reason=res.reason, gap=res.gap, F=res.F, lp_value=res.lp_value, cost=res.cost,
                       feasible=bool(res.feasible), n_violated=int(res.n_violated), t_done=res.t_done,
                       latency_s=res.latency)
        else:
            rec.update(reason="error", error=f"{type(err).__name__}: {err}", t_done=time.perf_counter())
        with self.log_lock:
            if self.log is not None:      # closed meanwhile: the record is dropped with the log
                self.log.write(json.dumps(rec) + "\n")
                self.log.flush()

    def _fail(self, r: _Req, err: BaseException):
        self._record(r, None, err)
        r.future.set_exception(err)

    def _build(self, req: _Req):
        with self.lock:
            # backpressure: a backlog waits as compact requests, not as layouts
            while len(self.waiting) >= self.max_built and not self.closed and not self._expired(
                    req, time.perf_counter()):
                self.cv.wait(timeout=0.05)
        if self._expired(req, time.perf_counter()):
            with self.lock:
                self.pending_builds -= 1
                self.cv.notify_all()
            self._fail(req, DeadlineExceeded(f"request {req.rid}: deadline passed before it was built"))
            return
        try:
            lp = req.lp() if callable(req.lp) else req.lp      # a request may carry a builder
            req.lp = None
            req.instance = T.Instance(lp)
            del lp
            p = T.thetis_params_default()
            p.beta, p.precision, p.refresh_every, p.seed = self.beta, self.precision, self.tick, req.seed
            req.ws_bytes = T.thetis_solver_workspace_bytes(req.instance.h, p)
            if req.ws_bytes > self.budget:
                raise T.ThetisError(T.EBUDGET, "request larger than the whole device-memory budget")
        except Exception as e:     # reported to the caller, never silently dropped
            with self.lock:
                self.pending_builds -= 1
                self.cv.notify_all()
            self._fail(req, e)
            return
        with self.lock:
            self.pending_builds -= 1
            self.waiting.append(req)
            self.cv.notify_all()

    def close(self, wait: bool = True):
        with self.lock:
            self.closed = True
            self.cv.notify_all()
        self.builders.shutdown(wait=wait)
        if wait:
            for g in self.groups.values():
                g["thread"].join()
        self.uploaders.shutdown(wait=wait)
        if self.log is not None:
            with self.log_lock:
                self.log.close()
                self.log = None

    # -------------------------------------------------------------- device side
    def _expire_locked(self, g: str) -> list:
        """Takes the waiting requests of group g whose deadline has passed
        off the queue (they are failed outside the lock)."""
        now = time.perf_counter()
        gone = [r for r in self.waiting if GROUP[r.kind] == g and self._expired(r, now)]
        for r in gone:
            self.waiting.remove(r)
        if gone:
            self.cv.notify_all()
        return gone

    def _admit_locked(self, g: str):
        grp = self.groups[g]
        reserved = {r.slot for r in grp["uploading"]}
        free = [k for k, s in enumerate(grp["slots"]) if s is None and k not in reserved]
        mine = [r for r in self.waiting if GROUP[r.kind] == g]
        if not mine or not free:
            return []
        # aging: once the oldest waiting request has waited AGING_S for
        # memory, newer requests (of any kind) wait until it fits
        hold = -1
        if self.waiting:
            old = self.waiting[0]
            if (old.ws_bytes > self.budget - self.used and
                    time.perf_counter() - old.t_arrival > self.AGING_S):
                hold = 0 if GROUP[old.kind] != g else mine.index(old) + 1
        picked = admit(mine, self.budget - self.used, {g: len(free)}, hold_from=hold)
        out = []
        for k in picked:
            r = mine[k]
            r.slot = free.pop(0)
            self.used += r.ws_bytes
            self.peak_used = max(self.peak_used, self.used)
            out.append(r)
        for r in out:
            self.waiting.remove(r)
        if out:
            self.cv.notify_all()
        return out

    def _make_solver(self, r: _Req):
        """Uploader thread: the request's device state, on this thread's own
        stream (the batch waits for that stream before its first epoch)."""
        import torch
        loc = self._local
        if getattr(loc, "stream", None) is None:
            loc.stream = torch.cuda.Stream(device=self.device)
        with torch.cuda.device(self.device), torch.cuda.stream(loc.stream):
            return T.Solver(r.instance, beta=self.beta, precision=self.precision,
                            refresh_every=self.tick, seed=r.seed)

    def _worker(self, g: str):
        import torch
        grp = self.groups[g]
        batch, stream = grp["batch"], grp["stream"]
        with torch.cuda.device(self.device), torch.cuda.stream(stream):
            while True:
                expired, stop = [], False
                with self.lock:
                    while True:
                        expired += self._expire_locked(g)
                        for r in self._admit_locked(g):
                            r.upload = self.uploaders.submit(self._make_solver, r)
                            grp["uploading"].append(r)
                        busy = any(s is not None for s in grp["slots"])
                        if busy or grp["uploading"] or expired:
                            break
                        if self.closed and self.pending_builds == 0 and not any(
                                GROUP[r.kind] == g for r in self.waiting):
                            stop = True
                            break
                        self.cv.wait(timeout=0.05)
                for r in expired:
                    r.instance.close()
                    r.instance = None
                    self._fail(r, DeadlineExceeded(f"request {r.rid}: deadline passed while waiting for a slot"))
                if stop:
                    return
                # uploaded requests join the batch
                if grp["uploading"] and not busy:
                    cf.wait([r.upload for r in grp["uploading"]], timeout=0.05,
                            return_when=cf.FIRST_COMPLETED)
                for r in [r for r in grp["uploading"] if r.upload.done()]:
                    grp["uploading"].remove(r)
                    try:
                        r.solver = r.upload.result()
                        r.t_admitted = time.perf_counter()
                        grp["slots"][r.slot] = r
                        batch.set(r.slot, r.solver)
                    except Exception as e:
                        grp["slots"][r.slot] = None
                        self._release(g, r)
                        self._fail(r, e)
                if not any(s is not None for s in grp["slots"]):
                    continue
                try:
                    done = batch.run(self.tick, self.gap_tol)
                except Exception as e:
                    # a failed batch call ends every request the batch held
                    self._fail_all(g, e)
                    continue
                status = batch.last_status
                now = time.perf_counter()
                for slot, r in enumerate(grp["slots"]):
                    if r is None:
                        continue
                    r.epochs += int(done[slot])
                    st = int(status[slot])
                    if st in (1, 3) or r.epochs >= self.cap:
                        self._finish(g, r, reached=(st == 1), reason={1: "gap", 3: "diverged"}.get(st, "cap"))
                    elif self._expired(r, now):
                        self._finish(g, r, reached=False, reason="deadline")

    def _finish(self, g: str, r: _Req, reached: bool, reason: str):
        grp = self.groups[g]
        try:
            s = r.solver
            m = s.metrics()
            sol, cost, _ = s.round(RULES[r.kind], seed=r.seed, reps=self.reps)
            feas, nv = s.check(RULES[r.kind])
            res = Result(r.kind, sol, cost, feas, nv, r.epochs, m["F"], m["lp_value"], m["gap"], reached,
                         r.t_arrival, r.t_admitted, time.perf_counter(), reason)
            err = None
        except Exception as e:
            err = e
        grp["batch"].set(r.slot, None)
        grp["slots"][r.slot] = None
        self._release(g, r)
        if err is None:
            self._record(r, res, None)
            r.future.set_result(res)
        else:
            self._fail(r, err)

    def _fail_all(self, g: str, err: Exception):
        grp = self.groups[g]
        for slot, r in enumerate(grp["slots"]):
            if r is None:
                continue
            grp["batch"].set(slot, None)
            grp["slots"][slot] = None
            self._release(g, r)
            self._fail(r, err)

    def _release(self, g: str, r: _Req):
        if r.solver is not None:
            r.solver.close()
            r.solver = None
        if r.instance is not None:
            r.instance.close()
            r.instance = None
        with self.lock:
            if r.slot >= 0:
                self.used -= r.ws_bytes
            self.cv.notify_all()


def solve_alone(lp, kind: str, seed: int = 0, gap_tol: float = 1e-4, epoch_cap: int = 200,
                epochs_per_tick: int = 5, precision: int = T.PREC_FP32, beta: float = 10.0, reps: int = 10):
    """The same solve as the server's, by itself: run to the gap (checked at
    every refresh) or the cap, round, check."""
    s = T.Solver(T.Instance(lp), beta=beta, precision=precision, refresh_every=epochs_per_tick, seed=seed)
    e = s.run(epoch_cap, gap_tol=gap_tol)
    m = s.metrics()
    sol, cost, _ = s.round(RULES[kind], seed=seed, reps=reps)
    feas, nv = s.check(RULES[kind])
    s.close()
    return dict(sol=sol, cost=cost, feasible=feas, epochs=e, F=m["F"], gap=m["gap"])
