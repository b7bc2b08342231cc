"""Continuous-batching FCIQMC solve server over the C ABI.

Requests (a Hamiltonian, run parameters and an arrival time) are admitted into
the slots of one batch handle as soon as a slot is free and their tables fit
in device memory (``fciqmc_batch_admit`` checks the footprint of the walker
target's main list and integrals against free HBM and fails with ENOMEM
otherwise). All admitted
systems advance together in graph-captured launches; each runs until its
projected-energy error bar reaches the tolerance (with a minimum number of
averaged iterations) or until its iteration budget is spent, then it is
retired and its slot and memory are reused. Requests that arrive while others
run are admitted between launches, so their work overlaps on the device.

Each system's trajectory depends only on its own inputs and its own iteration
count (the random numbers are keyed by determinant and iteration, merges are
integer sums), so a result is identical whether it was served alone or in the
mix. The launch shape can be autotuned once the server is busy; the trials
run on a snapshot of every admitted system, which is restored afterwards.
"""
from __future__ import annotations

import time
from dataclasses import dataclass, field

import numpy as np

from . import fciqmc as F


@dataclass
class Request:
    ham: object
    params: object
    arrival: float = 0.0          # seconds after the server starts
    max_iters: int = 20000
    tag: object = None


MILESTONES = (1e-2, 3e-3, 1e-3)   # error bars (Ha) whose first crossing is timed


@dataclass
class Result:
    tag: object
    arrival: float
    admitted: float
    finished: float
    iterations: int
    e_proj: float
    e_proj_err: float
    shift_energy: float
    attempts: int
    converged: bool
    failed: bool = False          # the system stopped with an error (status != 0)
    reached: dict = field(default_factory=dict)   # milestone -> seconds after arrival
    walkers: tuple | None = None

    @property
    def latency(self):
        return self.finished - self.arrival


def _pcts(x):
    x = np.asarray(x, dtype=float)
    if not x.size:
        return None, None
    return float(np.percentile(x, 50)), float(np.percentile(x, 99))


@dataclass
class ServerStats:
    results: list = field(default_factory=list)
    wall_s: float = 0.0
    launches: int = 0
    peak_active: int = 0
    tuned_shape: tuple | None = None

    def summary(self):
        res = self.results
        lat = [r.latency for r in res] or [0.0]
        conv = [r.latency for r in res if r.converged]
        att = sum(r.attempts for r in res)
        errs = [r.e_proj_err for r in res if not r.failed and np.isfinite(r.e_proj_err)]
        p50, p99 = _pcts(lat)
        c50, c99 = _pcts(conv)
        out = {"requests": len(res), "wall_s": self.wall_s,
               "p50_latency_s": p50, "p99_latency_s": p99,
               "converged": len(conv), "failed": sum(1 for r in res if r.failed),
               "p50_time_to_error_bar_s": c50, "p99_time_to_error_bar_s": c99,
               "throughput_req_per_s": len(res) / max(self.wall_s, 1e-9),
               "attempts_per_s": att / max(self.wall_s, 1e-9),
               "e_proj_err_p50": float(np.median(errs)) if errs else None,
               "iterations_p50": float(np.median([r.iterations for r in res])) if res else 0.0,
               "launches": self.launches, "peak_active": self.peak_active,
               "autotuned_shape": self.tuned_shape}
        for m in MILESTONES:
            t = [r.reached[m] for r in res if m in r.reached]
            a, b = _pcts(t)
            out[f"reached_{m:g}"] = {"requests": len(t), "p50_s": a, "p99_s": b}
        return out


class SolveServer:
    def __init__(self, max_slots=16, chunk_iters=64, tol=1e-3, min_samples=256,
                 keep_walkers=False, stream=None, clock=time.perf_counter, on_result=None,
                 autotune_iters=0, on_progress=None, progress_every_s=20.0):
        self.autotune_iters = autotune_iters   # > 0: tune once, when half the slots are busy
        self.max_slots = max_slots
        self.chunk_iters = chunk_iters
        self.tol = tol
        self.min_samples = min_samples
        self.keep_walkers = keep_walkers
        self.stream = stream if stream is not None else F.current_stream()
        self.clock = clock
        self.on_result = on_result        # called with each Result as it is retired
        self.on_progress = on_progress    # called with a status line after launches
        self.progress_every_s = progress_every_s

    def run(self, requests):
        """Serve `requests` (arrival times in seconds from now); returns ServerStats."""
        pending = sorted(requests, key=lambda r: r.arrival)
        h = F.fciqmc_batch_create(self.max_slots, [], [], self.stream)
        active = {}          # slot -> [request, admitted_at, iterations_done, milestones]
        stats = ServerStats()
        t0 = self.clock()
        last_note = t0
        try:
            while pending or active:
                now = self.clock() - t0
                # admit arrived requests while slots and memory allow
                while pending and pending[0].arrival <= now and len(active) < self.max_slots:
                    req = pending[0]
                    try:
                        slot = F.fciqmc_batch_admit(h, req.ham, req.params)
                    except F.FciqmcError as e:
                        if e.code == -2 and active:      # ENOMEM: wait for a retirement
                            break
                        if e.code != -1:
                            raise
                        # EINVAL: a request this batch cannot hold (bad parameters, or
                        # determinants of another width than the batch's one word)
                        pending.pop(0)
                        stats.results.append(Result(req.tag, req.arrival, now, now, 0, float("nan"),
                                                    float("nan"), float("nan"), 0, False, True, {},
                                                    None))
                        if self.on_result is not None:
                            self.on_result(stats.results[-1])
                        continue
                    pending.pop(0)
                    active[slot] = [req, now, 0, {}]
                stats.peak_active = max(stats.peak_active, len(active))
                if not active:
                    # idle until the next arrival
                    wait = pending[0].arrival - (self.clock() - t0)
                    if wait > 0:
                        time.sleep(min(wait, 0.05))
                    continue
                if (self.autotune_iters > 0 and stats.tuned_shape is None
                        and 2 * len(active) >= self.max_slots):
                    stats.tuned_shape = tuple(F.fciqmc_autotune(h, self.autotune_iters))
                n = np.zeros(self.max_slots, np.int32)
                for slot, (req, _, done, _) in active.items():
                    n[slot] = min(self.chunk_iters, req.max_iters - done)
                F.fciqmc_batch_iterate_each(h, n)
                stats.launches += 1
                now = self.clock() - t0
                for slot in list(active):
                    req, adm, done, reached = active[slot]
                    e = F.fciqmc_batch_slot_estimators(h, slot)
                    done = e["iteration"]                # iterations the system really ran
                    active[slot][2] = done
                    failed = e["status"] != 0
                    ok = e["n_samples"] >= self.min_samples and np.isfinite(e["e_proj_err"]) \
                        and e["e_proj_err"] > 0.0 and not failed
                    for m in MILESTONES:
                        if ok and m not in reached and e["e_proj_err"] <= m:
                            reached[m] = now - req.arrival
                    conv = ok and e["e_proj_err"] <= self.tol
                    if conv or failed or done >= req.max_iters:
                        walkers = F.fciqmc_batch_slot_walkers(h, slot) if self.keep_walkers else None
                        stats.results.append(Result(
                            req.tag, req.arrival, adm, now, done, e["e_proj_mean"],
                            e["e_proj_err"], e["shift_mean"], e["total_attempts"], bool(conv),
                            failed, dict(reached), walkers))
                        if self.on_result is not None:
                            self.on_result(stats.results[-1])
                        F.fciqmc_batch_retire(h, slot)
                        del active[slot]
                if self.on_progress is not None and self.clock() - last_note >= self.progress_every_s:
                    last_note = self.clock()
                    self.on_progress(f"t {now:.0f} s: {len(stats.results)} retired, {len(active)} "
                                     f"active, {len(pending)} waiting, {stats.launches} launches")
        finally:
            F.fciqmc_free(h)
        stats.wall_s = self.clock() - t0
        return stats
