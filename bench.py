"""Throughput benchmark of the FCIQMC iteration on one MI355X.

Workload (one step = one full iteration: spawning, death, annihilation,
estimators, shift): the 24-electron / 30-orbital synthetic system with a
12-orbital near-degenerate band (60 spin orbitals, one 64-bit word per
determinant), initiator threshold 3, tau = 5e-4, at >= 1e8 walkers.

Input preparation (untimed): a growth stage from walkers on the reference at a
raised constant shift (cloning everywhere) until N_w reaches the walker target;
the shift is then set to the instantaneous projected-energy estimate and varies
from there (update every 10 iterations with damping 0.5: the dominant eigenvalue
of this system's initiator dynamics lies ~20 Ha below E0, and the gap between
shift and eigenvalue shrinks by 1 - damping per update, so the population
settles within the warm-up instead of growing several-fold), W warm-up
iterations let it settle, and the table is sized for the window so that no
re-bucketing falls inside it.
Timed: K iterations on the library's production path (graph launches of up
to 64 iterations, walker list resident in device memory), wall clock between
device synchronisations. Beside it, a shorter window in profiling mode (every
kernel launched directly, bracketed by HIP events on the library's stream)
gives per-kernel times, from which the rooflines are computed with the
per-iteration counts of the same iterations (fciqmc_history).

Also reported: annihilated determinants/s (spawn records entering
annihilation), the CPU oracle on a bounded sample of the same walker list,
batching (64 systems, walker targets 1e4-1e6, 2000 iterations, batched vs the
same systems one after another) and serving (a Poisson stream of 200 requests
at 20 per second, each run to a 1e-3 Ha error bar or an iteration cap: 4000 in
the default run, 20000 for the full serving workload with --served-max-iters).
"""
import argparse
import json
import math
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

HBM_PEAK_GBS = 8000.0
# 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz: 32-bit vector lane-operations per second
# (one wave64 VALU instruction is 64 lane-operations and issues in 4 cycles)
ALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12
# Algorithmic lane-operations of one spawning attempt (double excitation, no point
# group), every instruction counted once: Philox4x32-10 block (10 rounds of two
# 32x32->64 products and two three-input XORs, + counter set-up: 42), type test (3),
# pair index by the square-root estimate with its two corrections (18), two
# electron selections by bit halving + byte table (2 x 18), allowed-hole sets and
# counts (10), two hole selections with their draws (2 x 19), the child determinant
# (12), the Slater-Condon double element with its two integral addresses and parity
# (50), acceptance: tau |H| / pgen with the IEEE division, floor, compare (20),
# spawn sign and queue append (15), attempt-to-walker bookkeeping (8).
OPS_PER_ATTEMPT = 252
PROFILES = os.path.join(ROOT, "profiles")
GROUPS = ["chunk_sums", "scans", "spawn", "annihilation", "statistics"]
# Kernels of each group (the annihilation group is the record sort and k_post).
GROUP_KERNELS = {"spawn": ["k_spawn"],
                 "annihilation": ["k_fix", "k_bscan_up", "k_bscan_top", "k_bscan_down",
                                  "k_scatter", "k_post"]}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


class Roctx:
    """roctxProfilerResume/Pause, so rocprofv3 --selected-regions covers the profiling window."""

    def __init__(self):
        self.mod = None
        py = "/opt/rocm/lib/python%d.%d/site-packages" % sys.version_info[:2]
        if os.path.isdir(os.path.join(py, "roctx")):
            sys.path.append(py)
            try:
                import roctx
                self.mod = roctx
            except Exception:
                self.mod = None

    def resume(self):
        if self.mod is not None:
            self.mod.profilerResume(0)

    def pause(self):
        if self.mod is not None:
            self.mod.profilerPause(0)


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def grow(solver, target, log_every=40):
    it = 0
    while True:
        e = solver.estimates()
        if e["n_walkers"] >= target:
            return e
        step = 20 if e["n_walkers"] * 4 < target else 2
        solver.iterate(step)
        it += step
        if it % log_every == 0 or step == 2:
            e = solver.estimates()
            log(f"[grow] iter {e['iteration']} N_w {e['n_walkers']} N_d {e['n_dets']} "
                f"C0 {e['ref_pop']} spawns {e['spawns']}")
        if it > 20000:
            raise RuntimeError("growth stage did not reach the walker target")


def history(F, h, first, n):
    """Per-iteration records first .. first + n - 1 (in pieces of at most 256)."""
    out = []
    while n > 0:
        m = min(n, 256)
        out += F.fciqmc_history(h, 0, first, m)
        first += m
        n -= m
    return out


def method_bytes(recs, nd_before):
    """Algorithmic HBM bytes per iteration of the annihilation group and of k_post alone
    (mean over the records), counted per occupied determinant (21 B read: key, population,
    H_DD and the initiator flag; 4 B population written by death), per spawn record (16 B
    read by the annihilation pass; 32 B more to partition it by bucket: read and write),
    per merged spawn target (8 B key + 4 B population read, 4 B written) and per new
    determinant (20 B: key, population, H_DD written)."""
    group, post = [], []
    prev = nd_before
    for r in recs:
        main = 25.0 * prev
        post.append(main + 16.0 * r["spawns"] + 16.0 * r["merged"] + 20.0 * r["born"])
        group.append(post[-1] + 32.0 * r["spawns"])
        prev = r["n_dets"]
    return float(np.mean(group)), float(np.mean(post))


def kernel_source_hash():
    import hashlib
    with open(os.path.join(ROOT, "paper_1305_6981_amd", "csrc", "kernels.hip"), "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def read_profile(name):
    """key: value pairs of profiles/<name>, or None when missing or when its kernels
    hash differs from the current source (the counters then describe other code)."""
    path = os.path.join(PROFILES, name)
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    if vals.get("kernels_sha256") != kernel_source_hash():
        return None
    return vals


def measured_traffic(kernels):
    """Calibrated HBM bytes per launch summed over `kernels` from the committed counter
    summary, or None."""
    v = read_profile("hbm_traffic_synth24e30o.txt")
    if v is None:
        return None
    try:
        return sum(float(v[f"{k}_bytes_per_launch"]) for k in kernels)
    except KeyError:
        return None


def issued_ops_per(kern, unit):
    v = read_profile(f"{kern}_valu_synth24e30o.txt")
    if v is None:
        return None
    try:
        return float(v[f"issued_lane_ops_per_{unit}"])
    except KeyError:
        return None


def cpu_baseline(ham, prm, det, pop, e, budget_attempts):
    from oracle import oracle as O
    rng = np.random.default_rng(7)
    order = rng.permutation(len(det))
    acc = np.cumsum(np.abs(pop[order].astype(np.int64)))
    n_take = min(len(order), int(np.searchsorted(acc, budget_attempts)) + 1)
    take = np.sort(order[:n_take])
    o = O.Oracle(ham, prm)
    o.load_walkers(det[take], pop[take], iteration=e["iteration"], shift=e["shift"],
                   n_prev=e["n_prev"], varying=1, n_var=e["n_var"])
    t0 = time.perf_counter()
    o.iterate(1)
    dt = time.perf_counter() - t0
    eo = o.estimates()
    w1 = o.walkers()
    o.close()
    model = cpu_model()
    out = {"value": eo["attempts"] / dt, "unit": "spawn attempts/s", "cores": 1,
           "kind": "oracle", "cpu_model": model,
           "annihilated_dets_per_s": eo["spawns"] / dt,
           "sample": f"one iteration of the single-threaded oracle on {len(take)} determinants "
                     f"({eo['attempts']} walkers) drawn at random from the timed walker list; "
                     f"{dt:.1f} s on one thread of {model}"}
    # The same iteration with the determinants distributed over one virtual
    # process per host thread (the paper's parallel scheme, on the host cores).
    threads = max(1, min(16, len(os.sched_getaffinity(0))))
    o = O.Oracle(ham, prm, n_procs=threads, n_threads=threads)
    o.load_walkers(det[take], pop[take], iteration=e["iteration"], shift=e["shift"],
                   n_prev=e["n_prev"], varying=1, n_var=e["n_var"])
    t0 = time.perf_counter()
    o.iterate(1)
    dt = time.perf_counter() - t0
    ep = o.estimates()
    same = all(np.array_equal(a, b) for a, b in zip(w1, o.walkers()))
    o.close()
    out["virtual_processes"] = {"value": ep["attempts"] / dt, "unit": "spawn attempts/s",
                                "cores": threads, "processes": threads, "cpu_model": model,
                                "annihilated_dets_per_s": ep["spawns"] / dt,
                                "same_walkers_as_single_thread": bool(same)}
    return out


def avg_start_for(prm):
    """Iterations after the shift starts varying before averaging: one unit of imaginary
    time (at least 200 iterations), which lets the shift and the walker distribution
    settle first."""
    return max(200, int(round(1.0 / prm.tau)))


def batched_vs_plain(F, S, iters, scale, tune_at):
    """Config-4 batching: 64 systems advanced together for `iters` iterations (autotuned
    on a snapshot after `tune_at`), then the same systems one after another. Every
    system follows the same trajectory either way (walkers are bit-identical), so the
    two legs reach the same error bars and the wall times compare directly."""
    systems = S.batch_workload(scale=scale)
    hams = [h for h, _ in systems]
    prms = [p for _, p in systems]
    for p in prms:
        p.avg_start = avg_start_for(p)
        # start at a quarter of the target on the reference: the slowest systems would
        # otherwise spend the whole run growing from a few walkers
        p.initial_walkers = max(10, p.target_walkers // 4)
    stream = F.current_stream()
    h = F.fciqmc_batch_create(len(systems), hams, prms, stream)
    t0 = time.perf_counter()
    F.fciqmc_batch_iterate(h, tune_at)
    tb = time.perf_counter() - t0
    shape_default = F.fciqmc_get_launch(h)
    t_tune = time.perf_counter()
    shape = F.fciqmc_autotune(h, 2)
    t_tune = time.perf_counter() - t_tune
    log(f"[batched] autotuned after {tune_at} iterations in {t_tune:.1f} s: "
        f"{shape_default} -> {shape}")
    t0 = time.perf_counter()
    F.fciqmc_batch_iterate(h, iters - tune_at)
    tb += time.perf_counter() - t0
    eb = [F.fciqmc_batch_slot_estimators(h, s) for s in range(len(systems))]
    F.fciqmc_free(h)
    log(f"[batched] {iters} iterations of {len(systems)} systems in {tb:.2f} s")
    t_plain = 0.0
    ep = []
    for i, (hm, pr) in enumerate(systems):
        if i % 16 == 0:
            log(f"[plain] system {i}")
        t0 = time.perf_counter()
        sv = F.Solver(hm, pr, stream)
        sv.iterate(iters)
        ep.append(sv.estimates())
        t_plain += time.perf_counter() - t0
        sv.close()
    same = all(a["n_walkers"] == b["n_walkers"] and a["shift"] == b["shift"] and
               a["total_attempts"] == b["total_attempts"] for a, b in zip(eb, ep))
    err_b = [e["e_proj_err"] for e in eb]
    err_p = [e["e_proj_err"] for e in ep]
    close = all((not math.isfinite(x) and not math.isfinite(y)) or
                abs(x - y) <= 1e-9 * max(1.0, abs(y)) for x, y in zip(err_b, err_p))
    att = sum(e["total_attempts"] for e in eb)
    return {"systems": len(systems), "iterations": iters,
            "walker_targets": [min(p.target_walkers for p in prms),
                               max(p.target_walkers for p in prms)],
            "batched_s": tb, "plain_s": t_plain, "speedup": t_plain / tb,
            "batched_attempts_per_s": att / tb, "plain_attempts_per_s": att / t_plain,
            "same_trajectories": bool(same), "same_error_bars": bool(close),
            "e_proj_err_median_ha": float(np.nanmedian(err_b)),
            "converged_1e-3": int(sum(1 for x in err_b if x <= 1e-3)),
            "autotune": {"after_iterations": tune_at, "seconds": t_tune,
                         "default_shape": list(shape_default), "tuned_shape": list(shape)}}


def served(F, S, n_requests, scale, max_iters, plain_every, seed=5):
    """Config-5 serving: Poisson request stream (mean 20 req/s) served with continuous
    batching; each request runs to a projected-energy error bar of 1e-3 Ha or max_iters
    iterations. A subset of the requests is then run alone for the same iteration
    counts (same trajectories, so the same error bars) to compare with serving."""
    from paper_1305_6981_amd import serve
    reqs = []
    for i, (t, ham, prm) in enumerate(S.serve_requests(n=n_requests, rate=20.0, seed=seed,
                                                       scale=scale)):
        prm.avg_start = avg_start_for(prm)
        prm.initial_walkers = max(10, prm.target_walkers // 2)
        reqs.append(serve.Request(ham, prm, arrival=t, max_iters=max_iters, tag=i))

    def progress(r):
        log(f"[served] request {r.tag} ({reqs[r.tag].ham.name}, target "
            f"{reqs[r.tag].params.target_walkers}) retired after {r.iterations} iterations"
            + (" (failed)" if r.failed else "")
            + f", error bar {r.e_proj_err:.2e} Ha, latency {r.latency:.1f} s")
    srv = serve.SolveServer(max_slots=32, chunk_iters=64, tol=1e-3, min_samples=512,
                            on_result=progress, autotune_iters=2,
                            on_progress=lambda m: log("[served] " + m))
    stats = srv.run(reqs)
    out = stats.summary()
    out["requests_scale"] = scale
    out["max_iters"] = max_iters
    # the same requests alone, for the iterations each ran in the server
    sub = [r for r in stats.results if r.tag % plain_every == 0 and not r.failed]
    t_plain, att = 0.0, 0
    same = True
    for r in sub:
        q = reqs[r.tag]
        t0 = time.perf_counter()
        log(f"[served] request {r.tag} alone for {r.iterations} iterations")
        sv = F.Solver(q.ham, q.params, F.current_stream())
        sv.iterate(r.iterations)
        e = sv.estimates()
        t_plain += time.perf_counter() - t0
        att += e["total_attempts"]
        same = same and e["total_attempts"] == r.attempts and \
            abs(e["e_proj_err"] - r.e_proj_err) <= 1e-9 * max(1.0, abs(r.e_proj_err))
        sv.close()
    out["plain_subset"] = {"requests": len(sub), "plain_s": t_plain,
                           "plain_attempts_per_s": att / max(t_plain, 1e-9),
                           "served_attempts_per_s": out["attempts_per_s"],
                           "same_error_bars_as_served": bool(same)}
    return out


def variant(F, S, name, walkers, warmup, steps, **mods):
    """The 24e/30o system at the benchmark's walker target in another sampling mode
    (spin-coupled functions, a restricted space, two-word determinants): grown and
    warmed up like the headline run, then `steps` iterations timed on the graph path."""
    ham, prm, _ = S.workload("synth24e30o")
    prm.target_walkers = int(walkers)
    prm.initial_walkers = 20000
    prm.initial_shift = 40.0
    prm.shift_damping = 0.5
    for k, v in mods.items():
        setattr(prm, k, v)
    sv = F.Solver(ham, prm, F.current_stream())
    e = grow(sv, prm.target_walkers)
    sv.set_shift(e["proj_num"] / e["ref_pop"] if e["ref_pop"] else 0.0, 1)
    sv.iterate(warmup)
    ew = sv.estimates()
    sv.reserve(int(ew["table_used"] * 1.3 * 8 / 5) + 1)
    e0 = sv.estimates()
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sv.iterate(steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    e1 = sv.estimates()
    sv.close()
    att = e1["total_attempts"] - e0["total_attempts"]
    log(f"[variant] {name}: {steps} iterations in {dt:.3f} s at N_w {e1['n_walkers']}, "
        f"N_d {e1['n_dets']}")
    return {"mode": mods, "walkers": e1["n_walkers"], "dets": e1["n_dets"],
            "spawn_attempts_per_s": att / dt, "ms_per_step": dt * 1e3 / steps,
            "annihilated_dets_per_s": (e1["total_spawns"] - e0["total_spawns"]) / dt}


def copy_calibration(roctx, nbytes=1 << 30):
    """One plain streaming kernel of known traffic inside a profiled region: an elementwise
    multiply reading nbytes and writing nbytes (caches evicted first by a 2x larger fill).
    The HBM counters of this kernel calibrate FETCH_SIZE / WRITE_SIZE."""
    import torch
    x = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    y = torch.empty_like(x)
    z = torch.empty(2 * nbytes // 4, dtype=torch.float32, device="cuda").fill_(2.0)
    torch.cuda.synchronize()
    del z
    roctx.resume()
    torch.mul(x, 1.0, out=y)
    torch.cuda.synchronize()
    roctx.pause()
    del x, y


def stream_bandwidth(nbytes=1 << 30, reps=5):
    """Measured device-to-device copy bandwidth (GB/s, read + write bytes over the best
    of `reps` copies of nbytes, timed with events on the current stream)."""
    import torch
    x = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    y = torch.empty_like(x)
    best = float("inf")
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        y.copy_(x)
        b.record()
        b.synchronize()
        best = min(best, a.elapsed_time(b) * 1e-3)
    del x, y
    return 2.0 * nbytes / best / 1e9


def pmc_means(path, last=0):
    """{(kernel, counter): (mean per dispatch, dispatches)} from a rocprofv3 --pmc CSV
    tree (only the last `last` dispatches of each kernel when last > 0)."""
    import csv
    import glob
    rows = {}
    for f in sorted(glob.glob(os.path.join(path, "**", "*counter_collection.csv"), recursive=True)):
        with open(f) as fh:
            for r in csv.DictReader(fh):
                name = (r.get("Kernel_Name") or r.get("Kernel-Name") or "?").split("(")[0]
                if "fq::" in name:   # void fq::k_spawn<true> -> fq::k_spawn
                    name = name.split("<")[0].replace("void ", "")
                ctr = r.get("Counter_Name") or r.get("Counter-Name") or "?"
                v = float(r.get("Counter_Value") or r.get("Counter-Value") or "nan")
                disp = int(r.get("Dispatch_Id") or r.get("Dispatch-Id") or 0)
                rows.setdefault((name, ctr), {}).setdefault(disp, 0.0)
                rows[(name, ctr)][disp] += v
    out = {}
    for key, d in rows.items():
        vals = [d[k] for k in sorted(d)]
        if last:
            vals = vals[-last:]
        out[key] = (sum(vals) / len(vals), len(vals))
    return out


TRAFFIC_KERNELS = ("k_spawn", "k_fix", "k_bscan_up", "k_bscan_top", "k_bscan_down",
                   "k_scatter", "k_post", "k_chunk_sum")
CALIBRATION_KERNEL = "MulFunctor"


def write_traffic(fetch_dir, write_dir, last, command):
    """profiles/hbm_traffic_synth24e30o.txt from a FETCH_SIZE run and a WRITE_SIZE run of
    `bench.py --calibrate-copy`: per-dispatch means of the last `last` dispatches of each
    iteration kernel, scaled by what the same counters read for the calibration
    multiply (1 GiB read + 1 GiB written)."""
    f = pmc_means(fetch_dir, last)
    w = pmc_means(write_dir, last)
    cal_f = [v for (k, c), v in f.items() if CALIBRATION_KERNEL in k and c == "FETCH_SIZE"]
    cal_w = [v for (k, c), v in w.items() if CALIBRATION_KERNEL in k and c == "WRITE_SIZE"]
    if not cal_f or not cal_w:
        raise SystemExit("no calibration kernel in the counter runs (use --calibrate-copy)")
    fc = 1048576.0 / cal_f[0][0]
    wc = 1048576.0 / cal_w[0][0]
    lines = []
    for kern in TRAFFIC_KERNELS:
        fk = [v for (k, c), v in f.items() if k.endswith("::" + kern) and c == "FETCH_SIZE"]
        wk = [v for (k, c), v in w.items() if k.endswith("::" + kern) and c == "WRITE_SIZE"]
        if not fk or not wk:
            continue
        fb, wb = fk[0][0] * 1024.0 * fc, wk[0][0] * 1024.0 * wc
        lines.append(f"{kern}_fetch_kib_raw: {fk[0][0]:.0f}\n"
                     f"{kern}_write_kib_raw: {wk[0][0]:.0f}\n"
                     f"{kern}_bytes_per_launch: {fb + wb:.6g}\n")
        print(f"{kern}: {(fb + wb) / 1e9:.4f} GB per launch (read {fb / 1e9:.4f}, "
              f"written {wb / 1e9:.4f})")
    with open(os.path.join(PROFILES, "hbm_traffic_synth24e30o.txt"), "w") as out:
        out.write("# HBM traffic per launch of the iteration kernels, from rocprofv3 FETCH_SIZE\n"
                  f"# and WRITE_SIZE (KiB per dispatch, mean of the last {last} dispatches of\n"
                  "# each kernel = the profiling window's iterations), each scaled by the\n"
                  "# counter's reading for an elementwise multiply that reads and writes 1 GiB\n"
                  "# (caches evicted first) in the same run.\n"
                  "# Workload: bench.py on the synthetic 24e/30o band system at >= 1e8 walkers.\n"
                  "# Commands (repository root, one MI355X):\n")
        for c in command:
            out.write(f"#   {c}\n")
        out.write(f"kernels_sha256: {kernel_source_hash()}\n"
                  f"fetch_calibration: {fc:.6f}\n"
                  f"write_calibration: {wc:.6f}\n")
        for ln in lines:
            out.write(ln)


def write_valu(counter_dir, last, attempts_per_launch, dets_per_launch, command):
    """profiles/k_spawn_valu_synth24e30o.txt and profiles/k_post_valu_synth24e30o.txt:
    issued VALU lane-operations (SQ_INSTS_VALU x 64) per attempt of k_spawn and per
    determinant of k_post, with the other instruction counters and the LDS
    bank-conflict share."""
    m = pmc_means(counter_dir, last)
    for kern, unit, units in (("k_spawn", "attempt", attempts_per_launch),
                              ("k_post", "det", dets_per_launch)):
        def get(c):
            v = [x for (k, cc), x in m.items() if k.endswith("::" + kern) and cc == c]
            return v[0][0] if v else float("nan")
        valu = get("SQ_INSTS_VALU")
        with open(os.path.join(PROFILES, f"{kern}_valu_synth24e30o.txt"), "w") as out:
            out.write(f"# {kern} instruction counters (rocprofv3 --pmc, per dispatch, mean of the\n"
                      f"# last {last} dispatches = the profiling window's iterations); per {unit}:\n"
                      f"# SQ_INSTS_VALU x 64 / {unit}s per launch.\n"
                      "# Commands (repository root, one MI355X):\n")
            for c in command:
                out.write(f"#   {c}\n")
            out.write(f"kernels_sha256: {kernel_source_hash()}\n"
                      f"{unit}s_per_launch: {units:.6g}\n")
            for c in ("SQ_INSTS_VALU", "SQ_INSTS_SALU", "SQ_INSTS_LDS", "SQ_INSTS_VMEM_RD",
                      "SQ_INSTS_VMEM_WR", "SQ_ACTIVE_INST_LDS", "SQ_LDS_BANK_CONFLICT",
                      "SQ_WAVE_CYCLES"):
                out.write(f"{c}: {get(c):.6g}\n")
            out.write(f"issued_lane_ops_per_{unit}: {valu * 64.0 / units:.4g}\n"
                      f"salu_per_{unit}: {get('SQ_INSTS_SALU') * 64.0 / units:.4g}\n"
                      f"lds_bank_conflict_share: "
                      f"{get('SQ_LDS_BANK_CONFLICT') / max(get('SQ_ACTIVE_INST_LDS'), 1.0):.4g}\n")
        print(f"{kern}: {valu * 64.0 / units:.1f} issued lane-ops per {unit}")


def pmc_summary(path, last=0):
    """Mean of each counter per dispatch, per kernel, from a rocprofv3 --pmc CSV tree
    (only the last `last` dispatches of each kernel when last > 0)."""
    m = pmc_means(path, last)
    print(f"# rocprofv3 --pmc summary of {path}; per-dispatch means"
          + (f" over the last {last} dispatches of each kernel" if last else ""))
    for (name, ctr), (v, n) in sorted(m.items()):
        print(f"{name:44s} {ctr:22s} dispatches {n:5d} mean {v:.6g}")


def trace_summary(path):
    """Per-kernel launches, mean and total duration from a rocprofv3 --kernel-trace
    --stats CSV tree (its *kernel_stats.csv)."""
    import csv
    import glob
    files = sorted(glob.glob(os.path.join(path, "**", "*kernel_stats.csv"), recursive=True))
    if not files:
        raise SystemExit(f"no kernel_stats.csv under {path}")
    rows = list(csv.DictReader(open(files[0])))
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    print(f"# kernel statistics of {files[0]}")
    print(f"{'kernel':34s} {'calls':>6s} {'mean_us':>10s} {'total_ms':>10s} {'pct':>6s}")
    for r in rows:
        name = r["Name"].split("(")[0].replace("fq::", "").replace("void ", "")[:34]
        print(f"{name:34s} {int(r['Calls']):6d} {float(r['AverageNs']) / 1e3:10.1f} "
              f"{float(r['TotalDurationNs']) / 1e6:10.3f} {float(r['Percentage']):6.2f}")


def main():
    if len(sys.argv) >= 3 and sys.argv[1] == "--trace-summary":
        trace_summary(sys.argv[2])
        return
    if len(sys.argv) >= 3 and sys.argv[1] == "--pmc-summary":
        pmc_summary(sys.argv[2], int(sys.argv[3]) if len(sys.argv) > 3 else 0)
        return
    if len(sys.argv) >= 5 and sys.argv[1] == "--write-traffic":
        # --write-traffic FETCH_DIR WRITE_DIR LAST [command lines ...]
        write_traffic(sys.argv[2], sys.argv[3], int(sys.argv[4]), sys.argv[5:])
        return
    if len(sys.argv) >= 6 and sys.argv[1] == "--write-valu":
        # --write-valu COUNTER_DIR LAST ATTEMPTS_PER_LAUNCH DETS_PER_LAUNCH [command lines ...]
        write_valu(sys.argv[2], int(sys.argv[3]), float(sys.argv[4]), float(sys.argv[5]),
                   sys.argv[6:])
        return
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200, help="timed iterations (graph path)")
    ap.add_argument("--warmup", type=int, default=300,
                    help="iterations after the growth stage with the shift varying")
    ap.add_argument("--profile-steps", type=int, default=20,
                    help="iterations of the profiling-mode window")
    ap.add_argument("--walkers", type=float, default=1e8)
    ap.add_argument("--growth-shift", type=float, default=40.0)
    ap.add_argument("--shift-damping", type=float, default=0.5)
    ap.add_argument("--initial-walkers", type=int, default=20000)
    ap.add_argument("--cpu-attempts", type=float, default=2.5e7)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--batched-scale", type=float, default=1.0)
    ap.add_argument("--batched-iters", type=int, default=2000)
    ap.add_argument("--no-served", action="store_true")
    ap.add_argument("--served-requests", type=int, default=200)
    ap.add_argument("--served-scale", type=float, default=1.0,
                    help="walker targets of the served requests, times 1e4..1e6")
    ap.add_argument("--served-max-iters", type=int, default=4000,
                    help="iteration cap per request (the full serving workload uses 20000)")
    ap.add_argument("--served-only", action="store_true",
                    help="run only the serving leg and print its summary")
    ap.add_argument("--served-plain-every", type=int, default=25,
                    help="run every n-th served request alone for comparison")
    ap.add_argument("--no-variants", action="store_true",
                    help="skip the spin-coupled and restricted-space runs of the workload")
    ap.add_argument("--det-words", type=int, default=0,
                    help="64-bit words per determinant for the headline run: 0 as needed (one "
                         "for this system), 2 to time the two-word kernels on it")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="add a 1 GiB elementwise multiply in its own profiled region")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    import torch
    from paper_1305_6981_amd import fciqmc as F
    from paper_1305_6981_amd import systems as S
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    roctx = Roctx()
    if args.served_only:
        print(json.dumps({"served": served(F, S, args.served_requests, args.served_scale,
                                           args.served_max_iters, args.served_plain_every)}),
              flush=True)
        return

    ham, prm, _ = S.workload("synth24e30o")
    target = int(args.walkers)
    prm.target_walkers = target
    prm.initial_walkers = args.initial_walkers
    prm.initial_shift = args.growth_shift
    prm.shift_damping = args.shift_damping
    prm.det_words = args.det_words
    log(f"[bench] growth stage to {target} walkers at shift +{args.growth_shift}")
    t_g = time.perf_counter()
    sv = F.Solver(ham, prm, F.current_stream())
    e = grow(sv, target)
    s_est = e["proj_num"] / e["ref_pop"] if e["ref_pop"] else 0.0
    sv.set_shift(s_est, 1)
    log(f"[bench] grown in {time.perf_counter() - t_g:.1f} s: N_w {e['n_walkers']} N_d "
        f"{e['n_dets']} C0 {e['ref_pop']}; shift set to E_proj - E0 = {s_est:.4f}")
    done = 0
    while done < args.warmup:
        n = min(100, args.warmup - done)
        sv.iterate(n)
        done += n
        ew = sv.estimates()
        log(f"[warm-up] iter {ew['iteration']} N_w {ew['n_walkers']} N_d {ew['n_dets']} "
            f"shift {ew['shift']:.4f}")
    # Size the table for the timed and profiled windows: the entries grow by at most
    # the largest increase of the last warm-up iterations, with 50 % slack; the
    # library re-buckets a system whose mean bucket fill passes 5/8, so the capacity
    # is set above 8/5 of the largest expected entry count.
    ew = sv.estimates()
    tail = history(F, sv.h, ew["iteration"] - 49, 50)
    gu = max([b["entries"] - a["entries"] for a, b in zip(tail, tail[1:])] + [0])
    n_after = args.steps + args.profile_steps + 8
    entries_max = tail[-1]["entries"] + 1.5 * gu * n_after
    sv.reserve(int(entries_max * 8 / 5 * 1.02) + 1)
    e0 = sv.estimates()
    log(f"[bench] warm-up done; {e0['table_slots']} slots for {tail[-1]['entries']} entries "
        f"(+{gu} per iteration at most); N_w {e0['n_walkers']} N_d {e0['n_dets']}")

    # timed window: the production path (graph launches)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sv.iterate(args.steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    e1 = sv.estimates()
    dt = t1 - t0
    attempts = e1["total_attempts"] - e0["total_attempts"]
    spawns = e1["total_spawns"] - e0["total_spawns"]
    win = history(F, sv.h, e0["iteration"] + 1, args.steps)
    nw = [r["n_walkers"] for r in win]
    rebucketed = e1["table_slots"] != e0["table_slots"] or e1["spills"] != e0["spills"]
    log(f"[bench] timed {args.steps} iterations in {dt:.3f} s: N_w {min(nw)} .. {max(nw)}, "
        f"N_d {e1['n_dets']}, attempts {attempts}, spawns {spawns}"
        + (" (re-bucketed inside the window)" if rebucketed else ""))

    # profiling window: direct launches bracketed by events, per-kernel-group times (and
    # the region a rocprofv3 kernel trace with --selected-regions records)
    F.fciqmc_set_profiling(sv.h, 1)
    ep0 = sv.estimates()
    torch.cuda.synchronize()
    roctx.resume()
    sv.iterate(args.profile_steps)
    torch.cuda.synchronize()
    roctx.pause()
    ep1 = sv.estimates()
    kms, kcnt = F.fciqmc_kernel_times(sv.h)
    F.fciqmc_set_profiling(sv.h, 0)
    if args.calibrate_copy:
        copy_calibration(roctx)
    prec = history(F, sv.h, ep0["iteration"] + 1, args.profile_steps)
    grp_ms = {g: float(kms[i] / max(kcnt[i], 1)) for i, g in enumerate(GROUPS)}
    prof_ms = (sum(kms) / max(kcnt[2], 1))
    att_launch = float(np.mean([r["attempts"] for r in prec]))
    b_group, b_post = method_bytes(prec, ep0["n_dets"])
    copy_gbs = stream_bandwidth()

    spawn_ms = grp_ms["spawn"]
    achieved_ops = OPS_PER_ATTEMPT * att_launch / (spawn_ms * 1e-3) / 1e12
    issued = issued_ops_per("k_spawn", "attempt")
    roofline = {"bound": "alu", "kernel": "k_spawn", "achieved": achieved_ops,
                "peak": ALU_PEAK_TOPS, "unit": "TOP/s", "frac": achieved_ops / ALU_PEAK_TOPS,
                "traffic": measured_traffic(GROUP_KERNELS["spawn"]),
                "ops_per_attempt": OPS_PER_ATTEMPT, "attempts_per_launch": att_launch,
                "avg_ms": spawn_ms,
                "issued_lane_ops_per_attempt": issued,
                "issue_frac": (issued * att_launch / (spawn_ms * 1e-3) / 1e12 / ALU_PEAK_TOPS
                               if issued else None)}
    ann_ms = grp_ms["annihilation"]
    ach = b_group / (ann_ms * 1e-3) / 1e9
    roofline_ann = {"bound": "hbm", "kernel": "annihilation (k_fix, k_bscan_*, k_scatter, k_post)",
                    "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": ach / HBM_PEAK_GBS,
                    "traffic": measured_traffic(GROUP_KERNELS["annihilation"]),
                    "algorithmic_bytes": b_group, "k_post_algorithmic_bytes": b_post,
                    "avg_ms": ann_ms, "measured_copy_gbs": copy_gbs,
                    "frac_of_measured_copy": ach / copy_gbs,
                    "k_post_issued_lane_ops_per_det": issued_ops_per("k_post", "det")}

    if F.fciqmc_det_words(sv.h) != 1:   # the committed counters describe the one-word kernels
        roofline.update(traffic=None, issued_lane_ops_per_attempt=None, issue_frac=None)
        roofline_ann.update(traffic=None, k_post_issued_lane_ops_per_det=None)
    mean = lambda k: float(np.mean([r[k] for r in win]))  # noqa: E731
    out = {
        "metric": "spawn attempts/s + annihilated dets/s at 1e8 walkers; batched vs plain",
        "value": attempts / dt,
        "unit": "spawn attempts/s",
        "annihilated_dets_per_s": spawns / dt,
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": dt * 1e3 / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": "synthetic 24e/30o with a 12-orbital band at +-0.2 Ha, initiator "
                               f"n_a=3, tau=5e-4, {min(nw)}..{max(nw)} walkers on "
                               f"{int(mean('n_dets'))} dets (window means)",
                   "walkers_min": min(nw), "walkers_max": max(nw),
                   "dets_mean": mean("n_dets"), "spawns_per_iteration": mean("spawns"),
                   "merged_per_iteration": mean("merged"), "born_per_iteration": mean("born"),
                   "table_slots": e1["table_slots"], "rebucketed_in_window": rebucketed,
                   "path": "graph launches (production path)", "parallelism": "1 GPU",
                   "det_words": F.fciqmc_det_words(sv.h)},
        "profiling_window": {"iterations": args.profile_steps, "ms_per_step": prof_ms,
                             "group_ms": grp_ms},
        "roofline": roofline,
        "roofline_annihilation": roofline_ann,
    }
    if not args.no_cpu_baseline:
        log("[bench] CPU oracle baseline")
        det, pop, _ = sv.walkers()
        out["cpu_baseline"] = cpu_baseline(ham, prm, det, pop, ep1, args.cpu_attempts)
        out["gpu_over_oracle"] = out["value"] / out["cpu_baseline"]["value"]
        del det, pop
    sv.close()
    if not args.no_variants:
        log("[bench] sampling variants of the workload")
        out["variants"] = {
            "spin_coupled_even_S": variant(F, S, "spin-coupled functions", args.walkers, 150, 50,
                                           hphf=1),
            "cisdtq": variant(F, S, "excitation level <= 4", args.walkers, 150, 50,
                              space=S.SPACE_EXCITATION, max_excitation=4),
            # the two-word kernels (determinants of 65-128 spin orbitals) on the same
            # system and trajectory: the cost of the second word
            "two_word_determinants": variant(F, S, "two-word determinants", args.walkers, 150,
                                             50, det_words=2),
        }
    if not args.no_batched:
        log("[bench] batched vs plain (64 systems)")
        out["batched"] = batched_vs_plain(F, S, args.batched_iters, args.batched_scale,
                                          min(400, args.batched_iters // 2))
    if not args.no_served:
        log("[bench] served Poisson stream")
        out["served"] = served(F, S, args.served_requests, args.served_scale,
                               args.served_max_iters, args.served_plain_every)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
