"""Parity at full size, in the launch configuration the benchmark times.

Config 3: the 24e/30o band system (initiator n_a = 3, tau = 5e-4) is grown on the
GPU to 1e8 walkers and warmed up exactly as bench.py does it (shift set to the
projected-energy estimate, damping 0.5, 300 iterations), with the default launch
shape. Config 2: the 10e/20o system (n_a = 3, tau = 1e-3) is grown to 1e7
walkers. From each snapshot the GPU runs three iterations in one call (one graph
launch plus the sampled last iteration, so the chunk sums that the annihilation
pass writes for the next iteration are used twice) and the oracle runs the same
three iterations with the determinants spread over one virtual process per host
thread (Sec. 4.1; the result does not depend on the process count, see
test_oracle_processes.py). Walker lists must be bit-identical, the integer
statistics and the shift identical, and the projected-energy numerator equal
to 1e-10 relative. For config 3 the same snapshot also runs through the
two-word kernels (determinants of more than 64 spin orbitals, forced here),
which must give the one-word run's lists and statistics exactly."""
import os
import time

import numpy as np
import pytest

from oracle import oracle as O
from paper_1305_6981_amd import fciqmc as F
from paper_1305_6981_amd import systems as S

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

K = 3


def _grow(sv, target, limit):
    while True:
        e = sv.estimates()
        if e["n_walkers"] >= target:
            return e
        sv.iterate(20 if e["n_walkers"] * 4 < target else 2)
        assert e["iteration"] < limit, "growth stage did not reach the walker target"


def _compare_k_iterations(ham, prm, sv, tag, two_words=False):
    e = sv.estimates()
    det, pop, _ = sv.walkers()
    sv2 = None
    if two_words:
        import copy
        p2 = copy.copy(prm)
        p2.det_words = 2
        sv2 = F.Solver(ham, p2, F.current_stream())
        sv2.reserve(e["table_slots"])
        sv2.load_walkers(det, pop, iteration=e["iteration"], shift=e["shift"],
                         n_prev=e["n_prev"], varying=e["shift_varying"], n_var=e["n_var"])
        print(f"[gpu] {tag}: snapshot loaded into the two-word kernels", flush=True)
    print(f"[gpu] {tag}: snapshot of {e['n_walkers']} walkers on {len(det)} determinants at "
          f"iteration {e['iteration']}", flush=True)
    threads = max(1, min(16, len(os.sched_getaffinity(0))))
    ref = O.Oracle(ham, prm, n_procs=threads, n_threads=threads)
    ref.load_walkers(det, pop, iteration=e["iteration"], shift=e["shift"], n_prev=e["n_prev"],
                     varying=e["shift_varying"], n_var=e["n_var"])
    del det, pop
    t1 = time.perf_counter()
    sv.iterate(K)
    hist = F.fciqmc_history(sv.h, 0, e["iteration"] + 1, K)
    for k in range(K):
        ref.iterate(1)
        eo = ref.estimates()
        r = hist[k]
        for f in ("iteration", "n_walkers", "n_dets", "ref_pop", "attempts", "spawns", "merged",
                  "aborted", "born"):
            assert r[f] == eo[f], (tag, k, f, r[f], eo[f])
        assert r["shift"] == eo["shift"], (tag, k)
        assert abs(r["proj_num"] - eo["proj_num"]) <= 1e-10 * abs(eo["proj_num"]), (tag, k)
        print(f"[gpu] {tag}: iteration {r['iteration']} statistics identical "
              f"({r['spawns']} spawns, {r['born']} new determinants)", flush=True)
    print(f"[gpu] {tag}: oracle {K} iterations on {threads} threads in "
          f"{time.perf_counter() - t1:.1f} s", flush=True)
    eg = sv.estimates()
    assert eg["shift_varying"] == eo["shift_varying"] and eg["n_prev"] == eo["n_prev"]
    dg, pg, fg = sv.walkers()
    do, po, fo = ref.walkers()
    assert len(dg) == len(do)
    assert np.array_equal(dg, do)
    assert np.array_equal(pg, po)
    assert np.array_equal(fg, fo)
    print(f"[gpu] {tag}: {len(dg)} determinants identical after {K} iterations", flush=True)
    ref.close()
    if sv2 is not None:
        sv2.iterate(K)
        h2 = F.fciqmc_history(sv2.h, 0, e["iteration"] + 1, K)
        for k in range(K):
            for f in ("iteration", "n_walkers", "n_dets", "ref_pop", "attempts", "spawns",
                      "merged", "aborted", "born", "shift"):
                assert h2[k][f] == hist[k][f], (tag, "two words", k, f)
        d2, p2_, f2 = sv2.walkers()
        assert d2.shape == (len(dg), 2) and np.array_equal(d2[:, 0], dg) and not d2[:, 1].any()
        assert np.array_equal(p2_, pg) and np.array_equal(f2, fg)
        print(f"[gpu] {tag}: two-word kernels identical after {K} iterations", flush=True)
        sv2.close()


def test_full_size_config3_matches_oracle():
    import torch
    assert torch.cuda.is_available()
    ham, prm, _ = S.workload("synth24e30o")
    target = 100_000_000
    prm.target_walkers = target
    prm.initial_walkers = 20000
    prm.initial_shift = 40.0
    prm.shift_damping = 0.5
    t0 = time.perf_counter()
    sv = F.Solver(ham, prm, F.current_stream())
    e = _grow(sv, target, 2000)
    sv.set_shift(e["proj_num"] / e["ref_pop"], 1)
    sv.iterate(300)
    print(f"[gpu] config 3 grown and warmed up in {time.perf_counter() - t0:.1f} s", flush=True)
    assert sv.estimates()["n_walkers"] >= target
    _compare_k_iterations(ham, prm, sv, "config 3", two_words=True)
    sv.close()


def test_full_size_config2_matches_oracle():
    ham, prm, _ = S.workload("synth10e20o")
    prm.initial_walkers = 10000
    prm.initial_shift = 5.0
    t0 = time.perf_counter()
    sv = F.Solver(ham, prm, F.current_stream())
    e = _grow(sv, prm.target_walkers, 20000)
    sv.set_shift(e["proj_num"] / e["ref_pop"], 1)
    sv.iterate(20)
    print(f"[gpu] config 2 grown in {time.perf_counter() - t0:.1f} s", flush=True)
    assert sv.estimates()["n_walkers"] >= 0.5 * prm.target_walkers
    _compare_k_iterations(ham, prm, sv, "config 2")
    sv.close()
