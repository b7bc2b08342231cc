"""Parity at the benchmark's full size and launch shape.

The 24e/30o band system (initiator n_a = 3, tau = 5e-4) is grown on the GPU to
1e8 walkers exactly as bench.py grows it, with the default launch shape. From
that snapshot the GPU and the oracle each run one iteration; the oracle spreads
the determinants over one virtual process per host thread (Sec. 4.1; the
result does not depend on the process count, see test_oracle_processes.py).
Walker lists must be bit-identical, the integer statistics and the shift
identical, and the projected-energy numerator equal to 1e-10 relative."""
import os
import time

import numpy as np
import pytest

from oracle import oracle as O
from paper_1305_6981_amd import fciqmc as F
from paper_1305_6981_amd import systems as S

pytestmark = [pytest.mark.gpu, pytest.mark.slow]


def test_full_size_iteration_matches_oracle():
    import torch
    assert torch.cuda.is_available()
    ham, prm, _ = S.workload("synth24e30o")
    target = 100_000_000
    prm.target_walkers = target
    prm.initial_walkers = 20000
    prm.initial_shift = 40.0
    t0 = time.perf_counter()
    sv = F.Solver(ham, prm, F.current_stream())
    while True:
        e = sv.estimates()
        if e["n_walkers"] >= target:
            break
        sv.iterate(20 if e["n_walkers"] * 4 < target else 2)
        assert e["iteration"] < 2000, "growth stage did not reach the walker target"
    sv.set_shift(e["proj_num"] / e["ref_pop"], 1)
    e = sv.estimates()
    det, pop, _ = sv.walkers()
    print(f"[gpu] full size: {e['n_walkers']} walkers on {len(det)} determinants after "
          f"{e['iteration']} iterations ({time.perf_counter() - t0:.1f} s)", flush=True)
    assert e["n_walkers"] >= target and len(det) > 10_000_000

    threads = max(1, min(16, len(os.sched_getaffinity(0))))
    ref = O.Oracle(ham, prm, n_procs=threads, n_threads=threads)
    ref.load_walkers(det, pop, iteration=e["iteration"], shift=e["shift"], n_prev=e["n_prev"],
                     varying=e["shift_varying"], n_var=e["n_var"])
    del det, pop
    t1 = time.perf_counter()
    ref.iterate(1)
    print(f"[gpu] oracle iteration on {threads} threads: {time.perf_counter() - t1:.1f} s",
          flush=True)
    sv.iterate(1)

    eg, eo = sv.estimates(), ref.estimates()
    for k in ("iteration", "n_walkers", "n_dets", "ref_pop", "attempts", "spawns", "merged",
              "aborted", "born", "shift_varying", "n_prev", "n_var"):
        assert eg[k] == eo[k], (k, eg[k], eo[k])
    assert eg["shift"] == eo["shift"]
    assert abs(eg["proj_num"] - eo["proj_num"]) <= 1e-10 * abs(eo["proj_num"])
    dg, pg, fg = sv.walkers()
    do, po, fo = ref.walkers()
    assert len(dg) == len(do)
    assert np.array_equal(dg, do)
    assert np.array_equal(pg, po)
    assert np.array_equal(fg, fo)
    print(f"[gpu] full size: {len(dg)} determinants identical; total {time.perf_counter() - t0:.1f} s",
          flush=True)
    sv.close()
    ref.close()
