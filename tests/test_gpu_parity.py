"""HIP path vs the CPU oracle, through the C ABI.

Walker lists (determinant, population, initiator flag) must be bit-identical
after every checked iteration; the shift is compared exactly (both sides use
the same operation order) and the projected-energy numerator to 1e-10
relative (its summation order differs)."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1305_6981_amd import fciqmc as F
from paper_1305_6981_amd import systems as S

pytestmark = pytest.mark.gpu


def _stream():
    import torch
    assert torch.cuda.is_available()
    return F.current_stream()


def _same_lists(gpu, ref, tag):
    dg, pg, fg = gpu.walkers()
    do, po, fo = ref.walkers()
    assert len(dg) == len(do), (tag, len(dg), len(do))
    assert np.array_equal(dg, do), tag
    assert np.array_equal(pg, po), tag
    assert np.array_equal(fg, fo), tag


def _same_estimates(eg, eo, tag):
    for k in ("iteration", "n_walkers", "n_dets", "ref_pop", "attempts", "spawns", "merged",
              "aborted", "born", "total_attempts", "total_spawns", "shift_varying", "n_samples"):
        assert eg[k] == eo[k], (tag, k, eg[k], eo[k])
    assert eg["shift"] == eo["shift"], (tag, eg["shift"], eo["shift"])
    assert eg["e_ref"] == eo["e_ref"] and eg["p_double"] == eo["p_double"]
    assert abs(eg["proj_num"] - eo["proj_num"]) <= 1e-10 * max(1.0, abs(eo["proj_num"])), tag


def _run_pair(ham, prm, blocks, per_block, tag):
    print(f"[gpu] {tag}: {ham.name} target={prm.target_walkers} blocks={blocks}x{per_block}", flush=True)
    gpu = F.Solver(ham, prm, _stream())
    ref = O.Oracle(ham, prm)
    _same_estimates(gpu.estimates() | {"attempts": 0, "spawns": 0, "merged": 0, "aborted": 0,
                                       "total_attempts": 0, "total_spawns": 0, "proj_num": 0.0,
                                       "iteration": 0},
                    ref.estimates() | {"proj_num": 0.0}, tag + "/init")
    for b in range(blocks):
        gpu.iterate(per_block)
        ref.iterate(per_block)
        _same_lists(gpu, ref, f"{tag}/block{b}")
        _same_estimates(gpu.estimates(), ref.estimates(), f"{tag}/block{b}")
    eg = gpu.estimates()
    gpu.close()
    return eg


def test_hubbard8_plain_bit_exact():
    ham, prm, _ = S.workload("hubbard8")
    prm.avg_start = 20
    eg = _run_pair(ham, prm, blocks=8, per_block=50, tag="hubbard8")
    assert eg["n_walkers"] > 1000


def test_estimator_averages_and_error_bars_match():
    """Blocking means and error bars of E_proj and the shift agree with the oracle's
    (the series are identical up to the summation order of the numerator)."""
    ham, prm, _ = S.workload("hubbard8")
    prm.avg_start = 0
    print("[gpu] averages", flush=True)
    gpu = F.Solver(ham, prm, _stream())
    ref = O.Oracle(ham, prm)
    gpu.iterate(700)
    ref.iterate(700)
    eg, eo = gpu.estimates(), ref.estimates()
    assert eg["n_samples"] == eo["n_samples"] and eg["n_samples"] > 300
    for k in ("e_proj_mean", "e_proj_err", "shift_mean", "shift_err"):
        assert np.isfinite(eo[k]), k
        assert abs(eg[k] - eo[k]) <= 1e-10 * max(1.0, abs(eo[k])), (k, eg[k], eo[k])
    gpu.close()


def test_synthetic_initiator_bit_exact():
    ham, prm, _ = S.workload("synth10e20o", scale=2e-4)
    prm.initial_walkers = 500
    prm.initial_shift = 0.5
    _run_pair(ham, prm, blocks=5, per_block=30, tag="synth10e20o")


def test_band_24e30o_bit_exact():
    # 60 spin orbitals: exercises the high bits of the 64-bit determinant.
    ham, prm, _ = S.workload("synth24e30o", scale=2e-5)
    prm.initial_walkers = 300
    prm.initial_shift = 1.0
    prm.tau = 2e-3
    _run_pair(ham, prm, blocks=4, per_block=20, tag="synth24e30o")


def test_point_group_labels_bit_exact():
    irr = np.array([0, 1, 2, 3, 0, 1, 2, 3, 0, 1, 4, 5], np.uint8)
    ham = S.synthetic_molecule(12, 3, 3, 77, irreps=irr)
    prm = S.Params(tau=5e-3, initiator_threshold=2, target_walkers=3000, initial_walkers=200,
                   initial_shift=0.3, seed=21)
    _run_pair(ham, prm, blocks=4, per_block=25, tag="irreps")


def test_forced_table_growth_is_result_neutral():
    # A tiny initial table forces the grow-and-redo path many times.
    ham, prm, _ = S.workload("hubbard8")
    prm.det_capacity = 4096
    prm.target_walkers = 30000
    _run_pair(ham, prm, blocks=3, per_block=60, tag="growth")


def test_table_stays_bounded_under_turnover():
    """A population that has levelled off keeps visiting new determinants; their
    vacated slots fill the table, and the rehash that follows must compact it
    rather than grow it without bound. The trajectory stays the oracle's.

    Bound: a rehash grows only when 2(live + 8g) exceeds the capacity, to at most
    1.5 times that, where g (new keys per iteration, 25 % slack, at least 256) is
    at most 1.25 x the spawns of one iteration."""
    ham = S.hubbard_ring(12, 4.0)
    prm = S.Params(tau=0.01, initiator_threshold=3, target_walkers=4000, initial_walkers=2000,
                   seed=3, shift_update_every=1, det_capacity=4096)
    print("[gpu] turnover hubbard12", flush=True)
    gpu = F.Solver(ham, prm, _stream())
    ref = O.Oracle(ham, prm)
    max_nd = max_sp = 0
    for b in range(8):
        for _ in range(5):
            gpu.iterate(15)
            e = gpu.estimates()
            max_nd, max_sp = max(max_nd, e["n_dets"]), max(max_sp, e["spawns"])
            # slots holding keys: at least the occupied ones, within the table
            assert e["n_dets"] <= e["table_used"] <= e["table_slots"]
        ref.iterate(75)
        _same_lists(gpu, ref, f"turnover{b}")
        _same_estimates(gpu.estimates(), ref.estimates(), f"turnover{b}")
    slots = gpu.estimates()["table_slots"]
    g = max(256, 1.25 * 1.5 * max_sp + 1)      # spawns sampled every 15 iterations: 50 % margin
    bound = 1.5 * 2 * (max_nd + 1 + 8 * g) + 4096
    print(f"[gpu] turnover: slots={slots} max_nd={max_nd} max_spawns={max_sp} bound={bound:.0f}",
          flush=True)
    assert e["total_spawns"] > 5 * slots, "too little turnover to exercise compaction"
    assert slots <= bound
    gpu.close()


def test_reserve_is_result_neutral():
    """Growing the table on request (odd sizes, mid-run, also a no-op request) changes
    nothing in the trajectory."""
    ham, prm, _ = S.workload("synth10e20o", scale=2e-4)
    prm.initial_walkers, prm.initial_shift = 400, 0.5
    print("[gpu] reserve", flush=True)
    gpu = F.Solver(ham, prm, _stream())
    ref = O.Oracle(ham, prm)
    for b, slots in enumerate([0, 12345, 100000, 50000, 4096 * 37]):
        gpu.reserve(slots)
        assert gpu.estimates()["table_slots"] >= slots
        assert gpu.estimates()["table_slots"] % 4096 == 0
        gpu.iterate(9)
        ref.iterate(9)
        _same_lists(gpu, ref, f"reserve{b}")
        _same_estimates(gpu.estimates(), ref.estimates(), f"reserve{b}")
    with pytest.raises(F.FciqmcError):
        gpu.reserve(-1)
    gpu.close()


def test_snapshot_restart_matches_oracle():
    ham, prm, _ = S.workload("synth10e20o", scale=2e-4)
    prm.initial_walkers = 400
    prm.initial_shift = 0.5
    gpu = F.Solver(ham, prm, _stream())
    gpu.iterate(40)
    det, pop, _ = gpu.walkers()
    e = gpu.estimates()
    ref = O.Oracle(ham, prm)
    ref.load_walkers(det, pop, iteration=e["iteration"], shift=e["shift"], n_prev=e["n_prev"],
                     varying=e["shift_varying"], n_var=e["n_var"])
    gpu.load_walkers(det, pop, iteration=e["iteration"], shift=e["shift"], n_prev=e["n_prev"],
                     varying=e["shift_varying"], n_var=e["n_var"])
    for b in range(3):
        gpu.iterate(7)
        ref.iterate(7)
        _same_lists(gpu, ref, f"restart{b}")
    gpu.close()


def test_zero_iterations_and_errors():
    ham, prm, _ = S.workload("hubbard8")
    gpu = F.Solver(ham, prm, _stream())
    gpu.iterate(0)
    d, p, f = gpu.walkers()
    assert d.tolist() == [ham.ref_det] and p.tolist() == [prm.initial_walkers]
    with pytest.raises(F.FciqmcError):
        gpu.load_walkers(np.array([ham.ref_det, ham.ref_det], np.uint64), np.array([1, 2], np.int32))
    with pytest.raises(F.FciqmcError):
        gpu.load_walkers(np.array([0b11], np.uint64), np.array([1], np.int32))
    gpu.close()
    bad = S.Params(tau=-1.0)
    with pytest.raises(F.FciqmcError):
        F.Solver(ham, bad, _stream())


def test_launch_shape_and_autotune_are_result_neutral():
    ham, prm, _ = S.workload("synth24e30o", scale=2e-5)
    prm.initial_walkers, prm.initial_shift, prm.tau = 300, 1.0, 2e-3
    print("[gpu] launch shapes", flush=True)
    runs = []
    for shape in [(64, 256, 16), (4096, 4096, 2048), None]:
        sv = F.Solver(ham, prm, _stream())
        if shape is None:
            F.fciqmc_autotune(sv.h, 1)        # 16 trial launches of one iteration each
            sv.iterate(40 - sv.estimates()["iteration"])
        else:
            F.fciqmc_set_launch(sv.h, *shape)
            sv.iterate(40)
        assert sv.estimates()["iteration"] == 40
        runs.append(sv.walkers())
        sv.close()
    ref = O.Oracle(ham, prm)
    ref.iterate(40)
    do, po, _ = ref.walkers()
    for d, p, _ in runs:
        assert np.array_equal(d, do) and np.array_equal(p, po)
