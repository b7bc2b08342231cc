"""Rarely taken paths of the HIP implementation, forced and checked bit for bit
against the oracle through the C ABI: the grow-and-redo path of a table that
overflows inside an iteration, spawn tiles located by search instead of the
tile map, large tiles, a reference population of zero, death that crosses
zero."""
import numpy as np
import pytest

from oracle import ed
from oracle import oracle as O
from paper_1305_6981_amd import fciqmc as F
from paper_1305_6981_amd import systems as S

from test_gpu_parity import _same_estimates, _same_lists, _stream

pytestmark = pytest.mark.gpu


def test_overflows_inside_iterations_are_handled_bit_exactly():
    """With the planner off, a 4096-entry main list and a 512-record spawn buffer
    overflow during iterations: an iteration whose records do not fit is
    abandoned and re-run after the buffer grows, and new determinants that do
    not fit their bucket complete the iteration through the spill list before
    the list is re-bucketed."""
    ham, prm, _ = S.workload("hubbard8")
    prm.det_capacity = 4096
    prm.target_walkers = 30000
    print("[gpu] overflow paths: hubbard8, planner off", flush=True)
    gpu = F.Solver(ham, prm, _stream())
    F.fciqmc_set_test_options(gpu.h, 0, -1, 512)
    ref = O.Oracle(ham, prm)
    for b in range(4):
        gpu.iterate(40)
        ref.iterate(40)
        _same_lists(gpu, ref, f"overflow{b}")
        _same_estimates(gpu.estimates(), ref.estimates(), f"overflow{b}")
    e = gpu.estimates()
    print(f"[gpu] overflow paths: {e['redos']} iterations re-run, {e['spills']} spilled, "
          f"{e['table_slots']} slots", flush=True)
    assert e["redos"] > 0 and e["spills"] > 0
    gpu.close()


@pytest.mark.parametrize("limit", [0, 37])
def test_tile_search_without_map(limit):
    """Spawn tiles beyond the tile map (none at all, or all but the first 37)
    find their chunk by the wavefront search over the chunk offsets."""
    ham, prm, _ = S.workload("synth24e30o", scale=2e-5)
    prm.initial_walkers, prm.initial_shift, prm.tau = 300, 1.0, 2e-3
    print(f"[gpu] tile search: map limit {limit}", flush=True)
    gpu = F.Solver(ham, prm, _stream())
    F.fciqmc_set_test_options(gpu.h, 1, limit, 0)
    F.fciqmc_set_launch(gpu.h, 512, 256, 256)       # small tiles: many of them
    ref = O.Oracle(ham, prm)
    for b in range(3):
        gpu.iterate(15)
        ref.iterate(15)
        _same_lists(gpu, ref, f"tiles{limit}/{b}")
        _same_estimates(gpu.estimates(), ref.estimates(), f"tiles{limit}/{b}")
    gpu.close()


@pytest.mark.parametrize("tile", [4096, 65536])
def test_large_tiles(tile):
    """A reference holding 20000 walkers fills whole tiles of 4096 attempts, or
    a large part of one tile of 65536 (the per-thread runs of the tile split are
    then long, and cross from the reference to the entries after it)."""
    ham, prm, _ = S.workload("hubbard8")
    prm.initial_walkers, prm.target_walkers = 20000, 40000
    print(f"[gpu] large tiles: {tile}", flush=True)
    gpu = F.Solver(ham, prm, _stream())
    F.fciqmc_set_launch(gpu.h, 512, tile, 256)
    ref = O.Oracle(ham, prm)
    for b in range(3):
        gpu.iterate(30)
        ref.iterate(30)
        _same_lists(gpu, ref, f"tile{tile}/{b}")
        _same_estimates(gpu.estimates(), ref.estimates(), f"tile{tile}/{b}")
    gpu.close()


def _loaded_pair(ham, prm, det, pop, **state):
    gpu = F.Solver(ham, prm, _stream())
    ref = O.Oracle(ham, prm)
    gpu.load_walkers(det, pop, **state)
    ref.load_walkers(det, pop, **state)
    return gpu, ref


def test_reference_population_zero():
    """C_0 = 0 (the reference keeps its slot): no projected energy for that
    iteration, nothing spawned from the reference, spawns onto it kept."""
    ham, prm, _ = S.workload("hubbard8")
    prm.target_walkers = 10**9
    o = O.Oracle(ham, prm)
    o.iterate(120)
    det, pop, _ = o.walkers()
    o.close()
    pop = pop.copy()
    pop[det == np.uint64(ham.ref_det)] = 0
    print("[gpu] C0 = 0", flush=True)
    gpu, ref = _loaded_pair(ham, prm, det, pop, iteration=120)
    gpu.iterate(1)
    ref.iterate(1)
    _same_lists(gpu, ref, "c0zero")
    eg = gpu.estimates()
    _same_estimates(eg, ref.estimates(), "c0zero")
    for _ in range(3):
        gpu.iterate(5)
        ref.iterate(5)
        _same_lists(gpu, ref, "c0zero+")
    gpu.close()


def test_death_crossing_zero():
    """tau (H_ii - E0 - S) |C| > |C|: one stochastic rounding per determinant
    flips the sign of the population (on both sides identically)."""
    ham = S.synthetic_molecule(4, 2, 2, 53)
    prm = S.Params(tau=0.9, initiator_threshold=0, seed=3, target_walkers=10**9)
    dets = ed.determinants(4, 2, 2)
    o = O.Oracle(ham, prm)
    dh = np.array([o.hdiag(int(d)) for d in dets]) - o.hdiag(int(ham.ref_det))
    o.close()
    hi = np.argsort(dh)[-6:]
    det = np.array(sorted(dets[hi]), np.uint64)
    pop = np.array([3, -4, 5, 2, -3, 7], np.int32)
    print("[gpu] death crossing zero", flush=True)
    gpu, ref = _loaded_pair(ham, prm, det, pop, shift=-2.0)
    gpu.iterate(1)
    ref.iterate(1)
    _same_lists(gpu, ref, "cross0")
    dg, pg, _ = gpu.walkers()
    before = dict(zip(det.tolist(), pop.tolist()))
    after = dict(zip(dg.tolist(), pg.tolist()))
    assert any(before[d] * after.get(d, 0) < 0 for d in before), (before, after)
    gpu.close()
