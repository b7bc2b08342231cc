"""Pins for the oracle's initiator rule (Sec. 4.2) and shift update (Sec. 2).

The initiator cases are hand-built one-electron lists whose next iteration the
rule fixes by construction (see tests/rule_cases.py): a strict threshold, the
OR of the parents' flags, and occupancy judged after death. The shift is
checked against its formula evaluated by hand on the recorded populations with
A = 10, and an A = 10 initiator run is checked against exact diagonalisation.
"""
import numpy as np

import rule_cases as R
from oracle import ed
from oracle import oracle as O
from paper_1305_6981_amd import systems as S


def make(ham, prm):
    return O.Oracle(ham, prm)


def test_initiator_threshold_is_strict():
    R.check_threshold_is_strict(make)


def test_merged_spawn_flag_is_or_of_parents():
    R.check_flags_are_ored(make)


def test_occupancy_for_initiator_test_is_after_death():
    R.check_occupancy_after_death(make)


def test_reference_is_always_an_initiator():
    R.check_reference_is_always_initiator(make)


def test_star_spawns_are_single_walkers_onto_the_hub():
    """The construction itself: from a leaf every attempt either picks the hub
    (one walker) or nothing; about a quarter of the attempts pick the hub."""
    ham = R.star(leaves=(R.P1,))
    o = O.Oracle(ham, R.params())
    od, pg, he = o.sample_excitations(R.det(R.P1), 4000)
    o.close()
    assert np.all(pg == 0.25)
    hub = od == np.uint64(R.det(R.HUB))
    assert np.all(he[hub] == -1.0) and np.all(he[~hub] == 0.0)
    assert abs(hub.mean() - 0.25) < 0.03


def test_shift_update_every_ten_iterations():
    ham, _, _ = S.workload("hubbard8")
    prm = S.Params(tau=0.01, shift_damping=0.05, shift_update_every=10, target_walkers=300,
                   initial_walkers=10, seed=4)
    hist = R.check_shift_schedule(make, ham, prm, 160)
    assert any(e["shift"] != 0.0 for e in hist)


def test_initiator_energy_with_shift_update_every_ten_matches_ed():
    """i-FCIQMC with A = 10 at N_w far above the size of the space (36 dets):
    every determinant is an initiator and both estimators reach the exact energy."""
    ham = S.synthetic_molecule(4, 2, 2, 61)
    exact, _, _ = ed.ground_state(ham)
    prm = S.Params(tau=0.02, initiator_threshold=3, target_walkers=8000, initial_walkers=4000,
                   shift_update_every=10, seed=8, avg_start=300)
    o = O.Oracle(ham, prm)
    o.iterate(2000)
    e = o.estimates()
    o.close()
    assert e["n_samples"] > 1000
    assert abs(e["e_proj_mean"] - exact) < 4 * e["e_proj_err"] + 1e-4
    assert abs(e["shift_mean"] - exact) < 4 * e["shift_err"] + 2e-3


def test_spawning_more_than_one_walker():
    R.check_multi_walker_spawns(make)
