"""The rule cases pinned in the oracle (initiator rule of Sec. 4.2, spawning of
more than one walker, the shift update of Sec. 2 with A = 10), run on the GPU
through the C ABI with the same expected outcomes."""
import pytest

import rule_cases as R
from paper_1305_6981_amd import fciqmc as F
from paper_1305_6981_amd import systems as S

pytestmark = pytest.mark.gpu


def make(ham, prm):
    import torch
    assert torch.cuda.is_available()
    return F.Solver(ham, prm, F.current_stream())


def test_initiator_threshold_is_strict():
    print("[gpu] rules: threshold", flush=True)
    R.check_threshold_is_strict(make)


def test_merged_spawn_flag_is_or_of_parents():
    print("[gpu] rules: OR of flags", flush=True)
    R.check_flags_are_ored(make)


def test_occupancy_for_initiator_test_is_after_death():
    print("[gpu] rules: after death", flush=True)
    R.check_occupancy_after_death(make)


def test_reference_is_always_an_initiator():
    print("[gpu] rules: reference", flush=True)
    R.check_reference_is_always_initiator(make)


def test_spawning_more_than_one_walker():
    print("[gpu] rules: multi-walker spawns", flush=True)
    R.check_multi_walker_spawns(make)


def test_shift_update_every_ten_iterations():
    print("[gpu] rules: shift schedule A=10", flush=True)
    ham, _, _ = S.workload("hubbard8")
    prm = S.Params(tau=0.01, shift_damping=0.05, shift_update_every=10, target_walkers=300,
                   initial_walkers=10, seed=4)
    R.check_shift_schedule(make, ham, prm, 160)
