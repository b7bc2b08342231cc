"""The oracle's time-averaged energies agree with exact diagonalisation."""
import numpy as np
import pytest

from oracle import ed
from oracle import oracle as O
from paper_1305_6981_amd import systems as S


@pytest.fixture(scope="module")
def hubbard8_exact():
    ham, _, _ = S.workload("hubbard8")
    e, _, _ = ed.ground_state(ham)
    return e


def test_hubbard8_plain_fciqmc_matches_ed(hubbard8_exact):
    ham, prm, info = S.workload("hubbard8")
    o = O.Oracle(ham, prm)
    o.iterate(info["iterations"])
    e = o.estimates()
    assert e["n_samples"] > 1000
    assert np.isfinite(e["e_proj_err"]) and e["e_proj_err"] < 0.1
    assert abs(e["e_proj_mean"] - hubbard8_exact) < 3 * e["e_proj_err"]
    assert abs(e["shift_mean"] - hubbard8_exact) < 3 * e["shift_err"] + 0.02


def test_initiator_bias_vanishes_with_many_walkers():
    """With N_w far above the size of the space every occupied det is an
    initiator and i-FCIQMC reaches the exact energy."""
    ham = S.synthetic_molecule(4, 2, 2, 61)
    exact, _, _ = ed.ground_state(ham)
    prm = S.Params(tau=0.02, initiator_threshold=3, target_walkers=20000, initial_walkers=5000,
                   shift_update_every=1, seed=5, avg_start=200)
    o = O.Oracle(ham, prm)
    o.iterate(1500)
    e = o.estimates()
    assert abs(e["e_proj_mean"] - exact) < 4 * e["e_proj_err"] + 1e-4
