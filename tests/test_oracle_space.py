"""Pins for restricted spaces (Sec. 5: children outside the space are null
excitations).

Each restricted space is enumerated here *constructively* -- CISD by moving at
most two electrons of the reference, a complete active space as a doubly
occupied core times all fillings of the active orbitals, a seniority-limited
space by placing electron pairs and single electrons -- and the Hamiltonian
restricted to it is diagonalised exactly (second-quantised construction of
oracle/ed.py). A run restricted to the space must keep every walker inside it
and sample the restricted ground state, which lies above the full one by 14 mHa
(CISD) to 130 mHa (CIS) for this system -- chosen so that the reference keeps
most of the ground-state weight (59 %), which keeps the projected energy an
unbiased and precise estimator. A restriction that admits every determinant
must leave the run bit-identical.
"""
import itertools

import numpy as np
import pytest

from oracle import ed
from oracle import oracle as O
from paper_1305_6981_amd import systems as S

EVEN = 0x5555555555555555
M, NA = 6, 3


def _ham():
    return S.synthetic_molecule(M, NA, NA, 76, orb_energy=np.linspace(-0.8, 0.8, M))


def _reference(ham):
    o = O.Oracle(ham, S.Params(tau=0.01))
    d0 = int(o.walkers()[0][0])
    o.close()
    return d0


def _cisd(d0, max_moved=2):
    occ = [p for p in range(2 * M) if d0 >> p & 1]
    emp = [p for p in range(2 * M) if not d0 >> p & 1]
    out = set()
    for k in range(max_moved + 1):
        for rem in itertools.combinations(occ, k):
            for add in itertools.combinations(emp, k):
                d = d0
                for p in rem:
                    d ^= 1 << p
                for p in add:
                    d |= 1 << p
                if bin(d & EVEN).count("1") == NA:      # spin counts kept
                    out.add(d)
    return out


def _cas(n_core, n_act):
    core = sum(3 << (2 * s) for s in range(n_core))
    act = range(n_core, n_core + n_act)
    return {core | sum(1 << (2 * s) for s in a) | sum(1 << (2 * s + 1) for s in b)
            for a in itertools.combinations(act, NA - n_core)
            for b in itertools.combinations(act, NA - n_core)}


def _seniority(smax):
    out = set()
    for npair in range(NA + 1):
        for pairs in itertools.combinations(range(M), npair):
            rest = [s for s in range(M) if s not in pairs]
            for a in itertools.combinations(rest, NA - npair):
                rest2 = [s for s in rest if s not in a]
                for b in itertools.combinations(rest2, NA - npair):
                    if len(a) + len(b) <= smax:
                        out.add(sum(3 << (2 * s) for s in pairs) | sum(1 << (2 * s) for s in a)
                                | sum(1 << (2 * s + 1) for s in b))
    return out


def _lowest(ham, dets):
    _, h = ed.build_hamiltonian(ham, np.array(sorted(dets), dtype=np.uint64))
    return float(np.linalg.eigvalsh(h)[0])


def _params(**space):
    return S.Params(tau=0.01, shift_damping=0.05, shift_update_every=10, target_walkers=15000,
                    initial_walkers=1500, seed=21, avg_start=400, **space)


def _cases():
    core, empty = S.cas_masks(1, 4, M)
    return {
        "cis": (dict(space=S.SPACE_EXCITATION, max_excitation=1), lambda d0: _cisd(d0, 1)),
        "cisd": (dict(space=S.SPACE_EXCITATION, max_excitation=2), lambda d0: _cisd(d0)),
        "cas(1,4)": (dict(space=S.SPACE_FROZEN, frozen_occupied=core, frozen_empty=empty),
                     lambda d0: _cas(1, 4)),
        "seniority<=2": (dict(space=S.SPACE_SENIORITY, max_seniority=2), lambda d0: _seniority(2)),
    }


def test_enumerations_are_consistent():
    """The constructive enumerations against a filter of the full space by their
    definitions (sizes and membership), so that a slip in either shows."""
    ham = _ham()
    d0 = _reference(ham)
    full = [int(d) for d in ed.determinants(M, NA, NA)]
    assert _cisd(d0) == {d for d in full if bin(d & ~d0).count("1") <= 2}
    assert len(_cas(1, 4)) == 36 and len(_seniority(0)) == 20     # C(4,2)^2, C(6,3)
    assert d0 in _cisd(d0) and d0 in _cas(1, 4) and d0 in _seniority(0)


@pytest.mark.parametrize("name", ["cis", "cisd", "cas(1,4)", "seniority<=2"])
def test_restricted_run_samples_the_restricted_ground_state(name):
    ham = _ham()
    d0 = _reference(ham)
    space, enum = _cases()[name]
    allowed = enum(d0)
    e_space = _lowest(ham, allowed)
    e_full = ed.ground_state(ham)[0]
    assert e_space - e_full > 0.01          # the restriction matters for this system
    o = O.Oracle(ham, _params(**space))
    for _ in range(8):
        o.iterate(275)
        det, _, _ = o.walkers()
        assert set(int(d) for d in det) <= allowed, name
    e = o.estimates()
    o.close()
    assert e["n_samples"] > 1000
    m, err = e["e_proj_mean"], e["e_proj_err"]
    assert abs(m - e_space) < 4 * err + 1e-3, (name, m, err, e_space)
    assert abs(m - e_full) > 4 * err + 1e-3, (name, m, err, e_full)
    # the shift carries the population-control bias (~ +8 mHa at these walker numbers)
    assert abs(e["shift_mean"] - e_space) < 4 * e["shift_err"] + 0.02, (name, e["shift_mean"])


def test_restriction_that_admits_everything_changes_nothing():
    ham = _ham()
    n = 2 * NA
    runs = [_params(), _params(space=S.SPACE_EXCITATION, max_excitation=n),
            _params(space=S.SPACE_SENIORITY, max_seniority=2 * M),
            _params(space=S.SPACE_FROZEN, frozen_occupied=0, frozen_empty=0)]
    lists = []
    for p in runs:
        o = O.Oracle(ham, p)
        o.iterate(150)
        lists.append(o.walkers())
        o.close()
    for other in lists[1:]:
        for a, b in zip(lists[0], other):
            assert np.array_equal(a, b)


def test_reference_outside_the_space_is_rejected():
    ham = _ham()
    d0 = _reference(ham)
    with pytest.raises(RuntimeError):
        O.Oracle(ham, _params(space=S.SPACE_FROZEN, frozen_empty=d0 & -d0))
    with pytest.raises(RuntimeError):
        O.Oracle(ham, _params(space=S.SPACE_FROZEN, frozen_occupied=3, frozen_empty=1))
