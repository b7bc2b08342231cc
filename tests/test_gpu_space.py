"""Restricted spaces on the GPU (Sec. 5: children outside the space are null
excitations), bit-exact against the oracle, whose restricted runs are pinned
against exact diagonalisation on each space (tests/test_oracle_space.py)."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1305_6981_amd import fciqmc as F
from paper_1305_6981_amd import systems as S

pytestmark = pytest.mark.gpu


def _stream():
    return F.current_stream()


def _small():
    return S.synthetic_molecule(6, 3, 3, 76, orb_energy=np.linspace(-0.8, 0.8, 6))


def _spaces(n_orb):
    core, empty = S.cas_masks(1, 4, n_orb)
    return {
        "cis": dict(space=S.SPACE_EXCITATION, max_excitation=1),
        "cisd": dict(space=S.SPACE_EXCITATION, max_excitation=2),
        "cas": dict(space=S.SPACE_FROZEN, frozen_occupied=core, frozen_empty=empty),
        "seniority2": dict(space=S.SPACE_SENIORITY, max_seniority=2),
        "cisdt+seniority4": dict(space=S.SPACE_EXCITATION | S.SPACE_SENIORITY, max_excitation=3,
                                 max_seniority=4),
    }


def _pair(ham, prm, blocks, per, tag):
    print(f"[gpu] space {tag}: {ham.name} target {prm.target_walkers}", flush=True)
    gpu = F.Solver(ham, prm, _stream())
    ref = O.Oracle(ham, prm)
    for b in range(blocks):
        gpu.iterate(per)
        ref.iterate(per)
        dg, pg, fg = gpu.walkers()
        do, po, fo = ref.walkers()
        assert np.array_equal(dg, do) and np.array_equal(pg, po) and np.array_equal(fg, fo), (tag, b)
        eg, eo = gpu.estimates(), ref.estimates()
        for k in ("n_walkers", "n_dets", "ref_pop", "attempts", "spawns", "merged", "aborted", "born"):
            assert eg[k] == eo[k], (tag, b, k)
        assert eg["shift"] == eo["shift"], (tag, b)
        assert abs(eg["proj_num"] - eo["proj_num"]) <= 1e-10 * max(1.0, abs(eo["proj_num"]))
    gpu.close()
    ref.close()


@pytest.mark.parametrize("name", ["cis", "cisd", "cas", "seniority2", "cisdt+seniority4"])
def test_small_restricted_space_bit_exact(name):
    prm = S.Params(tau=0.01, shift_update_every=10, target_walkers=5000, initial_walkers=500,
                   seed=21, **_spaces(6)[name])
    _pair(_small(), prm, 3, 60, name)


@pytest.mark.parametrize("name", ["cisd", "cas"])
def test_larger_restricted_space_bit_exact(name):
    """10e/20o with the initiator rule, several buckets and spawn tiles."""
    ham, prm, _ = S.workload("synth10e20o", scale=3e-3)
    prm.initial_walkers, prm.initial_shift = 3000, 0.5
    for k, v in _spaces(20)[name].items():
        setattr(prm, k, v)
    _pair(ham, prm, 3, 40, "10e20o-" + name)


def test_space_checks_at_the_boundary():
    ham = _small()
    ok = S.Params(tau=0.01, seed=3, space=S.SPACE_EXCITATION, max_excitation=1)
    sv = F.Solver(ham, ok, _stream())
    d0 = int(sv.walkers()[0][0])
    # a triple excitation of the reference is outside the space: rejected on load
    occ = [p for p in range(12) if d0 >> p & 1][:3]
    emp = [p for p in range(12) if not d0 >> p & 1]
    a_emp = [p for p in emp if p % 2 == 0][:2]
    bad = d0 ^ (1 << occ[0]) ^ (1 << occ[2]) | (1 << a_emp[0]) | (1 << a_emp[1])
    assert bin(bad).count("1") == 6
    with pytest.raises(F.FciqmcError):
        sv.load_walkers(np.array([d0, bad], np.uint64), np.array([5, 2], np.int32))
    sv.close()
    # the reference outside the space, and contradictory masks
    with pytest.raises(F.FciqmcError):
        F.Solver(ham, S.Params(tau=0.01, space=S.SPACE_FROZEN, frozen_empty=d0 & -d0), _stream())
    with pytest.raises(F.FciqmcError):
        F.Solver(ham, S.Params(tau=0.01, space=S.SPACE_FROZEN, frozen_occupied=3,
                               frozen_empty=1), _stream())
