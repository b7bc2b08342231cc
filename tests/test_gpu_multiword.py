"""Determinants of more than 64 spin orbitals on the GPU (Sec. 3: two 64-bit words
per determinant), bit-exact against the oracle, whose two-word runs are pinned by
operator-built elements, enumerated pgen and an exact energy across bit 64
(tests/test_oracle_multiword.py); and the two-word kernels forced on systems of
at most 64 spin orbitals, which must reproduce the one-word runs exactly."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1305_6981_amd import fciqmc as F
from paper_1305_6981_amd import systems as S

from test_gpu_parity import _same_estimates, _same_lists, _stream

pytestmark = pytest.mark.gpu


def _det(alpha, beta):
    return sum(1 << (2 * int(s)) for s in alpha) | sum(1 << (2 * int(s) + 1) for s in beta)


def _pair(ham, prm, blocks, per, tag, planner=True):
    print(f"[gpu] multiword {tag}: {ham.name} n_orb {ham.n_orb} target {prm.target_walkers}",
          flush=True)
    gpu = F.Solver(ham, prm, _stream())
    if not planner:
        F.fciqmc_set_test_options(gpu.h, 0, -1, 512)
    ref = O.Oracle(ham, prm)
    assert F.fciqmc_det_words(gpu.h) == ref.W
    for b in range(blocks):
        gpu.iterate(per)
        ref.iterate(per)
        _same_lists(gpu, ref, f"{tag}/{b}")
        _same_estimates(gpu.estimates(), ref.estimates(), f"{tag}/{b}")
    e = gpu.estimates()
    gpu.close()
    ref.close()
    return e


def test_molecule_in_72_spin_orbitals_with_initiators():
    ham = S.synthetic_molecule(36, 3, 3, 61, orb_energy=np.linspace(-4.0, 4.0, 36))
    prm = S.Params(tau=0.01, shift_damping=0.5, shift_update_every=5, target_walkers=6000,
                   initial_walkers=600, seed=31, initiator_threshold=2)
    _pair(ham, prm, 3, 50, "mol36")


def test_reference_in_the_second_word():
    # lowest orbitals last: the reference sits in spin orbitals 64..69
    ham = S.synthetic_molecule(35, 3, 3, 62, orb_energy=np.linspace(4.0, -4.0, 35))
    assert int(ham.ref_det) >> 64 and not int(ham.ref_det) & ((1 << 64) - 1)
    prm = S.Params(tau=0.01, shift_damping=0.5, shift_update_every=5, target_walkers=5000,
                   initial_walkers=500, seed=32)
    _pair(ham, prm, 3, 50, "ref-high")


def test_hubbard_ring_of_40_sites():
    ham = S.hubbard_ring(40, 3.0, n_alpha=3, n_beta=3)
    prm = S.Params(tau=0.01, shift_damping=0.5, shift_update_every=1, target_walkers=4000,
                   initial_walkers=400, seed=33)
    _pair(ham, prm, 3, 40, "hubbard40")


def test_largest_width_128_spin_orbitals():
    # 64 spatial orbitals, the reference in the four highest spin orbitals (124..127)
    ham = S.synthetic_molecule(64, 2, 2, 67, orb_energy=np.linspace(3.0, -3.0, 64))
    assert int(ham.ref_det) == (15 << 124)
    prm = S.Params(tau=0.01, shift_damping=0.5, shift_update_every=5, target_walkers=4000,
                   initial_walkers=400, seed=38, initiator_threshold=1)
    _pair(ham, prm, 3, 40, "mol64")


def test_point_group_labels_beyond_orbital_32():
    irr = np.array([(i * 5) % 4 for i in range(40)], np.uint8)
    ham = S.synthetic_molecule(40, 3, 3, 63, irreps=irr, orb_energy=np.linspace(-4.0, 4.0, 40))
    prm = S.Params(tau=0.01, shift_damping=0.5, shift_update_every=5, target_walkers=4000,
                   initial_walkers=400, seed=34)
    _pair(ham, prm, 3, 40, "irreps40")


def test_spin_coupled_functions_with_two_words():
    ham = S.synthetic_molecule(34, 3, 3, 64, orb_energy=np.linspace(-4.0, 4.0, 34))
    prm = S.Params(tau=0.01, shift_damping=0.5, shift_update_every=5, target_walkers=4000,
                   initial_walkers=400, seed=35, hphf=1)
    _pair(ham, prm, 3, 40, "hphf34")


def test_restricted_space_with_high_frozen_orbitals():
    # CAS: spatial orbital 0 doubly occupied, orbitals 34 and 35 (spin orbitals 68..71,
    # in the second word) empty, and at most a double excitation of the reference
    core, empty = S.cas_masks(1, 33, 36)
    assert empty >> 64
    ham = S.synthetic_molecule(36, 3, 3, 65, orb_energy=np.linspace(-4.0, 4.0, 36))
    prm = S.Params(tau=0.01, shift_damping=0.5, shift_update_every=5, target_walkers=3000,
                   initial_walkers=300, seed=36, space=S.SPACE_FROZEN | S.SPACE_EXCITATION,
                   frozen_occupied=core, frozen_empty=empty, max_excitation=2)
    _pair(ham, prm, 3, 40, "cas36")


def test_overflow_paths_with_two_words():
    """Planner off, small tables and a 512-record buffer: redo and spill paths with
    32-byte records and two-word spill entries."""
    ham = S.synthetic_molecule(34, 2, 2, 66, orb_energy=np.linspace(-4.0, 4.0, 34))
    prm = S.Params(tau=0.01, shift_damping=0.5, shift_update_every=5, target_walkers=20000,
                   initial_walkers=2000, seed=37, det_capacity=4096)
    e = _pair(ham, prm, 3, 40, "overflow34", planner=False)
    print(f"[gpu] multiword overflow: {e['redos']} re-run, {e['spills']} spilled", flush=True)
    assert e["redos"] > 0 and e["spills"] > 0


@pytest.mark.parametrize("name", ["hubbard8", "synth10e20o"])
def test_forced_two_words_reproduce_one_word_runs(name):
    if name == "hubbard8":
        ham, prm, _ = S.workload("hubbard8", scale=0.5)
    else:
        ham, prm, _ = S.workload("synth10e20o", scale=3e-3)
        prm.initial_walkers, prm.initial_shift = 3000, 0.5
    print(f"[gpu] multiword forced: {name}", flush=True)
    runs = []
    for w in (0, 2):
        prm.det_words = w
        gpu = F.Solver(ham, prm, _stream())
        assert F.fciqmc_det_words(gpu.h) == (2 if w == 2 else 1)
        gpu.iterate(80)
        det, pop, flg = gpu.walkers()
        ints = O.det_ints(det)
        runs.append((ints, pop, flg, gpu.estimates()))
        gpu.close()
    (d1, p1, f1, e1), (d2, p2, f2, e2) = runs
    assert d1 == d2 and np.array_equal(p1, p2) and np.array_equal(f1, f2)
    for k in ("n_walkers", "n_dets", "attempts", "spawns", "merged", "aborted", "born", "shift"):
        assert e1[k] == e2[k], k


def test_two_word_walker_lists_and_limits():
    ham = S.synthetic_molecule(36, 3, 3, 61, orb_energy=np.linspace(-1.5, 1.5, 36))
    prm = S.Params(tau=0.01, seed=3)
    gpu = F.Solver(ham, prm, _stream())
    d0 = int(ham.ref_det)
    dets = [d0, _det([0, 1, 33], [0, 1, 2]), _det([32, 33, 34], [0, 1, 35])]
    gpu.load_walkers(dets, np.array([7, -3, 2], np.int32))
    det, pop, _ = gpu.walkers()
    assert det.shape == (3, 2)
    assert dict(zip(O.det_ints(det), pop.tolist())) == {d0: 7, dets[1]: -3, dets[2]: 2}
    assert O.det_ints(det) == sorted(O.det_ints(det))
    with pytest.raises(F.FciqmcError):        # the staging export holds one word only
        F.fciqmc_walkers_noalloc(gpu.h, np.zeros(8, np.uint64), None, None)
    gpu.close()
    with pytest.raises(F.FciqmcError):        # one word cannot hold 72 spin orbitals
        F.Solver(ham, S.Params(tau=0.01, det_words=1), _stream())
    with pytest.raises(F.FciqmcError):        # one width per batch
        F.fciqmc_batch_create(2, [ham, S.hubbard_ring(8, 4.0)],
                              [S.Params(tau=0.01), S.Params(tau=0.01)], _stream())
