"""Pins for the oracle's Slater-Condon rules and diagonal elements.

Every matrix element is compared with a matrix built by applying
second-quantised operators to bit strings (oracle/ed.py), on small random
Hamiltonians with and without point-group labels; the energy is pinned by
closed forms (free fermions, the atomic limit)."""
import itertools
import math

import numpy as np
import pytest

from oracle import ed
from oracle import oracle as O
from paper_1305_6981_amd import systems as S


def _compare_all(ham, tol=1e-13):
    dets, H = ed.build_hamiltonian(ham)
    o = O.Oracle(ham, S.Params(tau=0.01))
    worst = 0.0
    for i, di in enumerate(dets):
        for j, dj in enumerate(dets):
            v = o.hel(int(di), int(dj))
            worst = max(worst, abs(v - H[i, j]))
    assert worst < tol, worst
    assert np.abs(H - H.T).max() < 1e-14
    return dets, H


@pytest.mark.parametrize("m,na,nb,seed", [(4, 2, 2, 11), (5, 2, 1, 12), (5, 3, 2, 13), (6, 1, 1, 14)])
def test_slater_condon_matches_second_quantisation(m, na, nb, seed):
    _compare_all(S.synthetic_molecule(m, na, nb, seed))


def test_slater_condon_with_point_group_labels():
    irr = np.array([0, 1, 2, 3, 0, 1], dtype=np.uint8)
    _compare_all(S.synthetic_molecule(6, 2, 2, 21, irreps=irr))


def test_hubbard_ring_elements():
    _compare_all(S.hubbard_ring(6, 3.0))


def test_free_fermion_closed_form():
    # U = 0: the ground state fills the lowest one-particle levels -2t cos(2 pi k / L) per spin.
    for L in (6, 8):
        e, _, _ = ed.ground_state(S.hubbard_ring(L, 0.0))
        levels = sorted(-2.0 * math.cos(2 * math.pi * k / L) for k in range(L))
        exact = 2 * sum(levels[: L // 2])
        assert abs(e - exact) < 1e-10


def test_atomic_limit_diagonal():
    # t = 0: H_DD = U x (number of doubly occupied sites).
    ham = S.hubbard_ring(6, 2.5, t=0.0)
    o = O.Oracle(ham, S.Params(tau=0.01))
    for d in ed.determinants(6, 3, 3)[:200]:
        d = int(d)
        docc = sum(1 for s in range(6) if (d >> (2 * s)) & 1 and (d >> (2 * s + 1)) & 1)
        assert o.hdiag(d) == pytest.approx(2.5 * docc, abs=1e-14)


def test_projected_energy_on_exact_eigenvector():
    # Eq. ProjE is exact for the exact wavefunction.
    ham = S.synthetic_molecule(5, 2, 2, 31)
    e, v, dets = ed.ground_state(ham)
    o = O.Oracle(ham, S.Params(tau=0.01))
    d0 = ham.ref_det
    i0 = int(np.nonzero(dets == np.uint64(d0))[0][0])
    num = o.proj_num(dets, v)
    assert abs(o.hdiag(d0) + num / v[i0] - e) < 1e-12


def test_decode_matches_bit_loop():
    rng = np.random.default_rng(2)
    for _ in range(2000):
        d = int(rng.integers(0, 2**63, dtype=np.uint64)) | (int(rng.integers(0, 2)) << 63)
        assert O.decode(d) == [b for b in range(64) if (d >> b) & 1]
    assert O.decode(0) == []


def test_storage_words_per_determinant():
    # ceil(2M/64) + 1 64-bit words per occupied determinant; 128 spin orbitals ->
    # 3 words, so 100 MB holds more than four million determinants (Sec. 3).
    words = math.ceil(128 / 64) + 1
    assert words == 3 and 100e6 / (8 * words) > 4e6
