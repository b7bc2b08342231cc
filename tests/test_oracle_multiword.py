"""Pins for determinants of more than 64 spin orbitals (Sec. 3: a determinant takes
as many 64-bit words as its spin orbitals need; two words here, up to 128).

The test's own arithmetic is on Python integers, which have no word boundary:
  - every element <D'|H|D> the oracle returns equals the coefficient of |D'> in
    H|D>, computed by applying the second-quantised operators of
    H = sum h_pq a+_p a_q + 1/2 sum (pq|rs) a+_p a+_r a_s a_q to the bit string
    (a_q |D> = (-1)^(occupied orbitals below q) |D - q>, likewise a+_p), for
    determinants with electrons on both sides of bit 64;
  - the generation probability of every sampled excitation equals the exhaustive
    enumeration of the generation process of Secs. 5.1-5.2 (the enumeration of
    tests/test_oracle_excitgen.py), and the sampled frequencies follow it;
  - a two-electron system in 34 orbitals whose reference lies in the second word
    is diagonalised exactly in the matrix built by the same operator action, and
    the run samples that ground-state energy;
  - two words forced on a system of at most 64 spin orbitals change nothing.
"""
from collections import defaultdict

import numpy as np
import pytest
from scipy import stats

from oracle import oracle as O
from paper_1305_6981_amd import systems as S
from test_oracle_excitgen import enumerate_generation


def _unpack(ham):
    """Full spatial (pq|rs) from the eight-fold packed array, vectorised."""
    m = ham.n_orb
    i = np.arange(m)
    hi, lo = np.maximum.outer(i, i), np.minimum.outer(i, i)
    pair = hi * (hi + 1) // 2 + lo                     # (m, m)
    a = pair[:, :, None, None]
    b = pair[None, None, :, :]
    big, small = np.maximum(a, b), np.minimum(a, b)
    return np.asarray(ham.eri)[big * (big + 1) // 2 + small]


def _ann(d, q):
    if not (d >> q) & 1:
        return 0, 0
    return (-1 if bin(d & ((1 << q) - 1)).count("1") & 1 else 1), d ^ (1 << q)


def _cre(d, p):
    if (d >> p) & 1:
        return 0, 0
    return (-1 if bin(d & ((1 << p) - 1)).count("1") & 1 else 1), d | (1 << p)


def apply_h(ham, g, ket):
    """H|ket> as {determinant: coefficient} by the operator definitions above."""
    n_so = 2 * ham.n_orb
    h1 = np.asarray(ham.h1)
    out = defaultdict(float)
    out[ket] += ham.e_core
    occ = [r for r in range(n_so) if (ket >> r) & 1]
    for q in occ:
        s1, d1 = _ann(ket, q)
        for p in range(q & 1, n_so, 2):
            v = h1[p >> 1, q >> 1]
            if v == 0.0:
                continue
            s2, d2 = _cre(d1, p)
            if s2:
                out[d2] += v * s1 * s2
    for q in occ:
        s1, d1 = _ann(ket, q)
        for s in occ:
            s2, d2 = _ann(d1, s)
            if not s2:
                continue
            for r in range(s & 1, n_so, 2):
                s3, d3 = _cre(d2, r)
                if not s3:
                    continue
                for p in range(q & 1, n_so, 2):
                    v = g[p >> 1, q >> 1, r >> 1, s >> 1]
                    if v == 0.0:
                        continue
                    s4, d4 = _cre(d3, p)
                    if s4:
                        out[d4] += 0.5 * v * s1 * s2 * s3 * s4
    return out


def _det(alpha, beta):
    return sum(1 << (2 * int(s)) for s in alpha) | sum(1 << (2 * int(s) + 1) for s in beta)


def _mol36():
    """3 alpha + 3 beta electrons in 36 orbitals (72 spin orbitals)."""
    return S.synthetic_molecule(36, 3, 3, 61, orb_energy=np.linspace(-1.5, 1.5, 36))


def test_two_words_and_limits():
    o = O.Oracle(_mol36(), S.Params(tau=0.01))
    assert o.W == 2
    o.close()
    assert O.Oracle(S.synthetic_molecule(6, 2, 2, 3), S.Params(tau=0.01)).W == 1
    assert O.Oracle(S.synthetic_molecule(6, 2, 2, 3), S.Params(tau=0.01, det_words=2)).W == 2
    with pytest.raises(RuntimeError):       # more than 128 spin orbitals
        O.Oracle(S.hubbard_ring(66, 2.0, n_alpha=1, n_beta=1), S.Params(tau=0.01))
    with pytest.raises(RuntimeError):       # one word cannot hold 72 spin orbitals
        O.Oracle(_mol36(), S.Params(tau=0.01, det_words=1))


def test_elements_match_operator_action_across_the_word_boundary():
    ham = _mol36()
    g = _unpack(ham)
    o = O.Oracle(ham, S.Params(tau=0.01))
    kets = [int(ham.ref_det),
            _det([30, 31, 33], [31, 32, 35]),       # electrons in spin orbitals 62..71
            _det([0, 32, 34], [1, 31, 33]),
            _det([5, 31, 32], [0, 32, 35])]
    rng = np.random.default_rng(8)
    for _ in range(3):
        kets.append(_det(sorted(rng.choice(36, 3, replace=False)), sorted(rng.choice(36, 3, replace=False))))
    for ket in kets:
        assert ket.bit_length() <= 72
        col = apply_h(ham, g, ket)
        checked = 0
        for bra, ref in col.items():
            got = o.hel(bra, ket)
            assert abs(got - ref) <= 1e-12 * max(1.0, abs(ref)), (ket, bra, got, ref)
            checked += 1
        assert checked > 1000
        # a determinant three electrons away: zero
        far, used = ket, set()
        for q in [r for r in range(72) if (ket >> r) & 1][:3]:
            a = next(r for r in range(72)
                     if not (ket >> r) & 1 and (r & 1) == (q & 1) and r not in used)
            used.add(a)
            far ^= (1 << q) | (1 << a)
        assert bin(far ^ ket).count("1") == 6 and o.hel(far, ket) == 0.0
    o.close()


def test_pgen_equals_enumeration_with_two_words():
    ham = S.synthetic_molecule(34, 2, 2, 62, orb_energy=np.linspace(1.5, -1.5, 34))
    o = O.Oracle(ham, S.Params(tau=0.01, seed=78))
    assert o.W == 2
    p_double = o.estimates()["p_double"]
    for det in (int(ham.ref_det), _det([1, 32], [31, 33])):
        probs, p_null = enumerate_generation(ham, det, p_double)
        assert abs(sum(probs.values()) + p_null - 1.0) < 1e-12
        n = 60000
        out, pgen, hel = o.sample_excitations(det, n, iteration=5)
        counts = defaultdict(int)
        nulls = 0
        for d, pg in zip(out, pgen):
            if d == 0:
                nulls += 1
                continue
            ref = probs.get(d, 0.0)
            assert ref > 0.0 and abs(pg - ref) <= 1e-14 * ref
            counts[d] += 1
        keys = sorted(probs)
        obs = np.array([counts[k] for k in keys] + [nulls], float)
        exp = np.array([probs[k] for k in keys] + [p_null]) * n
        keep = exp > 0
        chi2 = ((obs[keep] - exp[keep]) ** 2 / exp[keep]).sum()
        assert stats.chi2.sf(chi2, int(keep.sum()) - 1) > 1e-5
        assert any(k >> 64 for k in counts) and any(k & O.MASK64 for k in counts)
        for t in list(probs)[:400]:
            assert abs(o.pgen(det, t) - probs[t]) <= 1e-14 * probs[t]
    o.close()


def test_run_samples_the_exact_energy_with_the_reference_in_the_second_word():
    # 1 alpha + 1 beta electron in 34 orbitals, lowest orbital last: the reference is
    # spin orbitals 66 and 67, and excitations move the electrons across bit 64. The
    # reference carries 90 % of the ground state (correlation energy -111 mHa); the
    # run starts near its target so that 2700 iterations are averaged.
    ham = S.synthetic_molecule(34, 1, 1, 63, orb_energy=np.linspace(4.0, -4.0, 34))
    assert int(ham.ref_det) == (3 << 66)
    g = _unpack(ham)
    dets = sorted(_det([a], [b]) for a in range(34) for b in range(34))
    index = {d: i for i, d in enumerate(dets)}
    H = np.zeros((len(dets), len(dets)))
    for j, ket in enumerate(dets):
        for bra, v in apply_h(ham, g, ket).items():
            H[index[bra], j] += v
    assert np.abs(H - H.T).max() < 1e-12
    w, v = np.linalg.eigh(H)
    e_exact = w[0]
    assert v[index[int(ham.ref_det)], 0] ** 2 > 0.85
    prm = S.Params(tau=0.01, shift_update_every=10, target_walkers=5000, initial_walkers=4500,
                   seed=9, avg_start=300)
    o = O.Oracle(ham, prm)
    assert abs(e_exact - o.estimates()["e_ref"]) > 0.1
    o.iterate(3000)
    e = o.estimates()
    det, pop, _ = o.walkers()
    o.close()
    ints = O.det_ints(det)
    assert all(d in index for d in ints)
    assert any(d >> 64 == 0 for d in ints)                    # both words in use
    assert e["n_samples"] > 2500
    assert abs(e["e_proj_mean"] - e_exact) < 4 * e["e_proj_err"] + 1e-3, (e["e_proj_mean"],
                                                                          e["e_proj_err"], e_exact)


@pytest.mark.parametrize("name", ["hubbard8", "mol6"])
def test_forced_two_words_change_nothing(name):
    if name == "hubbard8":
        ham, prm, _ = S.workload("hubbard8", scale=0.3)
    else:
        ham = S.synthetic_molecule(6, 3, 3, 76, orb_energy=np.linspace(-0.8, 0.8, 6))
        prm = S.Params(tau=0.01, target_walkers=3000, initial_walkers=300, seed=4,
                       initiator_threshold=2)
    runs = []
    for w in (0, 2):
        prm.det_words = w
        o = O.Oracle(ham, prm)
        o.iterate(120)
        det, pop, flg = o.walkers()
        runs.append((O.det_ints(det), pop, flg, o.estimates()))
        o.close()
    (d1, p1, f1, e1), (d2, p2, f2, e2) = runs
    assert d1 == d2 and np.array_equal(p1, p2) and np.array_equal(f1, f2)
    for k in ("n_walkers", "n_dets", "attempts", "spawns", "merged", "aborted", "born", "shift"):
        assert e1[k] == e2[k], k


def test_walker_list_round_trip_with_two_words():
    ham = _mol36()
    o = O.Oracle(ham, S.Params(tau=0.01, seed=3))
    d0 = int(ham.ref_det)
    dets = [d0, _det([0, 1, 33], [0, 1, 2]), _det([32, 33, 34], [0, 1, 35])]
    o.load_walkers(dets, np.array([7, -3, 2], np.int32))
    det, pop, _ = o.walkers()
    assert det.shape == (3, 2)
    got = dict(zip(O.det_ints(det), pop.tolist()))
    assert got == {d0: 7, dets[1]: -3, dets[2]: 2}
    assert O.det_ints(det) == sorted(got)
    o.close()


def test_largest_width_128_spin_orbitals():
    """64 spatial orbitals, electrons up to spin orbital 127: elements against the
    operator action and pgen against the enumeration."""
    ham = S.synthetic_molecule(64, 2, 2, 67, orb_energy=np.linspace(3.0, -3.0, 64))
    assert int(ham.ref_det) == (15 << 124)          # the four highest spin orbitals
    g = _unpack(ham)
    o = O.Oracle(ham, S.Params(tau=0.01, seed=12))
    assert o.W == 2
    kets = [int(ham.ref_det), _det([0, 63], [31, 32]), _det([1, 62], [63, 0])]
    for ket in kets:
        col = apply_h(ham, g, ket)
        for bra, ref in col.items():
            got = o.hel(bra, ket)
            assert abs(got - ref) <= 1e-12 * max(1.0, abs(ref)), (ket, bra, got, ref)
    p_double = o.estimates()["p_double"]
    for det in kets[:2]:
        probs, p_null = enumerate_generation(ham, det, p_double)
        assert abs(sum(probs.values()) + p_null - 1.0) < 1e-12
        out, pgen, _ = o.sample_excitations(det, 20000, iteration=2)
        for d, pg in zip(out, pgen):
            if d:
                assert abs(pg - probs[d]) <= 1e-14 * probs[d]
    o.close()
