"""Pins for the oracle's walker dynamics (Sec. 2) and annihilation (Sec. 4)."""
import numpy as np
import pytest

from oracle import ed
from oracle import oracle as O
from paper_1305_6981_amd import systems as S


def test_one_step_expectation_matches_master_equation():
    """Averaged over seeds, one iteration reproduces Eq. master:
    C' = [1 - tau (H_ii - E0 - S)] C - tau sum_j H_ij C_j (plain mode)."""
    ham = S.synthetic_molecule(4, 2, 2, 51)
    dets, H = ed.build_hamiltonian(ham)
    rng = np.random.default_rng(6)
    c = rng.integers(5, 40, size=len(dets)) * rng.choice([-1, 1], size=len(dets))
    tau, shift = 0.02, 0.3
    e0 = H[np.nonzero(dets == np.uint64(ham.ref_det))[0][0]].max()
    i0 = int(np.nonzero(dets == np.uint64(ham.ref_det))[0][0])
    e0 = H[i0, i0]
    expect = c - tau * (H @ c) + tau * (e0 + shift) * c
    R = 1500
    acc = np.zeros(len(dets))
    acc2 = np.zeros(len(dets))
    for r in range(R):
        prm = S.Params(tau=tau, initiator_threshold=0, seed=1000 + r, target_walkers=10**9)
        o = O.Oracle(ham, prm)
        o.load_walkers(dets, c.astype(np.int32), iteration=r, shift=shift)
        o.iterate(1)
        d, p, _ = o.walkers()
        v = np.zeros(len(dets))
        idx = np.searchsorted(dets, d)
        v[idx] = p
        acc += v
        acc2 += v * v
        o.close()
    mean = acc / R
    sd = np.sqrt(np.maximum(acc2 / R - mean ** 2, 1e-12) / R)
    z = (mean - expect) / sd
    assert np.all(np.abs(z) < 4.5), np.abs(z).max()


def test_initiator_rule_discards_noninitiator_spawns_on_empty_dets():
    """With a huge threshold only the reference is an initiator, so new dets are
    created only from the reference; the aborted count is positive."""
    ham = S.synthetic_molecule(6, 2, 2, 52)
    prm = S.Params(tau=0.05, initiator_threshold=10**6, seed=9, initial_walkers=2000,
                   target_walkers=10**9)
    o = O.Oracle(ham, prm)
    o.iterate(1)
    d1, p1, _ = o.walkers()
    # after one iteration every occupied det is the reference or reachable from it
    ref = int(ham.ref_det)
    for d in d1:
        assert bin(int(d) ^ ref).count("1") <= 4
    aborted = 0
    for _ in range(20):
        o.iterate(1)
        aborted += o.estimates()["aborted"]
    assert aborted > 0


def test_walker_lists_independent_of_hash_layout():
    """Algorithm 1 and the table size only place determinants in memory: the
    walker list is the same for any map seed and table size."""
    ham, prm, _ = S.workload("hubbard8", scale=0.3)
    lists = []
    for hs, hr in [(1, 16), (99, 4096), (12345, 7)]:
        o = O.Oracle(ham, prm, hash_seed=hs, hash_range=hr)
        o.iterate(150)
        lists.append(o.walkers())
        e = o.estimates()
    for a in lists[1:]:
        assert np.array_equal(a[0], lists[0][0]) and np.array_equal(a[1], lists[0][1])


def test_hash_spreads_determinants_uniformly():
    ham = S.synthetic_molecule(20, 5, 5, 2)
    o = O.Oracle(ham, S.Params(tau=0.01), hash_seed=3)
    rng = np.random.default_rng(8)
    nb = 64
    counts = np.zeros(nb)
    seen = set()
    while len(seen) < 20000:
        a = rng.choice(20, 5, replace=False)
        b = rng.choice(20, 5, replace=False)
        d = 0
        for s in a:
            d |= 1 << (2 * int(s))
        for s in b:
            d |= 1 << (2 * int(s) + 1)
        if d in seen:
            continue
        seen.add(d)
        h = o.hash(d, nb)
        assert 0 <= h < nb
        counts[h] += 1
    from scipy import stats
    chi2 = ((counts - counts.mean()) ** 2 / counts.mean()).sum()
    assert stats.chi2.sf(chi2, nb - 1) > 1e-4


def test_death_can_cross_zero():
    """One stochastic rounding per determinant: when tau (H_ii - E0 - S) |C| exceeds
    |C| the population changes sign (a unit case of the death step)."""
    ham = S.synthetic_molecule(4, 2, 2, 53)
    o = O.Oracle(ham, S.Params(tau=0.9, initiator_threshold=0, seed=3, target_walkers=10**9))
    dets = ed.determinants(4, 2, 2)
    hi = max((o.hdiag(int(d)) - o.hdiag(int(ham.ref_det)), int(d)) for d in dets)
    o.load_walkers(np.array([hi[1]], np.uint64), np.array([3], np.int32), shift=-2.0)
    o.iterate(1)
    d, p, _ = o.walkers()
    got = dict(zip(d.tolist(), p.tolist())).get(hi[1], 0)
    # expected death count 0.9*(dH+2)*3 > 3 walkers: population flips sign or shrinks past zero
    assert 0.9 * (hi[0] + 2.0) * 3 > 3
    assert got <= 0
