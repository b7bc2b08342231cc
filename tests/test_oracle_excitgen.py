"""Pins for the oracle's excitation generator (Sec. 5).

The generation process described in Secs. 5.1-5.2 is enumerated exhaustively
here in Python (every electron / pair / orbital choice with its probability,
including the renormalisation over choices with no allowed partner). The pgen
the oracle returns for each sampled excitation must equal that enumerated
probability, the probabilities must be normalised with the null excitations,
and the sampled frequencies must follow them (chi-squared)."""
from collections import defaultdict
from math import comb

import numpy as np
import pytest
from scipy import stats

from oracle import oracle as O
from paper_1305_6981_amd import systems as S


def _cls(ham, r):
    irr = 0 if ham.orb_irrep is None else int(ham.orb_irrep[r >> 1])
    return (irr, r & 1)


def enumerate_generation(ham, det, p_double):
    n_so = 2 * ham.n_orb
    occ = [r for r in range(n_so) if (det >> r) & 1]
    emp = [r for r in range(n_so) if not (det >> r) & 1]
    probs = defaultdict(float)
    p_null = 0.0
    p_single = 1.0 - p_double
    movable = [e for e in occ if any(_cls(ham, a) == _cls(ham, e) for a in emp)]
    if movable:
        for e in movable:
            tgt = [a for a in emp if _cls(ham, a) == _cls(ham, e)]
            for a in tgt:
                probs[det ^ (1 << e) ^ (1 << a)] += p_single / len(movable) / len(tgt)
    else:
        p_null += p_single
    pairs = [(p, q) for i, p in enumerate(occ) for q in occ[i + 1:]]
    irr = lambda r: _cls(ham, r)[0]
    for p, q in pairs:
        pp = p_double / len(pairs)
        same = (p & 1) == (q & 1)
        first = [x for x in emp if (not same) or (x & 1) == (p & 1)]

        def partners(x):
            spin_b = (p & 1) if same else 1 - (x & 1)
            want = (irr(p) ^ irr(q) ^ irr(x), spin_b)
            return [y for y in emp if y != x and _cls(ham, y) == want]

        ok = [x for x in first if partners(x)]
        if not ok:
            p_null += pp
            continue
        for a in ok:
            pb = partners(a)
            for b in pb:
                probs[det ^ (1 << p) ^ (1 << q) ^ (1 << a) ^ (1 << b)] += pp / len(ok) / len(pb)
    if not pairs:
        p_null += p_double
    return probs, p_null


CASES = [
    ("c1", lambda: S.synthetic_molecule(5, 2, 2, 41), None),
    ("open", lambda: S.synthetic_molecule(6, 3, 2, 42), None),
    ("irreps", lambda: S.synthetic_molecule(6, 2, 2, 43, irreps=np.array([0, 1, 2, 3, 0, 1], np.uint8)), None),
    ("irreps_open", lambda: S.synthetic_molecule(6, 3, 1, 44, irreps=np.array([0, 0, 1, 1, 2, 3], np.uint8)), None),
    ("hubbard", lambda: S.hubbard_ring(6, 4.0), None),
]


@pytest.mark.parametrize("name,mk,_", CASES)
def test_pgen_equals_enumerated_probability(name, mk, _):
    ham = mk()
    o = O.Oracle(ham, S.Params(tau=0.01, seed=77))
    p_double = o.estimates()["p_double"]
    rng = np.random.default_rng(5)
    from oracle import ed
    dets = ed.determinants(ham.n_orb, ham.n_alpha, ham.n_beta)
    for det in [int(ham.ref_det)] + [int(d) for d in rng.choice(dets, size=min(6, len(dets)), replace=False)]:
        probs, p_null = enumerate_generation(ham, det, p_double)
        assert abs(sum(probs.values()) + p_null - 1.0) < 1e-12
        n = 60000
        out, pgen, hel = o.sample_excitations(det, n, iteration=3)
        nulls = out == 0
        for d, pg in zip(out[~nulls], pgen[~nulls]):
            ref = probs.get(int(d), 0.0)
            assert ref > 0.0
            assert abs(pg - ref) <= 1e-14 * ref
        # chi-squared on the outcome frequencies (null collected as one outcome)
        keys = sorted(probs)
        counts = defaultdict(int)
        for d in out[~nulls]:
            counts[int(d)] += 1
        obs = np.array([counts[k] for k in keys] + [int(nulls.sum())], float)
        exp = np.array([probs[k] for k in keys] + [p_null]) * n
        keep = exp > 0
        chi2 = ((obs[keep] - exp[keep]) ** 2 / exp[keep]).sum()
        dof = int(keep.sum()) - 1
        assert stats.chi2.sf(chi2, dof) > 1e-5, (name, det, chi2, dof)
        # Every element returned is <D'|H|D>.
        for d, h in list(zip(out[~nulls], hel[~nulls]))[:300]:
            assert h == o.hel(int(d), det)
        # The probability of a given target (used for spin-coupled functions) equals the
        # enumerated one for every determinant of the sector.
        for t in dets:
            ref = probs.get(int(t), 0.0)
            got = o.pgen(det, int(t))
            assert abs(got - ref) <= 1e-14 * ref if ref > 0 else got == 0.0, (name, det, int(t))


def _combinatorial_p_double(m, na, nb):
    ns = na * (m - na) + nb * (m - nb)
    nd = comb(na, 2) * comb(m - na, 2) + comb(nb, 2) * comb(m - nb, 2) + na * nb * (m - na) * (m - nb)
    return nd / (ns + nd)


@pytest.mark.parametrize("m,na,nb", [(20, 5, 5), (30, 12, 12), (16, 5, 5), (26, 7, 7)])
def test_p_double_from_reference_counts(m, na, nb):
    ham = S.synthetic_molecule(m, na, nb, 1)
    o = O.Oracle(ham, S.Params(tau=0.01))
    assert o.estimates()["p_double"] == _combinatorial_p_double(m, na, nb)


def test_hubbard_singles_only():
    ham = S.hubbard_ring(8, 4.0)
    o = O.Oracle(ham, S.Params(tau=0.01))
    assert o.estimates()["p_double"] == 0.0
    out, pgen, hel = o.sample_excitations(int(ham.ref_det), 5000)
    # every excitation is a single (two bits differ)
    for d in out[out != 0][:500]:
        assert bin(int(d) ^ int(ham.ref_det)).count("1") == 2
