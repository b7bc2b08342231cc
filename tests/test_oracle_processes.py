"""Pins for the distribution of determinants over processes (Sec. 4.1).

The paper places every determinant on the process chosen by a second
Algorithm-1 hash over the number of processes, spawns into one block per
destination, exchanges the blocks once per iteration and annihilates locally.
Because the random numbers are keyed by determinant and iteration and the
merges are integer sums, the trajectory must not depend on how many processes
(or host threads) there are; only the rounding order of the projected-energy
numerator changes."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1305_6981_amd import systems as S

INT_KEYS = ("iteration", "n_walkers", "n_dets", "ref_pop", "attempts", "spawns", "merged",
            "aborted", "born", "total_attempts", "total_spawns", "n_samples", "n_var", "n_prev",
            "shift_varying")


def _run(ham, prm, iters, **kw):
    o = O.Oracle(ham, prm, **kw)
    o.iterate(iters)
    out = o.walkers(), o.estimates(), o
    return out


def _same(a, b, tag, skip=()):
    (wa, ea, _), (wb, eb, _) = a, b
    for x, y in zip(wa, wb):
        assert np.array_equal(x, y), tag
    for k in INT_KEYS:
        if k in skip:
            continue
        assert ea[k] == eb[k], (tag, k)
    assert ea["shift"] == eb["shift"], tag          # depends on integers only
    assert abs(ea["proj_num"] - eb["proj_num"]) <= 1e-12 * max(1.0, abs(ea["proj_num"])), tag


def _systems():
    hub, hprm, _ = S.workload("hubbard8", scale=0.3)
    mol = S.synthetic_molecule(10, 3, 3, 7)
    mprm = S.Params(tau=0.01, initiator_threshold=3, seed=21, initial_walkers=50,
                    target_walkers=3000, shift_update_every=5)
    return [("hubbard8", hub, hprm, 120), ("molecule-initiator", mol, mprm, 80)]


@pytest.mark.parametrize("name,ham,prm,iters", _systems(), ids=lambda v: v if isinstance(v, str) else "")
def test_trajectory_independent_of_process_count(name, ham, prm, iters):
    base = _run(ham, prm, iters)
    assert base[1]["n_dets"] > 50, "the run must reach many determinants to mean anything"
    for kw in (dict(n_procs=2), dict(n_procs=3, n_threads=2), dict(n_procs=7, n_threads=3),
               dict(n_procs=4, ref_own_proc=True, n_threads=4),
               dict(n_procs=5, proc_seed=77)):
        _same(base, _run(ham, prm, iters, **kw), f"{name} {kw}")


def test_determinants_sit_on_their_owner_only():
    ham, prm, _ = S.workload("hubbard8", scale=0.3)
    P = 6
    (det, pop, _), est, o = _run(ham, prm, 100, n_procs=P, n_threads=2)
    per = np.array([o.proc_dets(p) for p in range(P)])
    # the reference keeps its slot at zero population, so it may be counted once extra
    extra = 1 if est["ref_pop"] == 0 else 0
    assert per.sum() == len(det) + extra
    owners = np.array([o.owner(int(d)) for d in det])
    assert owners.min() >= 0 and owners.max() < P
    assert np.array_equal(np.bincount(owners, minlength=P) + (np.arange(P) == o.owner(int(ham.ref_det))) * extra, per)
    with pytest.raises(RuntimeError):
        o.proc_dets(P)


def test_dedicated_reference_process():
    """Load balancing of Sec. 4.1: the reference alone on process 0, everything
    else hashed over the remaining processes."""
    ham, prm, _ = S.workload("hubbard8", scale=0.3)
    (det, _, _), _, o = _run(ham, prm, 60, n_procs=4, ref_own_proc=True)
    assert o.proc_dets(0) == 1
    assert o.owner(int(ham.ref_det)) == 0
    assert all(o.owner(int(d)) >= 1 for d in det if int(d) != int(ham.ref_det))
    with pytest.raises(RuntimeError):
        O.Oracle(ham, prm, n_procs=1, ref_own_proc=True)


def test_process_hash_balances_determinants():
    """The process hash spreads determinants evenly (chi-squared over 8 processes)."""
    ham = S.synthetic_molecule(20, 5, 5, 2)
    P = 8
    o = O.Oracle(ham, S.Params(tau=0.01), n_procs=P, proc_seed=5)
    rng = np.random.default_rng(4)
    counts = np.zeros(P)
    seen = set()
    while len(seen) < 16000:
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
        counts[o.owner(d)] += 1
    from scipy import stats
    chi2 = ((counts - counts.mean()) ** 2 / counts.mean()).sum()
    assert stats.chi2.sf(chi2, P - 1) > 1e-4
    # the process map is not the main-list map: ownership and bucket differ
    owners = [o.owner(d) for d in list(seen)[:2000]]
    buckets = [o.hash(d, P) for d in list(seen)[:2000]]
    assert np.mean(np.array(owners) == np.array(buckets)) < 0.5


def test_snapshot_reload_across_process_counts():
    """A walker list written by one process count and loaded into another
    continues on the same trajectory."""
    ham, prm, _ = S.workload("hubbard8", scale=0.3)
    o1 = O.Oracle(ham, prm)
    o1.iterate(60)
    det, pop, _ = o1.walkers()
    e = o1.estimates()
    o3 = O.Oracle(ham, prm, n_procs=3, n_threads=3)
    o3.load_walkers(det, pop, iteration=e["iteration"], shift=e["shift"], n_prev=e["n_prev"],
                    varying=e["shift_varying"], n_var=e["n_var"])
    o1.iterate(30)
    o3.iterate(30)
    # run totals and the averaging series restart at a reload
    _same((o1.walkers(), o1.estimates(), o1), (o3.walkers(), o3.estimates(), o3), "reload",
          skip=("total_attempts", "total_spawns", "n_samples"))
