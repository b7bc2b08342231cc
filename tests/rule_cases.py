"""Hand-built walker lists whose next iteration is fixed by the rules alone.

A one-electron "star" system (one alpha electron in M = 5 spatial orbitals,
singles only): the determinants are the five alpha spin orbitals, and a single
excitation p -> a has H = h_pa (no other electron, no two-electron integral).
The one-electron integrals connect the hub T = orbital 0 to the chosen leaves
with h = -1 and nothing else; every diagonal element is 0 unless a case sets
one. With tau = 0.25 the generation probability of every single is 1/4, so a
spawn attempt that picks the hub spawns exactly tau |h| / pgen = 1 walker of
sign -sign(C) sign(h) = +sign(C), and an attempt that picks any other orbital
spawns nothing (H = 0). With all diagonals 0 and S = 0 there is no death.

These cases pin the initiator rule of the paper's Sec. 4.2 as read here:
a parent is an initiator iff |C| > n_a (strict) or it is the reference; the
flag of a merged spawn is the OR of its parents' flags; a determinant counts as
occupied when it is occupied after death. The spawn counts that the expected
outcomes add up come from runs in which only one parent is loaded (the random
numbers are keyed by determinant and walker ordinal, so a parent draws the
same numbers whatever else is loaded).
"""
from __future__ import annotations

import numpy as np

from paper_1305_6981_amd import systems as S

M = 5
N_A = 50           # initiator threshold of every case
TAU = 0.25
HUB, P1, P2, P3, REF = 0, 1, 2, 3, 4


def det(orb: int) -> int:
    """The determinant with the alpha electron in spatial orbital `orb`."""
    return 1 << (2 * orb)


def star(leaves=(P1, P2, P3), ref_linked=False, hub_diag=0.0) -> S.Hamiltonian:
    h1 = np.zeros((M, M))
    for j in leaves:
        h1[HUB, j] = h1[j, HUB] = -1.0
    if ref_linked:
        h1[HUB, REF] = h1[REF, HUB] = -1.0
    h1[HUB, HUB] = hub_diag
    return S.Hamiltonian(M, 1, 0, 0.0, h1, np.zeros(S.n_eri(M)), None, 0.0, det(REF),
                         name="star5")


def params(seed: int = 11, tau: float = TAU) -> S.Params:
    return S.Params(tau=tau, initiator_threshold=N_A, target_walkers=10**9, seed=seed,
                    shift_update_every=1)


def as_dict(walkers):
    d, p, _ = walkers
    return dict(zip((int(x) for x in d), (int(x) for x in p)))


def one_step(make, ham, entries, seed: int = 11, iteration: int = 0, tau: float = TAU):
    """Load `entries` [(orbital, population)], run one iteration; return the walker
    list as {det: pop} and the estimates."""
    run = make(ham, params(seed, tau))
    try:
        run.load_walkers(np.array([det(o) for o, _ in entries], np.uint64),
                         np.array([p for _, p in entries], np.int32), iteration=iteration)
        run.iterate(1)
        return as_dict(run.walkers()), run.estimates()
    finally:
        run.close()


def check_threshold_is_strict(make):
    """|C| = n_a: not an initiator, its spawns onto the empty hub are discarded;
    |C| = n_a + 1: an initiator, they survive. Both signs of C."""
    ham = star(leaves=(P1,))
    for sign in (1, -1):
        w, e = one_step(make, ham, [(P1, sign * N_A), (REF, 10)])
        assert e["spawns"] > 0
        assert det(HUB) not in w
        assert e["aborted"] == e["spawns"]          # one walker per spawn, all onto the hub
        assert e["born"] == 0
        assert w[det(P1)] == sign * N_A and w[det(REF)] == 10
        w, e = one_step(make, ham, [(P1, sign * (N_A + 1)), (REF, 10)])
        assert e["spawns"] > 0 and e["aborted"] == 0
        assert w[det(HUB)] == sign * e["spawns"]     # spawned sign: -sign(C) sign(h) = sign(C)
        assert e["merged"] == 1 and e["born"] == 1


def _alone(make, ham, leaf, pop):
    w, e = one_step(make, ham, [(leaf, pop), (REF, 10)])
    assert e["spawns"] > 0
    return e["spawns"]


def check_flags_are_ored(make):
    """Two non-initiator parents and one initiator spawn onto the empty hub: the
    merged record carries the initiator flag (OR), so all their walkers survive;
    without the initiator everything is discarded."""
    ham = star()
    c1 = _alone(make, ham, P1, N_A)
    c2 = _alone(make, ham, P2, N_A)
    c3 = _alone(make, ham, P3, N_A + 1)
    w, e = one_step(make, ham, [(P1, N_A), (P2, N_A), (P3, N_A + 1), (REF, 10)])
    assert e["spawns"] == c1 + c2 + c3
    assert e["aborted"] == 0 and e["born"] == 1
    assert w[det(HUB)] == c1 + c2 + c3
    # signed sum: the second non-initiator parent negative
    w, e = one_step(make, ham, [(P1, N_A), (P2, -N_A), (P3, N_A + 1), (REF, 10)])
    assert e["aborted"] == 0
    assert w.get(det(HUB), 0) == c1 - c2 + c3
    # no initiator parent: the whole merged record is discarded
    w, e = one_step(make, ham, [(P1, N_A), (P2, N_A), (REF, 10)])
    assert det(HUB) not in w
    assert e["aborted"] == c1 + c2 and e["born"] == 0


def check_occupancy_after_death(make):
    """The hub holds one walker that death removes in the same iteration
    (tau (H_TT - E0 - S) |C| = 0.25 * 4 * 1 = 1 exactly). Spawns onto it from a
    non-initiator are then discarded, and an initiator's spawns re-occupy it with
    their sum alone."""
    ham = star(leaves=(P1,), hub_diag=4.0)
    c = _alone(make, ham, P1, N_A)
    w, e = one_step(make, ham, [(P1, N_A), (HUB, 1), (REF, 10)])
    assert det(HUB) not in w
    assert e["aborted"] == c
    assert w[det(P1)] in (N_A, N_A + 1)       # plus the hub's own attempt, if it picked P1
    ci = _alone(make, ham, P1, N_A + 1)
    w, e = one_step(make, ham, [(P1, N_A + 1), (HUB, 1), (REF, 10)])
    assert e["aborted"] == 0 and e["born"] == 1      # emptied by death, then re-entered
    assert w[det(HUB)] == ci


def check_reference_is_always_initiator(make):
    """The reference spawns with the initiator flag at any population."""
    ham = star(leaves=(), ref_linked=True)
    w, e = one_step(make, ham, [(REF, N_A)])
    assert e["spawns"] > 0 and e["aborted"] == 0
    assert w[det(HUB)] == e["spawns"]


def check_multi_walker_spawns(make):
    """tau |h| / pgen above 1 (Eq. pspawn): tau = 0.5 gives exactly 2 walkers per
    spawn onto the hub, tau = 0.6 gives 2 or 3 (2 + Bernoulli(0.4))."""
    ham = star(leaves=(P1,))
    w, e = one_step(make, ham, [(P1, N_A + 1), (REF, 10)], tau=0.5)
    assert e["spawns"] > 0 and w[det(HUB)] == 2 * e["spawns"]
    w, e = one_step(make, ham, [(P1, -(N_A + 1)), (REF, 10)], tau=0.6)
    n = e["spawns"]
    assert n > 0 and -3 * n < w[det(HUB)] < -2 * n    # some 3s, not all (P = 0.4 each)


def check_shift_schedule(make, ham, prm, n_iter):
    """Shift update of Sec. 2 with A = prm.shift_update_every, checked against the
    formula evaluated by hand (math.log) on the recorded populations: S is held
    until, at a multiple of A, N_w >= target; from then on, at every multiple of A,
    S <- S - zeta / (A tau) ln(N_w / N_prev) and N_prev <- N_w; between multiples
    S and N_prev do not change."""
    import math
    A, tau, zeta = prm.shift_update_every, prm.tau, prm.shift_damping
    run = make(ham, prm)
    try:
        prev = run.estimates()
        hist = []
        for _ in range(n_iter):
            run.iterate(1)
            e = run.estimates()
            hist.append(e)
            n = e["iteration"]
            if not prev["shift_varying"]:
                if n % A == 0 and e["n_walkers"] >= prm.target_walkers:
                    assert e["shift_varying"] == 1 and e["n_var"] == n
                    assert e["n_prev"] == e["n_walkers"]
                else:
                    assert e["shift_varying"] == 0
                assert e["shift"] == prm.initial_shift
            elif n % A == 0:
                want = prev["shift"] - zeta / (A * tau) * math.log(e["n_walkers"] / prev["n_prev"])
                assert abs(e["shift"] - want) <= 1e-13 * max(1.0, abs(want)), (n, e["shift"], want)
                assert e["n_prev"] == e["n_walkers"]
            else:
                assert e["shift"] == prev["shift"] and e["n_prev"] == prev["n_prev"]
            prev = e
    finally:
        run.close()
    updates = [e for e in hist if e["shift_varying"] and e["iteration"] % A == 0
               and e["iteration"] > e["n_var"]]
    assert hist[0]["shift_varying"] == 0 and len(updates) >= 3
    return hist
