"""Seeded synthetic inputs: Hamiltonians in the packed integral format and the
run parameters of the five benchmark workloads.

This module only *generates inputs*. It holds none of the FCIQMC arithmetic
(no matrix elements, excitation generation, pgen, hashing or dynamics), so that
both the HIP path and the CPU oracle can be driven from the same seeded data
without sharing any part of the method.

Integral format (the C ABI's input, Sec. 2 of the paper: one-electron h_pq and
two-electron (pq|rs) in chemists' notation, stored with the eight-fold
permutational packing mentioned in the Sec. 2 footnote):

* ``h1``: M x M row-major float64, symmetric.
* ``eri``: packed float64. Pair index ``ij = i(i+1)/2 + j`` for ``i >= j``;
  element index ``IJ(IJ+1)/2 + KL`` for ``IJ >= KL``.
* spin orbital ``p = 2*s + sigma`` (s spatial, sigma 0 = alpha, 1 = beta); a
  determinant is a uint64 with bit p set when p is occupied.

Recipes
-------
* Hubbard ring: h_{s,s+-1 mod L} = -t, (ss|ss) = U, everything else zero; Neel
  reference (alpha on even sites, beta on odd sites); singles only.
* Synthetic molecule: h_pp = orbital energies (evenly spaced in [-2, 2] unless a
  band layout is given), off-diagonal h_pq ~ N(0, 0.05);
  (pq|rs) ~ N(0, 0.1) * exp(-(|p-q| + |r-s|)/3) for canonical p>=q, r>=s,
  pq>=rs, and (pp|qq) ~ U[0.3, 0.8] (p = q included). The second argument of
  N(.,.) is the standard deviation.
* Transition-metal-dimer-shaped band (24e/30o): orbitals 0-5 evenly in
  [-2, -0.3], 6-17 evenly in [-0.2, 0.2] (a near-degenerate band of 12 orbitals
  straddling the Fermi level), 18-29 evenly in [0.3, 2].
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "Hamiltonian", "Params", "hubbard_ring", "synthetic_molecule",
    "band_energies", "npair", "n_eri", "aufbau_det", "neel_det",
    "workload", "batch_workload", "serve_requests",
    "SPACE_EXCITATION", "SPACE_SENIORITY", "SPACE_FROZEN", "cas_masks",
]

# Restricted-space conditions (combined with a bitwise OR in Params.space).
SPACE_EXCITATION = 1   # at most max_excitation electrons moved away from the reference
SPACE_SENIORITY = 2    # at most max_seniority singly occupied spatial orbitals
SPACE_FROZEN = 4       # frozen_occupied spin orbitals filled, frozen_empty ones empty


def cas_masks(n_core: int, n_active: int, n_orb: int):
    """(frozen_occupied, frozen_empty) spin-orbital masks of a complete active space:
    the n_core lowest spatial orbitals doubly occupied, the next n_active free, the
    rest empty (orbitals in the given order)."""
    core = (1 << (2 * n_core)) - 1
    used = (1 << (2 * (n_core + n_active))) - 1
    full = (1 << (2 * n_orb)) - 1
    return core, full & ~used


def npair(m: int) -> int:
    return m * (m + 1) // 2


def n_eri(m: int) -> int:
    p = npair(m)
    return p * (p + 1) // 2


@dataclass
class Hamiltonian:
    """Host-side Hamiltonian description, mirroring ``fciqmc_hamiltonian``."""
    n_orb: int
    n_alpha: int
    n_beta: int
    e_core: float
    h1: np.ndarray                  # (M, M) float64
    eri: np.ndarray                 # packed float64
    orb_irrep: np.ndarray | None = None   # uint8 per spatial orbital, or None (C1)
    p_double: float = -1.0          # < 0: derive from the reference determinant
    ref_det: int | None = None      # None: aufbau by h_pp
    name: str = ""

    @property
    def n_elec(self) -> int:
        return self.n_alpha + self.n_beta


@dataclass
class Params:
    """Run parameters, mirroring ``fciqmc_params``."""
    tau: float
    shift_damping: float = 0.05
    initial_shift: float = 0.0
    shift_update_every: int = 10
    initiator_threshold: int = 0
    target_walkers: int = 10_000
    initial_walkers: int = 10
    det_capacity: int = 0
    spawn_capacity: int = 0
    seed: int = 1
    avg_start: int = 0
    # restricted space: a bitwise OR of SPACE_* (0: the full space) and its limits
    space: int = 0
    max_excitation: int = 0
    max_seniority: int = 0
    frozen_occupied: int = 0
    frozen_empty: int = 0
    # spin-coupled functions: 0 off, +1 / -1 for even / odd total spin
    hphf: int = 0
    # 64-bit words per determinant: 0 as the spin orbitals need (1 up to 64, 2 up to
    # 128); 2 forces two words for fewer
    det_words: int = 0
    extra: dict = field(default_factory=dict)


def _canonical_index_arrays(m: int):
    """(p, q, r, s) for every packed element, in packed order."""
    pi, qi = [], []
    for p in range(m):
        for q in range(p + 1):
            pi.append(p)
            qi.append(q)
    pi = np.asarray(pi, dtype=np.int64)
    qi = np.asarray(qi, dtype=np.int64)
    npq = len(pi)
    ij, kl = [], []
    for a in range(npq):
        ij.extend([a] * (a + 1))
        kl.extend(range(a + 1))
    ij = np.asarray(ij, dtype=np.int64)
    kl = np.asarray(kl, dtype=np.int64)
    return pi[ij], qi[ij], pi[kl], qi[kl]


def neel_det(n_sites: int) -> int:
    """Alpha on even sites, beta on odd sites."""
    d = 0
    for s in range(n_sites):
        sigma = 0 if s % 2 == 0 else 1
        d |= 1 << (2 * s + sigma)
    return d


def aufbau_det(orb_energy, n_alpha: int, n_beta: int) -> int:
    """Lowest n_alpha alpha and n_beta beta orbitals by energy (ties: lower index)."""
    order = sorted(range(len(orb_energy)), key=lambda s: (orb_energy[s], s))
    d = 0
    for s in order[:n_alpha]:
        d |= 1 << (2 * s)
    for s in order[:n_beta]:
        d |= 1 << (2 * s + 1)
    return d


def hubbard_ring(n_sites: int, u: float, t: float = 1.0, n_alpha: int | None = None,
                 n_beta: int | None = None) -> Hamiltonian:
    """Real-space 1D Hubbard ring with periodic boundaries at half filling."""
    m = n_sites
    if n_alpha is None:
        n_alpha = (m + 1) // 2
    if n_beta is None:
        n_beta = m // 2
    h1 = np.zeros((m, m))
    for s in range(m):
        nb = (s + 1) % m
        h1[s, nb] = -t
        h1[nb, s] = -t
    eri = np.zeros(n_eri(m))
    for s in range(m):
        ss = s * (s + 1) // 2 + s
        eri[ss * (ss + 1) // 2 + ss] = u
    ref = neel_det(m) if (n_alpha == (m + 1) // 2 and n_beta == m // 2) else None
    return Hamiltonian(m, n_alpha, n_beta, 0.0, h1, eri, None, 0.0, ref,
                       name=f"hubbard{m}_U{u:g}")


def band_energies(m: int) -> np.ndarray:
    """24e/30o-style layout: a 12-orbital band inside +-0.2 Ha at the Fermi level."""
    if m != 30:
        raise ValueError("the band layout is defined for 30 orbitals")
    return np.concatenate([np.linspace(-2.0, -0.3, 6), np.linspace(-0.2, 0.2, 12),
                           np.linspace(0.3, 2.0, 12)])


def synthetic_molecule(m: int, n_alpha: int, n_beta: int, seed: int,
                       orb_energy: np.ndarray | None = None,
                       irreps: np.ndarray | None = None) -> Hamiltonian:
    """Seeded random FP64 integrals with eight-fold symmetry (recipe in the module doc)."""
    rng = np.random.default_rng(seed)
    eps = np.linspace(-2.0, 2.0, m) if orb_energy is None else np.asarray(orb_energy, float)
    h1 = np.diag(eps).astype(np.float64)
    off = rng.normal(0.0, 0.05, size=m * (m - 1) // 2)
    k = 0
    for p in range(1, m):
        for q in range(p):
            h1[p, q] = h1[q, p] = off[k]
            k += 1
    p, q, r, s = _canonical_index_arrays(m)
    gauss = rng.normal(0.0, 0.1, size=len(p))
    unif = rng.uniform(0.3, 0.8, size=len(p))
    eri = gauss * np.exp(-(np.abs(p - q) + np.abs(r - s)) / 3.0)
    coul = (p == q) & (r == s)
    eri[coul] = unif[coul]
    if irreps is not None:
        # Zero the elements forbidden by an abelian point group (product = XOR).
        irr = np.asarray(irreps, dtype=np.int64)
        allowed = (irr[p] ^ irr[q] ^ irr[r] ^ irr[s]) == 0
        eri[~allowed] = 0.0
        for a in range(m):
            for b in range(m):
                if irr[a] != irr[b]:
                    h1[a, b] = 0.0
    ref = aufbau_det(np.diag(h1), n_alpha, n_beta)
    return Hamiltonian(m, n_alpha, n_beta, 0.0, h1, eri.astype(np.float64),
                       None if irreps is None else np.asarray(irreps, np.uint8),
                       -1.0, ref, name=f"synth{n_alpha + n_beta}e{m}o_s{seed}")


# ---------------------------------------------------------------------------
# The five benchmark workloads (seeds fixed here).
# ---------------------------------------------------------------------------

def workload(name: str, scale: float = 1.0):
    """Return (Hamiltonian, Params, info) for a named workload.

    ``scale`` multiplies the walker target (used by tests to shrink a workload
    while keeping its shape).
    """
    if name == "hubbard8":
        ham = hubbard_ring(8, 4.0)
        prm = Params(tau=0.01, shift_damping=0.05, shift_update_every=1,
                     initiator_threshold=0, target_walkers=int(1e4 * scale),
                     initial_walkers=10, seed=1, avg_start=500)
        return ham, prm, {"iterations": 2000, "seeds": list(range(1, 33))}
    if name == "synth10e20o":
        ham = synthetic_molecule(20, 5, 5, seed=2)
        prm = Params(tau=1e-3, shift_damping=0.05, shift_update_every=10,
                     initiator_threshold=3, target_walkers=int(1e7 * scale),
                     initial_walkers=10, seed=12, avg_start=0)
        return ham, prm, {"iterations": 1000}
    if name == "synth24e30o":
        ham = synthetic_molecule(30, 12, 12, seed=3, orb_energy=band_energies(30))
        prm = Params(tau=5e-4, shift_damping=0.05, shift_update_every=10,
                     initiator_threshold=3, target_walkers=int(1e8 * scale),
                     initial_walkers=10, seed=13, avg_start=0)
        return ham, prm, {"iterations": 20000}
    raise KeyError(name)


def batch_workload(scale: float = 1.0, n_hubbard: int = 32, n_synth: int = 32):
    """64 independent solves: Hubbard rings of 10-16 sites at half filling with
    U/t in [2, 8], and synthetic molecules from 10e/16o to 14e/26o. Walker
    targets are log-uniform in [1e4, 1e6]; Philox seeds 100, 101, ..."""
    rng = np.random.default_rng(4)
    out = []
    sizes = [10, 12, 14, 16]
    for i in range(n_hubbard):
        L = sizes[(i * len(sizes)) // max(n_hubbard, 1)]
        u = float(rng.uniform(2.0, 8.0))
        target = int(round(10 ** rng.uniform(4.0, 6.0) * scale))
        ham = hubbard_ring(L, u)
        prm = Params(tau=0.01, initiator_threshold=0, target_walkers=max(target, 20),
                     initial_walkers=10, seed=100 + i, shift_update_every=1)
        out.append((ham, prm))
    for i in range(n_synth):
        frac = i / max(n_synth - 1, 1)
        ne = 10 + 2 * int(round(2 * frac))          # 10, 12, 14 electrons
        m = 16 + int(round(10 * frac))              # 16 .. 26 orbitals
        target = int(round(10 ** rng.uniform(4.0, 6.0) * scale))
        ham = synthetic_molecule(m, ne // 2, ne // 2, seed=200 + i)
        prm = Params(tau=1e-3, initiator_threshold=3, target_walkers=max(target, 20),
                     initial_walkers=10, seed=100 + n_hubbard + i)
        out.append((ham, prm))
    return out


def serve_requests(n: int = 200, rate: float = 20.0, seed: int = 5, scale: float = 1.0):
    """Poisson request stream of solves of the three workload shapes: the 8-site
    Hubbard ring (U/t in [2, 8]), the synthetic 10e/20o molecule and the 24e/30o
    band molecule, drawn with equal probability. Walker targets are log-uniform
    in [1e4, 1e6], and in [1e6, 1e7] for the 24e/30o shape (shift damping 0.5
    there, 0.05 otherwise). Returns a list of
    (arrival_time_s, Hamiltonian, Params)."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for i in range(n):
        t += float(rng.exponential(1.0 / rate))
        kind = int(rng.integers(0, 3))
        lo, hi = (6.0, 7.0) if kind == 2 else (4.0, 6.0)
        target = int(round(10 ** rng.uniform(lo, hi) * scale))
        if kind == 0:
            ham = hubbard_ring(8, float(rng.uniform(2.0, 8.0)))
            prm = Params(tau=0.01, initiator_threshold=0, target_walkers=max(target, 20),
                         seed=1000 + i, shift_update_every=1)
        elif kind == 1:
            ham = synthetic_molecule(20, 5, 5, seed=300 + i)
            prm = Params(tau=1e-3, initiator_threshold=3, target_walkers=max(target, 20),
                         seed=1000 + i)
        else:
            # the dominant eigenvalue of this shape's initiator dynamics lies far below
            # E0: a strongly damped shift (gap x 0.5 per update) keeps the population
            # near its target instead of letting it grow many-fold first
            ham = synthetic_molecule(30, 12, 12, seed=300 + i, orb_energy=band_energies(30))
            prm = Params(tau=5e-4, initiator_threshold=3, target_walkers=max(target, 20),
                         seed=1000 + i, shift_damping=0.5)
        out.append((t, ham, prm))
    return out
