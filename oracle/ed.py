"""Exact diagonalisation in the determinant space (test infrastructure only).

The Hamiltonian matrix is built by *applying second-quantised operators* to
bit-string determinants,

    H = sum_pq h_pq a+_p a_q + 1/2 sum_pqrs (pq|rs) a+_p a+_r a_s a_q ,

over spin orbitals p = 2 s + sigma, with (pq|rs) nonzero only when p, q share a
spin and r, s share a spin. Fermionic signs come from the definition of the
operators on an ordered bit string (a_q on |D> gives (-1)^(number of occupied
orbitals below q)). This is the plain definition of the matrix that the
Slater-Condon rules evaluate, and of the ground-state energy that FCIQMC samples
(Sec. 2 of the paper); it shares no code with the oracle's Slater-Condon rules.
"""
from __future__ import annotations

import itertools

import numpy as np


def _pair(i, j):
    if i < j:
        i, j = j, i
    return i * (i + 1) // 2 + j


def unpack_eri(eri, m):
    """Full (m,m,m,m) spatial array from the eight-fold packed format."""
    g = np.zeros((m, m, m, m))
    for p, q, r, s in itertools.product(range(m), repeat=4):
        a, b = _pair(p, q), _pair(r, s)
        if a < b:
            a, b = b, a
        g[p, q, r, s] = eri[a * (a + 1) // 2 + b]
    return g


def determinants(m, n_alpha, n_beta):
    """All determinants with the given electron counts, sorted ascending."""
    dets = []
    for a in itertools.combinations(range(m), n_alpha):
        for b in itertools.combinations(range(m), n_beta):
            d = 0
            for s in a:
                d |= 1 << (2 * s)
            for s in b:
                d |= 1 << (2 * s + 1)
            dets.append(d)
    return np.array(sorted(dets), dtype=np.uint64)


def _below_parity(dets, p):
    """(-1)^(number of set bits below p), vectorised over determinants."""
    mask = np.uint64((1 << p) - 1)
    x = dets & mask
    cnt = np.zeros(len(dets), dtype=np.int64)
    for b in range(p):
        cnt += ((x >> np.uint64(b)) & np.uint64(1)).astype(np.int64)
    return np.where(cnt % 2 == 0, 1.0, -1.0)


def _annihilate(dets, sign, q):
    bit = np.uint64(1 << q)
    ok = (dets & bit) != 0
    return dets ^ bit, sign * _below_parity(dets, q) * ok


def _create(dets, sign, p):
    bit = np.uint64(1 << p)
    ok = (dets & bit) == 0
    return dets | bit, sign * _below_parity(dets, p) * ok


def build_hamiltonian(ham, dets=None):
    """Dense H in the basis ``dets`` (all determinants of the sector by default)."""
    m = ham.n_orb
    n_so = 2 * m
    if dets is None:
        dets = determinants(m, ham.n_alpha, ham.n_beta)
    dets = np.sort(np.asarray(dets, dtype=np.uint64))
    g = unpack_eri(np.asarray(ham.eri), m)
    h1 = np.asarray(ham.h1)
    dim = len(dets)
    H = np.zeros((dim, dim))
    H[np.arange(dim), np.arange(dim)] += ham.e_core
    cols = np.arange(dim)

    def scatter(new, sgn, val):
        nz = np.nonzero(sgn)[0]
        if len(nz) == 0:
            return
        rows = np.searchsorted(dets, new[nz])
        rows = np.minimum(rows, dim - 1)
        hit = dets[rows] == new[nz]
        np.add.at(H, (rows[hit], cols[nz][hit]), val * sgn[nz][hit])

    ones = np.ones(dim)
    for p in range(n_so):
        for q in range(n_so):
            if (p & 1) != (q & 1):
                continue
            v = h1[p >> 1, q >> 1]
            if v == 0.0:
                continue
            d1, s1 = _annihilate(dets, ones, q)
            d2, s2 = _create(d1, s1, p)
            scatter(d2, s2, v)
    for p, q, r, s in itertools.product(range(n_so), repeat=4):
        if (p & 1) != (q & 1) or (r & 1) != (s & 1):
            continue
        v = g[p >> 1, q >> 1, r >> 1, s >> 1]
        if v == 0.0:
            continue
        # a+_p a+_r a_s a_q, applied right to left
        d1, s1 = _annihilate(dets, ones, q)
        d2, s2 = _annihilate(d1, s1, s)
        d3, s3 = _create(d2, s2, r)
        d4, s4 = _create(d3, s3, p)
        scatter(d4, s4, 0.5 * v)
    return dets, H


def ground_state(ham):
    """(E_0, eigenvector, dets): dense diagonalisation for small spaces, Lanczos
    (scipy ``eigsh``) on the same matrix above 1500 determinants."""
    dets, H = build_hamiltonian(ham)
    if len(dets) <= 1500:
        w, v = np.linalg.eigh(H)
        return w[0], v[:, 0], dets
    import scipy.sparse as sp
    import scipy.sparse.linalg as sla
    w, v = sla.eigsh(sp.csr_matrix(H), k=1, which="SA", tol=1e-13)
    return w[0], v[:, 0], dets
