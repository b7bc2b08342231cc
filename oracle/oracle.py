"""ctypes binding to the C oracle (test infrastructure only)."""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None


class OrcHam(C.Structure):
    _fields_ = [("n_orb", C.c_int32), ("n_alpha", C.c_int32), ("n_beta", C.c_int32),
                ("pad0", C.c_int32), ("e_core", C.c_double),
                ("h1", C.POINTER(C.c_double)), ("eri", C.POINTER(C.c_double)),
                ("orb_irrep", C.POINTER(C.c_uint8)), ("p_double", C.c_double),
                ("ref_det", C.POINTER(C.c_uint64))]


class OrcParams(C.Structure):
    _fields_ = [("tau", C.c_double), ("zeta", C.c_double), ("shift0", C.c_double),
                ("shift_every", C.c_int32), ("n_a", C.c_int32),
                ("target", C.c_int64), ("n_init", C.c_int64), ("seed", C.c_uint64),
                ("avg_start", C.c_int32), ("pad0", C.c_int32),
                ("hash_seed", C.c_uint64), ("hash_range", C.c_int64),
                ("n_procs", C.c_int32), ("ref_own_proc", C.c_int32),
                ("proc_seed", C.c_uint64), ("n_threads", C.c_int32),
                ("space", C.c_int32), ("max_excitation", C.c_int32), ("max_seniority", C.c_int32),
                ("hphf", C.c_int32), ("frozen_occupied", C.c_uint64),
                ("frozen_empty", C.c_uint64), ("frozen_occupied_hi", C.c_uint64),
                ("frozen_empty_hi", C.c_uint64), ("det_words", C.c_int32), ("pad1", C.c_int32)]


class OrcEst(C.Structure):
    _fields_ = [(n, C.c_int64) for n in
                ("iteration", "n_walkers", "n_dets", "ref_pop", "attempts", "spawns",
                 "merged", "aborted", "total_attempts", "total_spawns", "n_samples", "n_var")] + \
               [(n, C.c_double) for n in
                ("shift", "e_ref", "p_double", "proj_num", "e_proj_inst", "e_proj_mean",
                 "e_proj_err", "shift_mean", "shift_err")] + \
               [("shift_varying", C.c_int32), ("pad0", C.c_int32), ("n_prev", C.c_int64),
                ("born", C.c_int64)]


def lib():
    global _LIB
    if _LIB is None:
        path = os.path.join(HERE, "liboracle.so")
        if not os.path.exists(path):
            from . import build as _b
            _b.build()
        L = C.CDLL(path)
        vp = C.c_void_p
        L.orc_create.argtypes = [C.POINTER(OrcHam), C.POINTER(OrcParams), C.POINTER(vp)]
        L.orc_iterate.argtypes = [vp, C.c_int32]
        L.orc_estimates.argtypes = [vp, C.POINTER(OrcEst)]
        L.orc_walkers.argtypes = [vp, vp, vp, vp, C.c_int64]
        L.orc_walkers.restype = C.c_int64
        L.orc_load_walkers.argtypes = [vp, vp, vp, C.c_int64, C.c_int64, C.c_double,
                                       C.c_int64, C.c_int32, C.c_int64]
        L.orc_free.argtypes = [vp]
        L.orc_last_error.restype = C.c_char_p
        L.orc_philox4x32_10.argtypes = [vp, vp, vp]
        L.orc_decode.argtypes = [vp, C.c_int32, vp]
        L.orc_hash.argtypes = [vp, vp, C.c_int64]
        L.orc_hash.restype = C.c_int64
        L.orc_proc_dets.argtypes = [vp, C.c_int32]
        L.orc_proc_dets.restype = C.c_int64
        L.orc_owner.argtypes = [vp, vp]
        L.orc_owner.restype = C.c_int32
        L.orc_det_words.argtypes = [vp]
        L.orc_det_words.restype = C.c_int32
        L.orc_hel.argtypes = [vp, vp, vp]
        L.orc_hel.restype = C.c_double
        L.orc_hdiag.argtypes = [vp, vp]
        L.orc_hdiag.restype = C.c_double
        L.orc_proj_num.argtypes = [vp, vp, vp, C.c_int64]
        L.orc_proj_num.restype = C.c_double
        L.orc_sample_excitations.argtypes = [vp, vp, C.c_int64, C.c_int64, vp, vp, vp]
        L.orc_pgen.argtypes = [vp, vp, vp]
        L.orc_pgen.restype = C.c_double
        L.orc_fn_hel.argtypes = [vp, vp, vp]
        L.orc_fn_hel.restype = C.c_double
        L.orc_fn_diag.argtypes = [vp, vp]
        L.orc_fn_diag.restype = C.c_double
        L.orc_blocking.argtypes = [vp, vp, C.c_int64, C.POINTER(C.c_double),
                                   C.POINTER(C.c_double), C.POINTER(C.c_int32)]
        _LIB = L
    return _LIB


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


def philox4x32_10(ctr, key):
    c = np.asarray(ctr, dtype=np.uint32)
    k = np.asarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().orc_philox4x32_10(_ptr(c), _ptr(k), _ptr(out))
    return out


MASK64 = (1 << 64) - 1


def words_of(det: int, w: int) -> np.ndarray:
    """A determinant (Python int) as w 64-bit words, low word first."""
    return np.array([(int(det) >> (64 * i)) & MASK64 for i in range(w)], dtype=np.uint64)


def det_array(dets, w: int) -> np.ndarray:
    """Determinants as the API's array: shape (n,) for one word, (n, 2) for two
    (columns: low word, high word). Accepts ints or an array already in shape."""
    a = np.asarray(dets)
    if w == 1:
        return np.ascontiguousarray(a, dtype=np.uint64).reshape(-1)
    if a.ndim == 2:
        return np.ascontiguousarray(a, dtype=np.uint64)
    if a.dtype == np.uint64:     # one-word values: a zero high word
        return np.ascontiguousarray(np.stack([a.reshape(-1), np.zeros(a.size, np.uint64)], axis=1))
    return np.array([[int(d) & MASK64, int(d) >> 64] for d in a.reshape(-1)],
                    dtype=np.uint64).reshape(-1, 2)


def det_ints(arr) -> list:
    """Python ints from the API's determinant array (either shape)."""
    a = np.asarray(arr)
    if a.ndim == 1:
        return [int(x) for x in a]
    return [int(lo) | (int(hi) << 64) for lo, hi in a]


def decode(det: int):
    occ = np.zeros(128, dtype=np.int32)
    n = lib().orc_decode(_ptr(words_of(det, 2)), 2, _ptr(occ))
    return occ[:n].tolist()


def blocking(num, den=None):
    num = np.ascontiguousarray(num, dtype=np.float64)
    d = None if den is None else np.ascontiguousarray(den, dtype=np.float64)
    mean, err, lvl = C.c_double(), C.c_double(), C.c_int32()
    lib().orc_blocking(_ptr(num), _ptr(d), len(num), C.byref(mean), C.byref(err), C.byref(lvl))
    return mean.value, err.value, lvl.value


class Oracle:
    """One FCIQMC run on the CPU.

    By default one main list on one thread. With ``n_procs`` > 1 the
    determinants are distributed over that many virtual processes by the
    process hash of Sec. 4.1 (``ref_own_proc``: the reference alone on process
    0), which run on ``n_threads`` host threads."""

    def __init__(self, ham, params, hash_seed: int = 0, hash_range: int = 0,
                 n_procs: int = 1, ref_own_proc: bool = False, proc_seed: int = 0,
                 n_threads: int = 1):
        L = lib()
        self._h1 = np.ascontiguousarray(ham.h1, dtype=np.float64)
        self._eri = np.ascontiguousarray(ham.eri, dtype=np.float64)
        self._irr = None if ham.orb_irrep is None else np.ascontiguousarray(ham.orb_irrep, np.uint8)
        self._ref = None if ham.ref_det is None else words_of(ham.ref_det, 2)
        h = OrcHam(ham.n_orb, ham.n_alpha, ham.n_beta, 0, ham.e_core,
                   self._h1.ctypes.data_as(C.POINTER(C.c_double)),
                   self._eri.ctypes.data_as(C.POINTER(C.c_double)),
                   None if self._irr is None else self._irr.ctypes.data_as(C.POINTER(C.c_uint8)),
                   ham.p_double,
                   None if self._ref is None else self._ref.ctypes.data_as(C.POINTER(C.c_uint64)))
        p = OrcParams(params.tau, params.shift_damping, params.initial_shift,
                      params.shift_update_every, params.initiator_threshold,
                      params.target_walkers, params.initial_walkers, params.seed,
                      params.avg_start, 0, hash_seed, hash_range, n_procs,
                      int(bool(ref_own_proc)), proc_seed, n_threads, params.space,
                      params.max_excitation, params.max_seniority, params.hphf,
                      int(params.frozen_occupied) & MASK64, int(params.frozen_empty) & MASK64,
                      int(params.frozen_occupied) >> 64, int(params.frozen_empty) >> 64,
                      getattr(params, "det_words", 0), 0)
        self._h = C.c_void_p()
        if L.orc_create(C.byref(h), C.byref(p), C.byref(self._h)) != 0:
            raise RuntimeError(L.orc_last_error().decode())
        self.n_elec = ham.n_alpha + ham.n_beta
        self.W = L.orc_det_words(self._h)

    def close(self):
        if self._h:
            lib().orc_free(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc):
        if rc != 0:
            raise RuntimeError(lib().orc_last_error().decode())

    def iterate(self, n: int = 1):
        self._check(lib().orc_iterate(self._h, n))

    def estimates(self) -> dict:
        e = OrcEst()
        self._check(lib().orc_estimates(self._h, C.byref(e)))
        return {f[0]: getattr(e, f[0]) for f in OrcEst._fields_ if f[0] != "pad0"}

    def _w(self, det: int) -> np.ndarray:
        return words_of(det, self.W)

    def walkers(self):
        """(det, pop, flags) sorted by determinant; det has shape (n,) with one word
        per determinant, (n, 2) with two."""
        n = lib().orc_walkers(self._h, None, None, None, 0)
        det = np.zeros(max(n, 1) * self.W, dtype=np.uint64)
        pop = np.zeros(max(n, 1), dtype=np.int32)
        flg = np.zeros(max(n, 1), dtype=np.uint32)
        m = lib().orc_walkers(self._h, _ptr(det), _ptr(pop), _ptr(flg), n)
        if m < 0:
            raise RuntimeError(lib().orc_last_error().decode())
        det = det[:n * self.W]
        return (det if self.W == 1 else det.reshape(-1, 2)), pop[:n], flg[:n]

    def load_walkers(self, det, pop, iteration=0, shift=0.0, n_prev=0, varying=0, n_var=0):
        det = det_array(det, self.W)
        pop = np.ascontiguousarray(pop, dtype=np.int32)
        self._check(lib().orc_load_walkers(self._h, _ptr(det), _ptr(pop), len(pop), iteration,
                                           shift, n_prev, varying, n_var))

    def hel(self, bra: int, ket: int) -> float:
        return lib().orc_hel(self._h, _ptr(self._w(bra)), _ptr(self._w(ket)))

    def hdiag(self, det: int) -> float:
        return lib().orc_hdiag(self._h, _ptr(self._w(det)))

    def proc_dets(self, p: int) -> int:
        n = lib().orc_proc_dets(self._h, p)
        if n < 0:
            raise RuntimeError(lib().orc_last_error().decode())
        return n

    def owner(self, det: int) -> int:
        return lib().orc_owner(self._h, _ptr(self._w(det)))

    def hash(self, det: int, rng: int) -> int:
        return lib().orc_hash(self._h, _ptr(self._w(det)), rng)

    def proj_num(self, det, c) -> float:
        det = det_array(det, self.W)
        c = np.ascontiguousarray(c, dtype=np.float64)
        return lib().orc_proj_num(self._h, _ptr(det), _ptr(c), len(c))

    def fn_hel(self, bra: int, ket: int) -> float:
        """<bra|H|ket> between stored functions of the run, ket the source."""
        return lib().orc_fn_hel(self._h, _ptr(self._w(bra)), _ptr(self._w(ket)))

    def fn_diag(self, fn: int) -> float:
        return lib().orc_fn_diag(self._h, _ptr(self._w(fn)))

    def pgen(self, det: int, target: int) -> float:
        """Probability that the excitation generator produces target from det."""
        return lib().orc_pgen(self._h, _ptr(self._w(det)), _ptr(self._w(target)))

    def sample_excitations(self, det: int, n: int, iteration: int = 0):
        """(children, pgen, element) of n attempts; children as Python ints when the
        determinants take two words."""
        od = np.zeros(n * self.W, dtype=np.uint64)
        pg = np.zeros(n)
        he = np.zeros(n)
        self._check(lib().orc_sample_excitations(self._h, _ptr(self._w(det)), iteration, n,
                                                 _ptr(od), _ptr(pg), _ptr(he)))
        return (od if self.W == 1 else det_ints(od.reshape(-1, 2))), pg, he
