"""ctypes binding to libfciqmc.so: the calls of include/fciqmc.h with the same
names. Argument marshalling only -- every step of the iteration runs in the
library's HIP kernels. There is no fallback: without the built library (or a
GPU) every call raises."""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfciqmc.so")
_LIB = None

FCIQMC_ERRORS = {-1: "EINVAL", -2: "ENOMEM", -3: "EDEVICE", -4: "ECAPACITY", -5: "EOVERFLOW",
                 -6: "ESTATE"}


class FciqmcError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{FCIQMC_ERRORS.get(code, code)}: {msg}")
        self.code = code


class Hamiltonian(C.Structure):
    _fields_ = [("n_orb", C.c_int32), ("n_alpha", C.c_int32), ("n_beta", C.c_int32),
                ("reserved0", C.c_int32), ("e_core", C.c_double),
                ("h1", C.POINTER(C.c_double)), ("eri", C.POINTER(C.c_double)),
                ("orb_irrep", C.POINTER(C.c_uint8)), ("p_double", C.c_double),
                ("ref_det", C.POINTER(C.c_uint64))]


class Params(C.Structure):
    _fields_ = [("tau", C.c_double), ("shift_damping", C.c_double),
                ("initial_shift", C.c_double), ("shift_update_every", C.c_int32),
                ("initiator_threshold", C.c_int32), ("target_walkers", C.c_int64),
                ("initial_walkers", C.c_int64), ("det_capacity", C.c_int64),
                ("spawn_capacity", C.c_int64), ("seed", C.c_uint64),
                ("avg_start", C.c_int32), ("space", C.c_int32),
                ("max_excitation", C.c_int32), ("max_seniority", C.c_int32),
                ("frozen_occupied", C.c_uint64), ("frozen_empty", C.c_uint64),
                ("hphf", C.c_int32), ("reserved1", C.c_int32),
                ("frozen_occupied_hi", C.c_uint64), ("frozen_empty_hi", C.c_uint64),
                ("det_words", C.c_int32), ("reserved2", C.c_int32)]


_EST_INT = ("iteration", "n_walkers", "n_dets", "ref_pop", "attempts", "spawns", "merged",
            "aborted", "total_attempts", "total_spawns", "n_samples", "n_var", "n_prev",
            "table_slots", "table_used")
_EST_DBL = ("shift", "e_ref", "p_double", "proj_num", "e_proj_inst", "e_proj_mean",
            "e_proj_err", "shift_mean", "shift_err", "ms_last_call")


class Estimates(C.Structure):
    _fields_ = [(n, C.c_int64) for n in _EST_INT] + [(n, C.c_double) for n in _EST_DBL] + \
               [("shift_varying", C.c_int32), ("status", C.c_int32), ("redos", C.c_int64),
                ("spills", C.c_int64)] + \
               [(n, C.c_double) for n in ("ms_spawn", "ms_death", "ms_annihilate",
                                          "ms_estimators")] + [("born", C.c_int64)]


class Iteration(C.Structure):
    _fields_ = [(n, C.c_int64) for n in
                ("iteration", "n_walkers", "n_dets", "ref_pop", "attempts", "spawns", "merged",
                 "aborted", "born", "entries")] + \
               [("proj_num", C.c_double), ("shift", C.c_double),
                ("shift_varying", C.c_int32), ("status", C.c_int32)]


EXPORTED = ["fciqmc_init", "fciqmc_iterate", "fciqmc_estimators", "fciqmc_free",
            "fciqmc_walkers", "fciqmc_load_walkers", "fciqmc_set_shift", "fciqmc_reserve",
            "fciqmc_last_error",
            "fciqmc_batch_create", "fciqmc_batch_iterate", "fciqmc_batch_iterate_each",
            "fciqmc_batch_admit", "fciqmc_batch_retire", "fciqmc_batch_slot_estimators",
            "fciqmc_batch_slot_walkers", "fciqmc_footprint_bytes", "fciqmc_batch_active",
            "fciqmc_set_profiling", "fciqmc_kernel_times", "fciqmc_set_launch",
            "fciqmc_get_launch", "fciqmc_autotune", "fciqmc_blocking",
            "fciqmc_set_test_options", "fciqmc_walkers_noalloc", "fciqmc_history",
            "fciqmc_det_words"]


def lib():
    """Load libfciqmc.so (raises if it has not been built)."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise FileNotFoundError(f"{LIB_PATH} is missing: run __graft_entry__.build()")
        L = C.CDLL(LIB_PATH)
        vp, i32, i64 = C.c_void_p, C.c_int32, C.c_int64
        H, P, E = C.POINTER(Hamiltonian), C.POINTER(Params), C.POINTER(Estimates)
        sig = {
            "fciqmc_init": ([H, P, vp, C.POINTER(vp)], C.c_int),
            "fciqmc_iterate": ([vp, i32], C.c_int),
            "fciqmc_estimators": ([vp, E], C.c_int),
            "fciqmc_free": ([vp], C.c_int),
            "fciqmc_walkers": ([vp, vp, vp, vp, i64], i64),
            "fciqmc_load_walkers": ([vp, vp, vp, i64, i64, C.c_double, i64, i32, i64], C.c_int),
            "fciqmc_set_shift": ([vp, C.c_double, i32], C.c_int),
            "fciqmc_reserve": ([vp, C.c_int64], C.c_int),
            "fciqmc_last_error": ([], C.c_char_p),
            "fciqmc_batch_create": ([i32, i32, H, P, vp, C.POINTER(vp)], C.c_int),
            "fciqmc_batch_iterate": ([vp, i32], C.c_int),
            "fciqmc_batch_iterate_each": ([vp, vp], C.c_int),
            "fciqmc_batch_admit": ([vp, H, P, C.POINTER(i32)], C.c_int),
            "fciqmc_batch_retire": ([vp, i32], C.c_int),
            "fciqmc_batch_slot_estimators": ([vp, i32, E], C.c_int),
            "fciqmc_batch_slot_walkers": ([vp, i32, vp, vp, vp, i64], i64),
            "fciqmc_footprint_bytes": ([H, P], i64),
            "fciqmc_batch_active": ([vp], i32),
            "fciqmc_set_profiling": ([vp, i32], C.c_int),
            "fciqmc_kernel_times": ([vp, vp, vp], C.c_int),
            "fciqmc_set_launch": ([vp, i32, i32, i32], C.c_int),
            "fciqmc_get_launch": ([vp, C.POINTER(i32), C.POINTER(i32), C.POINTER(i32)], C.c_int),
            "fciqmc_autotune": ([vp, i32], C.c_int),
            "fciqmc_blocking": ([vp, vp, i64, C.POINTER(C.c_double), C.POINTER(C.c_double)],
                                C.c_int),
            "fciqmc_set_test_options": ([vp, i32, i64, i64], C.c_int),
            "fciqmc_walkers_noalloc": ([vp, vp, vp, vp, i64], i64),
            "fciqmc_history": ([vp, i32, i64, i64, C.POINTER(Iteration)], i64),
            "fciqmc_det_words": ([vp], i32),
        }
        for name, (args, res) in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _LIB = L
    return _LIB


def _check(rc):
    if rc < 0:
        raise FciqmcError(int(rc), lib().fciqmc_last_error().decode())
    return rc


class _Keep:
    """Host arrays referenced by a marshalled Hamiltonian (kept alive for the call)."""


def marshal_hamiltonian(ham):
    k = _Keep()
    k.h1 = np.ascontiguousarray(ham.h1, dtype=np.float64)
    k.eri = np.ascontiguousarray(ham.eri, dtype=np.float64)
    k.irr = None if ham.orb_irrep is None else np.ascontiguousarray(ham.orb_irrep, dtype=np.uint8)
    k.ref = None if ham.ref_det is None else det_words_of(ham.ref_det)
    h = Hamiltonian(ham.n_orb, ham.n_alpha, ham.n_beta, 0, ham.e_core,
                    k.h1.ctypes.data_as(C.POINTER(C.c_double)),
                    k.eri.ctypes.data_as(C.POINTER(C.c_double)),
                    None if k.irr is None else k.irr.ctypes.data_as(C.POINTER(C.c_uint8)),
                    ham.p_double,
                    None if k.ref is None else k.ref.ctypes.data_as(C.POINTER(C.c_uint64)))
    return h, k


MASK64 = (1 << 64) - 1


def det_words_of(det: int) -> np.ndarray:
    """A determinant (Python int, up to 128 bits) as two 64-bit words, low first."""
    return np.array([int(det) & MASK64, int(det) >> 64], dtype=np.uint64)


def det_array(dets, w: int) -> np.ndarray:
    """Determinants as the ABI's array of w words each: shape (n,) for one word,
    (n, 2) for two (columns low, high); accepts ints or an array in either shape."""
    a = np.asarray(dets)
    if w == 1:
        return np.ascontiguousarray(a, dtype=np.uint64).reshape(-1)
    if a.ndim == 2:
        return np.ascontiguousarray(a, dtype=np.uint64)
    if a.dtype == np.uint64:     # one-word values: a zero high word
        return np.ascontiguousarray(np.stack([a.reshape(-1), np.zeros(a.size, np.uint64)], axis=1))
    return np.array([[int(d) & MASK64, int(d) >> 64] for d in a.reshape(-1)],
                    dtype=np.uint64).reshape(-1, 2)


def marshal_params(p):
    fo, fe = int(p.frozen_occupied), int(p.frozen_empty)
    return Params(p.tau, p.shift_damping, p.initial_shift, p.shift_update_every,
                  p.initiator_threshold, p.target_walkers, p.initial_walkers, p.det_capacity,
                  p.spawn_capacity, p.seed, p.avg_start, p.space, p.max_excitation,
                  p.max_seniority, fo & MASK64, fe & MASK64, p.hphf, 0, fo >> 64, fe >> 64,
                  getattr(p, "det_words", 0), 0)


def current_stream():
    """The current torch HIP stream handle (None when torch has no GPU)."""
    try:
        import torch
        if torch.cuda.is_available():
            return torch.cuda.current_stream().cuda_stream
    except Exception:
        pass
    return None


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _est_dict(e):
    return {f[0]: getattr(e, f[0]) for f in Estimates._fields_}


# ---- the C ABI, name for name ---------------------------------------------

def fciqmc_init(ham, params, stream=None):
    h, keep = marshal_hamiltonian(ham)
    p = marshal_params(params)
    out = C.c_void_p()
    _check(lib().fciqmc_init(C.byref(h), C.byref(p), stream, C.byref(out)))
    return out


def fciqmc_iterate(handle, n):
    _check(lib().fciqmc_iterate(handle, int(n)))


def fciqmc_estimators(handle):
    e = Estimates()
    _check(lib().fciqmc_estimators(handle, C.byref(e)))
    return _est_dict(e)


def fciqmc_free(handle):
    if handle:
        lib().fciqmc_free(handle)


def fciqmc_det_words(handle):
    return _check(lib().fciqmc_det_words(handle))


def _walkers(fn, w, *lead):
    n = _check(fn(*lead, None, None, None, 0))
    det = np.zeros(max(n, 1) * w, np.uint64)
    pop = np.zeros(max(n, 1), np.int32)
    flg = np.zeros(max(n, 1), np.uint32)
    m = _check(fn(*lead, _ptr(det), _ptr(pop), _ptr(flg), n))
    assert m == n
    det = det[:n * w]
    return (det if w == 1 else det.reshape(-1, 2)), pop[:n], flg[:n]


def fciqmc_walkers(handle):
    """(det, pop, flags): det of shape (n,) with one word per determinant, (n, 2)
    with two (low, high)."""
    return _walkers(lib().fciqmc_walkers, fciqmc_det_words(handle), handle)


def fciqmc_walkers_noalloc(handle, det, pop, flags):
    """Fill the caller's arrays (any may be None; the shortest non-None length is the
    capacity) through the library's fixed staging area; returns the determinant count."""
    arrs = [a for a in (det, pop, flags) if a is not None]
    cap = min(len(a) for a in arrs) if arrs else 0
    for a, dt in ((det, np.uint64), (pop, np.int32), (flags, np.uint32)):
        if a is not None:
            assert a.dtype == dt and a.flags.c_contiguous
    return _check(lib().fciqmc_walkers_noalloc(handle, _ptr(det), _ptr(pop), _ptr(flags), cap))


def fciqmc_load_walkers(handle, det, pop, iteration=0, shift=0.0, n_prev=0, varying=0, n_var=0):
    det = det_array(det, fciqmc_det_words(handle))
    pop = np.ascontiguousarray(pop, dtype=np.int32)
    _check(lib().fciqmc_load_walkers(handle, _ptr(det), _ptr(pop), len(pop), iteration, shift,
                                     n_prev, varying, n_var))


def fciqmc_set_shift(handle, shift, varying=1):
    _check(lib().fciqmc_set_shift(handle, shift, varying))


def fciqmc_reserve(handle, slots):
    _check(lib().fciqmc_reserve(handle, int(slots)))


def fciqmc_last_error():
    return lib().fciqmc_last_error().decode()


def fciqmc_batch_create(max_slots, hams, params, stream=None):
    n = len(hams)
    HA = (Hamiltonian * max(n, 1))()
    PA = (Params * max(n, 1))()
    keep = []
    for i, (hm, pr) in enumerate(zip(hams, params)):
        h, k = marshal_hamiltonian(hm)
        keep.append(k)
        HA[i] = h
        PA[i] = marshal_params(pr)
    out = C.c_void_p()
    _check(lib().fciqmc_batch_create(max_slots, n, HA, PA, stream, C.byref(out)))
    return out


def fciqmc_batch_iterate(handle, n):
    _check(lib().fciqmc_batch_iterate(handle, int(n)))


def fciqmc_batch_iterate_each(handle, n_iter):
    a = np.ascontiguousarray(n_iter, dtype=np.int32)
    _check(lib().fciqmc_batch_iterate_each(handle, _ptr(a)))


def fciqmc_batch_admit(handle, ham, params):
    h, keep = marshal_hamiltonian(ham)
    p = marshal_params(params)
    slot = C.c_int32()
    _check(lib().fciqmc_batch_admit(handle, C.byref(h), C.byref(p), C.byref(slot)))
    return slot.value


def fciqmc_batch_retire(handle, slot):
    _check(lib().fciqmc_batch_retire(handle, slot))


def fciqmc_batch_slot_estimators(handle, slot):
    e = Estimates()
    _check(lib().fciqmc_batch_slot_estimators(handle, slot, C.byref(e)))
    return _est_dict(e)


def fciqmc_batch_slot_walkers(handle, slot):
    return _walkers(lib().fciqmc_batch_slot_walkers, fciqmc_det_words(handle), handle,
                    C.c_int32(slot))


def fciqmc_footprint_bytes(ham, params):
    h, keep = marshal_hamiltonian(ham)
    p = marshal_params(params)
    return _check(lib().fciqmc_footprint_bytes(C.byref(h), C.byref(p)))


def fciqmc_batch_active(handle):
    return lib().fciqmc_batch_active(handle)


def fciqmc_set_profiling(handle, on):
    _check(lib().fciqmc_set_profiling(handle, int(on)))


def fciqmc_kernel_times(handle):
    ms = np.zeros(5)
    cnt = np.zeros(5, np.int64)
    _check(lib().fciqmc_kernel_times(handle, _ptr(ms), _ptr(cnt)))
    return ms, cnt


def fciqmc_set_launch(handle, spawn_grid, tile, post_grid):
    _check(lib().fciqmc_set_launch(handle, spawn_grid, tile, post_grid))


def fciqmc_get_launch(handle):
    a, b, c = C.c_int32(), C.c_int32(), C.c_int32()
    _check(lib().fciqmc_get_launch(handle, C.byref(a), C.byref(b), C.byref(c)))
    return a.value, b.value, c.value


def fciqmc_history(handle, slot, first, n):
    """Records of iterations first .. first + n - 1 of a slot, as a list of dicts."""
    out = (Iteration * max(n, 1))()
    _check(lib().fciqmc_history(handle, slot, first, n, out))
    return [{f[0]: getattr(out[i], f[0]) for f in Iteration._fields_} for i in range(n)]


def fciqmc_autotune(handle, iters_per_trial=2):
    _check(lib().fciqmc_autotune(handle, iters_per_trial))
    return fciqmc_get_launch(handle)


def fciqmc_blocking(num, den=None):
    """(mean, error) of <num>/<den> (or <num>) by the library's blocking analysis."""
    num = np.ascontiguousarray(num, dtype=np.float64)
    d = None if den is None else np.ascontiguousarray(den, dtype=np.float64)
    m, e = C.c_double(), C.c_double()
    _check(lib().fciqmc_blocking(_ptr(num), _ptr(d), len(num), C.byref(m), C.byref(e)))
    return m.value, e.value


def fciqmc_set_test_options(handle, planner=1, tile_map_limit=-1, record_capacity=0):
    _check(lib().fciqmc_set_test_options(handle, int(planner), int(tile_map_limit),
                                         int(record_capacity)))


class Solver:
    """Owning wrapper around one handle (single system)."""

    def __init__(self, ham, params, stream=None):
        self.h = fciqmc_init(ham, params, stream)

    def iterate(self, n=1):
        fciqmc_iterate(self.h, n)

    def estimates(self):
        return fciqmc_estimators(self.h)

    def walkers(self):
        return fciqmc_walkers(self.h)

    def load_walkers(self, *a, **k):
        fciqmc_load_walkers(self.h, *a, **k)

    def set_shift(self, shift, varying=1):
        fciqmc_set_shift(self.h, shift, varying)

    def reserve(self, slots):
        fciqmc_reserve(self.h, slots)

    def close(self):
        if self.h:
            fciqmc_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
