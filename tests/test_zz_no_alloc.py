"""The export that allocates nothing (fciqmc_walkers_noalloc), through the C ABI,
against fciqmc_walkers on the same handle: two calls in a row, the second on a
smaller list (the fixed staging area keeps the first call's contents), a capacity
smaller than the list, and a list beyond the staging limit."""
import numpy as np
import pytest

from paper_1305_6981_amd import fciqmc as F
from paper_1305_6981_amd import systems as S

pytestmark = pytest.mark.gpu

LIMIT = 1 << 21


def _stream():
    import torch
    assert torch.cuda.is_available()
    return F.current_stream()


def _noalloc(h, n):
    det = np.zeros(n, np.uint64)
    pop = np.zeros(n, np.int32)
    flg = np.zeros(n, np.uint32)
    m = F.fciqmc_walkers_noalloc(h, det, pop, flg)
    return m, det, pop, flg


def test_noalloc_export_matches_walkers():
    ham, prm, _ = S.workload("synth10e20o", scale=2e-3)
    prm.initial_walkers, prm.initial_shift, prm.tau = 3000, 5.0, 3e-3
    print("[gpu] noalloc: first list", flush=True)
    sv = F.Solver(ham, prm, _stream())
    sv.iterate(80)
    d1, p1, f1 = sv.walkers()
    assert len(d1) > 3000
    m, d, p, f = _noalloc(sv.h, len(d1) + 7)
    assert m == len(d1)
    assert np.array_equal(d[:m], d1) and np.array_equal(p[:m], p1) and np.array_equal(f[:m], f1)
    # second call, smaller list: load a quarter of it back, export again
    print("[gpu] noalloc: second, smaller list", flush=True)
    keep = np.arange(0, len(d1), 4)
    sv.load_walkers(d1[keep], p1[keep], iteration=80)
    d2, p2, f2 = sv.walkers()
    assert len(d2) < len(d1)
    m2, d, p, f = _noalloc(sv.h, len(d2))
    assert m2 == len(d2)
    assert np.array_equal(d, d2) and np.array_equal(p, p2) and np.array_equal(f, f2)
    # capacity below the count: the first cap entries of the sorted list
    m3, d, p, f = _noalloc(sv.h, 100)
    assert m3 == len(d2)
    assert np.array_equal(d, d2[:100]) and np.array_equal(p, p2[:100])
    # one array only
    det_only = np.zeros(len(d2), np.uint64)
    assert F.fciqmc_walkers_noalloc(sv.h, det_only, None, None) == len(d2)
    assert np.array_equal(det_only, d2)
    sv.close()


def test_noalloc_export_rejects_lists_beyond_the_limit():
    ham, prm, _ = S.workload("synth10e20o", scale=1e-4)
    rng = np.random.default_rng(3)
    n = LIMIT + 5000
    dets = set()
    while len(dets) < n:
        a = np.argsort(rng.random((n, 20)), axis=1)[:, :5]
        b = np.argsort(rng.random((n, 20)), axis=1)[:, :5]
        w = (np.left_shift(np.uint64(1), (2 * a).astype(np.uint64)).sum(axis=1) +
             np.left_shift(np.uint64(1), (2 * b + 1).astype(np.uint64)).sum(axis=1))
        dets.update(int(x) for x in w)
    det = np.array(sorted(dets)[:n], np.uint64)
    pop = np.ones(n, np.int32)
    print(f"[gpu] noalloc: {n} dets (limit {LIMIT})", flush=True)
    sv = F.Solver(ham, prm, _stream())
    sv.load_walkers(det, pop)
    assert len(sv.walkers()[0]) >= n
    with pytest.raises(F.FciqmcError) as ei:
        _noalloc(sv.h, 16)
    assert ei.value.code == -4
    # the handle still works afterwards, also for the staging path
    sv.load_walkers(det[:1000], pop[:1000])
    m, d, p, f = _noalloc(sv.h, 2000)
    dw, pw, fw = sv.walkers()
    assert m == len(dw) and np.array_equal(d[:m], dw)
    sv.close()
