"""Serving: requests admitted while others run (continuous batching) give
exactly the walker lists of their solo runs (and of the oracle)."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1305_6981_amd import serve
from paper_1305_6981_amd import systems as S

pytestmark = pytest.mark.gpu


def _requests():
    reqs = []
    h, p, _ = S.workload("hubbard8", scale=0.1)
    reqs.append(serve.Request(h, p, arrival=0.0, max_iters=70, tag="hub8"))
    h2 = S.hubbard_ring(10, 5.0)
    p2 = S.Params(tau=0.01, shift_update_every=1, target_walkers=2000, seed=301)
    reqs.append(serve.Request(h2, p2, arrival=0.0, max_iters=45, tag="hub10"))
    h3, p3, _ = S.workload("synth10e20o", scale=1e-4)
    p3.initial_walkers, p3.initial_shift = 200, 0.5
    reqs.append(serve.Request(h3, p3, arrival=0.0, max_iters=90, tag="syn20"))
    h4 = S.synthetic_molecule(16, 5, 5, 404)
    p4 = S.Params(tau=2e-3, initiator_threshold=3, target_walkers=3000, initial_walkers=150,
                  initial_shift=0.4, seed=305)
    reqs.append(serve.Request(h4, p4, arrival=0.02, max_iters=64, tag="syn16"))
    h5 = S.hubbard_ring(12, 2.5)
    p5 = S.Params(tau=0.01, shift_update_every=1, target_walkers=1500, seed=306)
    reqs.append(serve.Request(h5, p5, arrival=0.03, max_iters=33, tag="hub12"))
    return reqs


def test_served_results_equal_solo_runs():
    reqs = _requests()
    print(f"[gpu] serving {len(reqs)} requests on 3 slots", flush=True)
    srv = serve.SolveServer(max_slots=3, chunk_iters=16, tol=0.0, keep_walkers=True)
    stats = srv.run(reqs)
    assert len(stats.results) == len(reqs)
    assert stats.peak_active == 3
    by_tag = {r.tag: r for r in stats.results}
    for req in reqs:
        res = by_tag[req.tag]
        assert res.iterations == req.max_iters
        o = O.Oracle(req.ham, req.params)
        o.iterate(res.iterations)
        d, p, _ = o.walkers()
        gd, gp, _ = res.walkers
        assert np.array_equal(gd, d) and np.array_equal(gp, p), req.tag
        o.close()
    # at least one request was admitted while others were already running
    late = [r for r in stats.results if r.admitted > 0.0]
    assert late
    summ = stats.summary()
    assert summ["p99_latency_s"] >= summ["p50_latency_s"] > 0


def test_request_the_batch_cannot_hold_fails_alone():
    """A request of another determinant width (72 spin orbitals: two words) than the
    server's one-word batch is recorded as failed; the others are served."""
    reqs = _requests()[:2]
    big = S.synthetic_molecule(36, 2, 2, 7, orb_energy=np.linspace(-4.0, 4.0, 36))
    reqs.insert(1, serve.Request(big, S.Params(tau=0.01, seed=9), arrival=0.0, max_iters=20,
                                 tag="two-word"))
    print(f"[gpu] serving {len(reqs)} requests, one of two-word determinants", flush=True)
    stats = serve.SolveServer(max_slots=3, chunk_iters=16, tol=0.0).run(reqs)
    by_tag = {r.tag: r for r in stats.results}
    assert len(by_tag) == 3
    assert by_tag["two-word"].failed and by_tag["two-word"].iterations == 0
    for req in reqs:
        if req.tag != "two-word":
            assert not by_tag[req.tag].failed and by_tag[req.tag].iterations == req.max_iters
