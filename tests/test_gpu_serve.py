"""Continuous batching on the GPU: every request's (A, N) is identical when it
is served in the mix and when it is scored alone (integers: tolerance 0), and
matches the oracle on sampled requests."""
import sys

import numpy as np
import pytest

import oracle
from paper_2507_14222_amd import ig, synth
from paper_2507_14222_amd.serve import Server, drive, serve_one_at_a_time

pytestmark = pytest.mark.gpu


def say(*a):
    print("[serve]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def setup():
    nb = synth.mixture41_nbins()
    ps = synth.make_pattern_set(seed=43, per_class=20000)
    model = ig.import_patterns(ps.codes[0], ps.f[0], ps.codes[1], ps.f[1], nb)
    pool = synth.make_flows(seed=44, n=30000)
    reqs = synth.make_requests(45, 2e5, 80, pool.shape[0])
    codes = [pool[r.start:r.start + r.size] for r in reqs]
    return ps, nb, model, codes, [r.arrival_s for r in reqs]


def test_mix_equals_alone(setup):
    import torch
    ps, nb, model, codes, arrivals = setup
    say("mix of", len(codes), "requests,", sum(c.shape[0] for c in codes), "flows")
    with Server(model, n_slots=4, max_batch_flows=8192) as srv:
        futs = [srv.submit(c) for c in codes]        # all at once: they share micro-batches
        mixed = [f.result(timeout=120) for f in futs]
        batches = srv.batches
    assert batches < len(codes)
    for c, got in zip(codes, mixed):
        alone = ig.score(model, c)
        torch.cuda.synchronize()
        assert np.array_equal(got, alone.cpu().numpy())
    om = oracle.model_from_patterns(ps.codes[0], ps.f[0], ps.codes[1], ps.f[1], nb)
    for k in (0, len(codes) // 2, len(codes) - 1):
        A, N = oracle.score(om, codes[k], nb)
        assert np.array_equal(mixed[k][:, 0], A) and np.array_equal(mixed[k][:, 1], N)


def test_open_loop_and_baseline_agree(setup):
    ps, nb, model, codes, arrivals = setup
    say("open loop")
    with Server(model, n_slots=3, max_batch_flows=4096) as srv:
        futs, _ = drive(srv, codes[:40], arrivals[:40])
        got = [f.result(timeout=120) for f in futs]
    base, lat = serve_one_at_a_time(model, codes[:40], arrivals[:40])
    for a, b in zip(got, base):
        assert np.array_equal(a, b)
    assert all(x >= 0 for x in lat)


def test_memory_budget_and_cancel(setup):
    ps, nb, model, codes, arrivals = setup
    say("budget")
    budget = 6000 * (2 * 41 + 16)
    with Server(model, n_slots=4, max_batch_flows=4096, mem_budget_bytes=budget) as srv:
        futs = [srv.submit(c) for c in codes[:30]]
        futs[-1].cancel()
        for f, c in zip(futs[:-1], codes[:29]):
            assert f.result(timeout=120).shape == (c.shape[0], 2)
        assert srv.max_in_flight_bytes <= budget
