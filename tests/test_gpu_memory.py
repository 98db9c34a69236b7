"""Device memory of the library: the caller-allocator boundary (ig_fit_opts.alloc)
and the library's own arena.  A fit through torch's caching allocator gives the
same model as through the arena; an allocator that fails part-way leaves no model,
no error but IG_E_NOMEM and no block behind; repeated fits reuse the arena without
growing it; ig_release_memory gives free chunks back."""
import gc
import sys

import numpy as np
import pytest

import oracle
from paper_2507_14222_amd import ig, synth

pytestmark = pytest.mark.gpu


def say(*a):
    print("[memory]", *a, flush=True)
    sys.stdout.flush()


def _same(a, b):
    for c in (0, 1):
        for x, y in zip(a.export(c), b.export(c)):
            assert np.array_equal(x, y)


def test_fit_through_torch_allocator():
    import torch
    p = synth.make_random_problem(11, 170, 41, bins_lo=10, bins_hi=14, attack_frac=0.55)
    alloc = ig.torch_allocator()
    m = ig.fit(p.codes, p.labels, p.nbins, allocator=alloc)
    say("torch allocator: calls", alloc._state["n"], "held", len(alloc._state["live"]))
    assert alloc._state["n"] > 0 and len(alloc._state["live"]) > 0   # the model's buffers
    _same(m, ig.fit(p.codes, p.labels, p.nbins))
    om = oracle.fit(p.codes, p.labels, p.nbins)
    for c in (0, 1):
        assert np.array_equal(m.export(c)[0], om.patterns[c])
    out = ig.score(m, p.codes)
    torch.cuda.synchronize()
    A, N = oracle.score(om, p.codes, p.nbins)
    assert np.array_equal(out[:, 0].cpu().numpy(), A) and np.array_equal(out[:, 1].cpu().numpy(), N)
    m.free()
    assert len(alloc._state["live"]) == 0   # every block went back
    B = ig.fit_batch([p, synth.make_random_problem(12, 90, 20, bins_lo=3, bins_hi=6)], allocator=alloc)
    _same(B[0], ig.fit(p.codes, p.labels, p.nbins))
    del B
    gc.collect()
    assert len(alloc._state["live"]) == 0


@pytest.mark.parametrize("fail_after", [0, 1, 3, 8, 20, 40])
def test_failing_allocator_leaves_nothing(fail_after):
    p = synth.make_random_problem(8, 200, 30, bins_lo=4, bins_hi=8)
    alloc = ig.torch_allocator(fail_after=fail_after)
    full = ig.torch_allocator()
    ig.fit(p.codes, p.labels, p.nbins, allocator=full).free()
    say("allocations of a whole fit:", full._state["n"], "fail after", fail_after)
    if fail_after >= full._state["n"]:
        pytest.skip("the fit needs fewer allocations")
    with pytest.raises(ig.IGError) as e:
        ig.fit(p.codes, p.labels, p.nbins, allocator=alloc)
    assert e.value.status == ig.IG_E_NOMEM
    assert len(alloc._state["live"]) == 0, "blocks left behind by a failed fit"
    ok = ig.fit(p.codes, p.labels, p.nbins)        # the library still works afterwards
    assert sum(ok.n_patterns()) > 0
    ok.free()   # (the raised error's traceback keeps this frame alive until a collection)


def test_arena_is_reused_and_released():
    gc.collect()   # models of earlier tests held only by reference cycles
    ig.release_memory()
    base = ig.memory_stats()   # what other live models of the process hold
    w = synth.make_tiny(0)
    ms = [ig.fit(w.codes, w.labels, w.nbins) for _ in range(2)]
    first = ig.memory_stats()
    for _ in range(6):
        ms.append(ig.fit(w.codes, w.labels, w.nbins))
        ms.pop(0).free()
    again = ig.memory_stats()
    say("arena", first, again)
    assert again["reserved"] == first["reserved"], "repeated fits grew the arena"
    for m in ms:
        m.free()
    ig.release_memory()
    after = ig.memory_stats()
    say("released", after)
    assert after["in_use"] == base["in_use"] and after["cached"] == 0
    assert after["reserved"] <= first["reserved"]
