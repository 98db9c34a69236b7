"""ig_score_noalloc, the scoring entry point that allocates nothing (its pruned
scoring's work goes to a fixed device array of the library): through the C ABI,
its output equals ig_score's bit for bit on two calls in a row, the second with
a smaller input (the array keeps the first call's contents), and sizes beyond the
array are rejected before any device work."""
import sys

import numpy as np
import pytest

from paper_2507_14222_amd import ig, synth

pytestmark = pytest.mark.gpu


def say(*a):
    print("[no-alloc]", *a, flush=True)
    sys.stdout.flush()


def _dev_flows(codes):
    import torch
    return torch.from_numpy(np.ascontiguousarray(codes, np.uint16).view(np.int16)).cuda()


def _both(m, flows):
    import torch
    dc = _dev_flows(flows)
    ref = ig.score(m, dc)
    out = torch.full((dc.shape[0], 2), 0x5A5A5A5A, dtype=torch.int64, device="cuda")   # unwritten rows show
    ig.score_noalloc(m, dc, out)
    torch.cuda.synchronize()
    return ref.cpu().numpy(), out.cpu().numpy()


def test_noalloc_equals_ig_score_twice_second_smaller():
    w = synth.make_15k()
    m = ig.fit(w.codes, w.labels, w.nbins)
    assert m.bucketed
    flows = w.test_codes.copy()
    flows[10, 3] = w.nbins[3]   # a flow with a code out of range: (-1, -1) from both
    for n in (flows.shape[0], 1234):
        say("15k model,", n, "flows")
        ref, got = _both(m, flows[:n])
        assert np.array_equal(ref, got)
        assert got[10, 0] == -1 and got[10, 1] == -1


def test_noalloc_on_models_without_buckets_and_empty_input():
    p = synth.make_random_problem(12, 140, 50, bins_lo=10, bins_hi=14)
    m = ig.fit(p.codes, p.labels, p.nbins, kernels="valu")
    say("model without buckets:", m.bucketed)
    for n in (140, 33):
        ref, got = _both(m, p.codes[:n])
        assert np.array_equal(ref, got)
    import torch
    out = torch.zeros((0, 2), dtype=torch.int64, device="cuda")
    ig.score_noalloc(m, _dev_flows(p.codes[:0]), out)


def test_noalloc_rejects_sizes_beyond_the_array():
    import torch
    w = synth.make_tiny(0)
    m = ig.fit(w.codes, w.labels, w.nbins)
    assert m.bucketed
    words = (8 << 20) // 4
    W = int(m.info().mfma_words)

    def need(n):   # the call's scratch words: lists and units, then 2 W uint4 per flow
        return (n * int(w.d) + 5 * int(w.L) + 3 + 3) // 4 * 4 + 8 * W * n

    n = words // (int(w.d) + 8 * W)
    while need(n) > words:
        n -= 1
    n += 1                                              # one flow too many
    say("oversize", n, "flows of", w.d)
    dc = torch.zeros((n, int(w.d)), dtype=torch.int16, device="cuda")
    out = torch.zeros((n, 2), dtype=torch.int64, device="cuda")
    with pytest.raises(ig.IGError) as e:
        ig.score_noalloc(m, dc, out)
    assert e.value.status == ig.IG_E_UNSUPPORTED
    ig.score_noalloc(m, dc[: n - 1], out[: n - 1])     # the largest size that fits
    ref = ig.score(m, dc[: n - 1])
    torch.cuda.synchronize()
    assert torch.equal(ref, out[: n - 1])
