"""Benchmark of the IG hot path on one MI355X.

One step = ig_fit of the 15k workload (41 features, L = 464, K = 8; ~10.5k
training records) followed by ig_score of its ~4.5k held-out flows, with every
input already resident in HBM.  The reported throughput is subset tests per
second: the tests the method has to make in one step --

  coherence  sum over distinct candidates of t(b) (records of the other class
             examined up to and including the first that contains b)   Eq. 3
  support    |P^c| * n_c for both classes                              Eq. 2
  scoring    (|P^0| + |P^1|) * n_flows                                 Eq. 4

Also printed: the fit wall time at 15k and 148k, the roofline of the coherence
kernel (integer VALU bound) and the CPU oracle timed on a bounded sample.

    python bench.py [--gpus 1] [--steps 5] [--warmup 2] [--no-cpu] [--no-148k]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "subset tests/sec + IG fit wall-time at 15k/148k; served flows/sec with p99 latency"
# MI355X: 256 CUs x 64 lanes x 2.4 GHz, one 32-bit integer VALU op per lane per clock
VALU_INT32_PEAK_OPS = 256 * 64 * 2.4e9
# MI355X dense fp4 matrix-core peak (operations: 2 per multiply-add)
MFMA_FP4_PEAK_OPS = 10.1e15
HBM_PEAK_GBS = 8000.0


def counted_traffic(path, kernel):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter summary,
    or None when the summary is missing, covers another kernel, or the kernel
    source changed since the counters were taken."""
    import hashlib
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if ":" in line and not line.startswith(" "):
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    src = os.path.join(ROOT, "paper_2507_14222_amd", "csrc", "subset.hip")
    now = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
    if vals.get("kernel_source_sha256_16") != now or "bytes_per_launch" not in vals:
        return None
    if vals.get("kernel") != kernel:
        return None
    return int(vals["bytes_per_launch"])


def measure_batch():
    """64 problems (n 500..20,000, d 20..80, bins 4..32): ig_fit_batch against 64
    plain ig_fit calls.  The 64 models hold ~2.2e9 patterns, more than HBM, so both
    runs go through memory-sized slices of the problem list; each model is reduced
    to its device digest and freed."""
    import numpy as np
    import torch

    from paper_2507_14222_amd import ig, synth, tune

    probs = synth.make_batch()
    table = tune.load(os.path.join(ROOT, "paper_2507_14222_amd", "tuning_gfx950.json"))
    dev = [(torch.from_numpy(p.codes.view(np.int16)).cuda(), torch.from_numpy(p.labels).cuda(), p.nbins)
           for p in probs]

    class P:
        def __init__(self, c, l, nb):
            self.codes, self.labels, self.nbins = c, l, nb

    def est_bytes(p):
        n1 = int(p.labels.sum())
        n0 = p.n - n1
        K = tune.ig_storage_words((p.L + 63) // 64)
        return (n0 * (n0 + 1) // 2 + n1 * (n1 + 1) // 2) * (K * 8 + 12)

    slices, cur, acc = [], [], 0
    for i, p in enumerate(probs):
        b = est_bytes(p)
        if cur and acc + b > 90e9:
            slices.append(cur)
            cur, acc = [], 0
        cur.append(i)
        acc += b
    slices.append(cur)
    log("batch: %d problems in %d slices" % (len(probs), len(slices)))
    tests = 0
    dig_b, dig_s = {}, {}
    torch.cuda.synchronize()
    t_batch = 0.0
    for sl in slices:
        a = time.perf_counter()
        ms = ig.fit_batch([P(*dev[i]) for i in sl], tune=table)
        t_batch += time.perf_counter() - a
        for i, m in zip(sl, ms):
            st = m.stats()
            tests += sum(st.tests) + sum(st.support_tests)
            dig_b[i] = (m.digest(0), m.digest(1), tuple(st.coherent))
            m.free()
        log("batched slice of", len(sl), "done")
    t_seq = 0.0
    for i in range(len(probs)):
        a = time.perf_counter()
        m = ig.fit(*dev[i], tune=table)
        t_seq += time.perf_counter() - a
        st = m.stats()
        dig_s[i] = (m.digest(0), m.digest(1), tuple(st.coherent))
        m.free()
        if i % 8 == 7:
            log("sequential fits done:", i + 1)
    same = all(dig_b[i] == dig_s[i] for i in range(len(probs)))
    pats = sum(sum(dig_b[i][2]) for i in dig_b)
    return {"workload": "64 problems (seed 3)", "problems": len(probs), "slices": len(slices),
            "patterns": pats, "subset_tests": tests,
            "batched_s": t_batch, "sequential_s": t_seq,
            "batched_tests_per_s": tests / t_batch, "sequential_tests_per_s": tests / t_seq,
            "batched_problems_per_s": len(probs) / t_batch, "sequential_problems_per_s": len(probs) / t_seq,
            "identical": same, "tuning_rows": len(table or [])}


def measure_serving(seconds):
    """Served scoring: 10^6 patterns per class resident, Poisson arrivals of
    requests of 1..4096 flows; continuous batching vs one request at a time."""
    import numpy as np
    import torch

    from paper_2507_14222_amd import ig, synth
    from paper_2507_14222_amd.serve import Server, drive, serve_one_at_a_time

    log("serving: building 2 x 10^6 patterns")
    ps = synth.make_pattern_set()
    model = ig.import_patterns(ps.codes[0], ps.f[0], ps.codes[1], ps.f[1], ps.nbins)
    pool = synth.make_flows(n=200000)
    out = {"patterns": list(model.n_patterns()), "rates": []}

    def one_rate(rate, n_req, seed):
        reqs = synth.make_requests(seed, rate, n_req, pool.shape[0])
        codes = [pool[r.start:r.start + r.size] for r in reqs]
        arr = [r.arrival_s for r in reqs]
        return codes, arr

    # warm: code objects, pinned buffers
    codes, arr = one_rate(1e5, 20, 99)
    with Server(model, n_slots=4, max_batch_flows=16384) as srv:
        for f in [srv.submit(c) for c in codes]:
            f.result()
    for rate, seed in ((1e4, 11), (1e5, 12), (5e5, 13), (1e6, 14)):
        n_req = int(max(100, rate * seconds / 492))
        codes, arr = one_rate(rate, n_req, seed)
        with Server(model, n_slots=4, max_batch_flows=16384) as srv:
            futs, t0 = drive(srv, codes, arr)
            for f in futs:
                f.result()
            done = srv.completed
            batches = srv.batches
        lat = np.array([r.t_done - r.t_arrival for r in done])
        flows = sum(c.shape[0] for c in codes)
        span = max(r.t_done for r in done) - t0
        out["rates"].append({"offered_flows_per_s": rate, "requests": n_req, "flows": flows,
                             "served_flows_per_s": flows / span, "batches": batches,
                             "p50_ms": float(np.percentile(lat, 50) * 1e3),
                             "p99_ms": float(np.percentile(lat, 99) * 1e3)})
        log("serving", out["rates"][-1])
    # one request at a time at the middle rate
    codes, arr = one_rate(1e5, int(max(100, 1e5 * seconds / 492)), 12)
    _, lat1 = serve_one_at_a_time(model, codes, arr)
    flows = sum(c.shape[0] for c in codes)
    span = arr[-1] + lat1[-1]
    lat1 = np.array(lat1)
    out["one_at_a_time"] = {"offered_flows_per_s": 1e5, "requests": len(codes), "flows": flows,
                            "served_flows_per_s": flows / span,
                            "p50_ms": float(np.percentile(lat1, 50) * 1e3),
                            "p99_ms": float(np.percentile(lat1, 99) * 1e3)}
    # saturated throughput: every request queued at once
    codes, arr = one_rate(1e6, 2000, 15)
    with Server(model, n_slots=4, max_batch_flows=16384) as srv:
        t0 = time.perf_counter()
        for f in [srv.submit(c) for c in codes]:
            f.result()
        dt = time.perf_counter() - t0
    out["saturated_flows_per_s"] = sum(c.shape[0] for c in codes) / dt
    log("serving saturated", out["saturated_flows_per_s"])
    del model
    torch.cuda.synchronize()
    return out


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-148k", action="store_true", help="skip the 148k fit wall time")
    ap.add_argument("--no-serve", action="store_true", help="skip the served-scoring measurement")
    ap.add_argument("--serve-seconds", type=float, default=2.0, help="offered load duration per rate")
    ap.add_argument("--cpu-records", type=int, default=7000, help="training records in the oracle sample")
    ap.add_argument("--batch", action="store_true",
                    help="only run the 64-problem workload: batched fit vs 64 plain fits")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a plain device copy of 1 GiB, 4 times (calibrates HBM byte counters)")
    ap.add_argument("--traffic", type=str, default=os.path.join(ROOT, "profiles", "dominant_kernel_15k_traffic.txt"))
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the multi-GPU design is "
              "described, not built", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2507_14222_amd import ig, synth

    torch.cuda.set_device(0)
    if args.copy_probe:
        src = torch.empty(1 << 30, dtype=torch.uint8, device="cuda").fill_(1)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        for _ in range(4):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": 1 << 30, "copies": 4}))
        return
    if args.batch:
        print(json.dumps(measure_batch()), flush=True)
        return
    w = synth.make_15k()
    log("15k workload", w.codes.shape, "test", w.test_codes.shape)
    d_codes = torch.from_numpy(w.codes.view(np.int16)).cuda()
    d_labels = torch.from_numpy(w.labels).cuda()
    d_flows = torch.from_numpy(w.test_codes.view(np.int16)).cuda()
    out = torch.empty((w.test_codes.shape[0], 2), dtype=torch.int64, device="cuda")
    stream = torch.cuda.current_stream()

    score_ev = []

    def step():
        m = ig.fit(d_codes, d_labels, w.nbins, stream=stream)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        ig.score(m, d_flows, out=out, stream=stream)
        e1.record(stream)
        score_ev.append((e0, e1))
        return m

    for i in range(args.warmup):
        m = step()
        torch.cuda.synchronize()
        log("warmup", i, "done")
    torch.cuda.synchronize()
    fit_s, models = [], []
    t0 = time.perf_counter()
    for i in range(args.steps):
        a = time.perf_counter()
        m = step()
        fit_s.append(time.perf_counter() - a)   # ig_fit returns once the model is complete
        models.append(m)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    log("timed steps done: %.2f ms/step" % ms_per_step)

    st = models[-1].stats()
    npat = models[-1].n_patterns()
    K = models[-1].K
    L = int(w.L)
    n_flows = w.test_codes.shape[0]
    # the method's subset tests: sum of t(b) in input order (from one untimed fit on the
    # early-exit path), |P^c| * n_c support tests and |P| * n_flows scoring tests
    ref = ig.fit(d_codes, d_labels, w.nbins, kernels="valu", stream=stream)
    coh_tests = sum(ref.stats().tests)
    del ref
    sup_tests = sum(st.support_tests)
    score_tests = (npat[0] + npat[1]) * n_flows
    tests_per_step = coh_tests + sup_tests + score_tests
    value = tests_per_step / (ms_per_step / 1e3)
    on_mfma = sum(st.tests) != coh_tests            # dense count: the matrix-core kernels ran
    coh_ms = sum(mm.stats().ms[4] for mm in models) / len(models)
    sup_ms = sum(mm.stats().ms[6] for mm in models) / len(models)
    # the subset-test kernels alone (event pairs around their launches), where timed
    kcoh_ms = sum(mm.stats().kernel_ms[0] for mm in models) / len(models)
    ksup_ms = sum(mm.stats().kernel_ms[1] for mm in models) / len(models)
    score_ms = sum(a.elapsed_time(b) for a, b in score_ev[-len(models):]) / len(models)
    n_cls = list(st.n_class)
    kernels = {}
    info = models[-1].info()
    L_mfma = int(info.mfma_tokens)                      # tokens per row of the matrix-core operands
    if on_mfma:
        dense = sum(st.tests)                           # every (candidate, other-class record) pair
        kernels["k_contain_mfma[coherence]"] = {"bound": "mfma", "ms": kcoh_ms or coh_ms,
                                                "ops": 2.0 * L_mfma * dense,
                                                "peak": MFMA_FP4_PEAK_OPS, "unit": "TFLOP/s (fp4 dense)"}
        kernels["k_contain_mfma[support]"] = {"bound": "mfma", "ms": ksup_ms or sup_ms,
                                              "ops": 2.0 * L_mfma * sup_tests,
                                              "peak": MFMA_FP4_PEAK_OPS, "unit": "TFLOP/s (fp4 dense)"}
    else:
        kernels["k_coherence"] = {"bound": "alu", "ms": coh_ms, "ops": 2.0 * K * coh_tests,
                                  "peak": VALU_INT32_PEAK_OPS, "unit": "TOP/s (int32 VALU)"}
        kernels["k_support"] = {"bound": "alu", "ms": sup_ms, "ops": 2.0 * K * sup_tests,
                                "peak": VALU_INT32_PEAK_OPS, "unit": "TOP/s (int32 VALU)"}
    if models[-1].score_on_matrix_cores:
        kernels["k_score_mfma"] = {"bound": "mfma", "ms": score_ms, "ops": 2.0 * L_mfma * score_tests,
                                   "peak": MFMA_FP4_PEAK_OPS, "unit": "TFLOP/s (fp4 dense)"}
    else:
        kernels["k_score"] = {"bound": "alu", "ms": score_ms, "ops": 2.0 * K * score_tests,
                              "peak": VALU_INT32_PEAK_OPS, "unit": "TOP/s (int32 VALU)"}
    for k, v in kernels.items():
        v["achieved"] = v["ops"] / (v["ms"] / 1e3) / 1e12
        v["frac"] = v["ops"] / (v["ms"] / 1e3) / v["peak"]
    dom = max(kernels, key=lambda k: kernels[k]["ms"])
    d = kernels[dom]
    roofline = {"bound": d["bound"], "kernel": dom, "achieved": d["achieved"], "peak": d["peak"] / 1e12,
                "unit": d["unit"], "frac": d["frac"], "traffic": counted_traffic(args.traffic, dom),
                "avg_ms": d["ms"]}
    res = {
        "metric": METRIC, "value": value, "unit": "subset tests/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": w.name, "n_train": int(w.n), "n_flows": int(n_flows), "d": int(w.d),
                   "L": int(w.L), "K": int(K), "mfma_tokens": L_mfma, "mfma_words": int(info.mfma_words)},
        "fit_wall_s_15k": float(np.median(fit_s)),
        "tests_per_step": {"coherence": coh_tests, "support": sup_tests, "scoring": score_tests},
        "patterns": list(npat), "distinct": list(st.distinct),
        "stage_ms": {k: round(v, 3) for k, v in zip(
            ["pack", "pairs", "sort", "dedup", "coherence", "order", "support", "fit_total"], st.ms)},
        "roofline": roofline,
        "kernels": {k: {"ms": round(v["ms"], 3), "achieved": round(v["achieved"], 2), "frac": round(v["frac"], 4),
                        "bound": v["bound"]} for k, v in kernels.items()},
    }
    del models
    if not args.no_148k:
        w2 = synth.make_148k()
        log("148k workload", w2.codes.shape)
        dc2 = torch.from_numpy(w2.codes.view(np.int16)).cuda()
        dl2 = torch.from_numpy(w2.labels).cuda()
        m2 = ig.fit(dc2, dl2, w2.nbins)   # warm (allocations, code load)
        del m2
        torch.cuda.synchronize()
        a = time.perf_counter()
        m2 = ig.fit(dc2, dl2, w2.nbins)
        res["fit_wall_s_148k"] = time.perf_counter() - a
        st2 = m2.stats()
        res["fit_148k"] = {"n_train": int(w2.n), "patterns": list(m2.n_patterns()), "tests": list(st2.tests),
                           "coherence_ms": st2.ms[4]}
        del m2
    if not args.no_serve:
        res["serve"] = measure_serving(args.serve_seconds)
    if not args.no_cpu:
        import oracle
        ns = min(args.cpu_records, w.n)
        nf = 300
        log("cpu oracle on", ns, "records,", nf, "flows")
        a = time.perf_counter()
        om = oracle.fit(w.codes[:ns], w.labels[:ns], w.nbins)
        oracle.score(om, w.test_codes[:nf], w.nbins)
        dt = time.perf_counter() - a
        t_or = sum(om.stats["tests"]) + sum(p.shape[0] * n for p, n in zip(om.patterns, om.stats["n_class"])) \
            + sum(p.shape[0] for p in om.patterns) * nf
        res["cpu_baseline"] = {"value": t_or / dt, "unit": "subset tests/s", "cores": oracle.max_threads(),
                               "kind": "oracle", "seconds": dt,
                               "sample": f"oracle fit of the first {ns} training records of the 15k workload "
                                         f"+ scoring {nf} held-out flows"}
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
