"""Benchmark of the IG hot path on one MI355X.

One step = ig_fit of the 15k workload (41 features, L = 464, K = 8; 10,500
training records) followed by ig_score of its 4,500 held-out flows, with every
input already resident in HBM.  The reported throughput is subset tests per
second: the tests the method has to make in one step --

  coherence  sum over distinct candidates of t(b) (records of the other class
             examined in input order up to and including the first that
             contains b)                                               Eq. 3
  support    |P^c| * n_c for both classes                              Eq. 2
  scoring    (|P^0| + |P^1|) * n_flows                                 Eq. 4

The subset tests run as dense fp4 contractions on the matrix cores (exact:
small integers accumulated in fp32; scoring also weights in int8 -> int32).
Each contraction kernel's roofline is reported per launch: achieved = the
method's operations of the launch (2 * tokens per test, tests counted as above)
/ the launch's duration from HIP events on its stream, against the vendor's
dense fp4 peak and the peak measured in the same run (ig_probe_mfma_fp4); the
fraction of executed matrix-core operations (every (row, column) pair of the
padded tiles) is given beside it.

Also printed: the fit wall time at 15k and 148k (from device inputs, and from
host arrays including the export of both sorted pattern sets), scoring wall
time, served scoring, the 64-problem batched fit against 64 plain fits, and the
CPU oracle built for this host and timed on a bounded sample.

    python bench.py [--gpus 1] [--steps 5] [--warmup 2] [--no-cpu] [--no-148k] [--no-serve] [--no-batch]
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
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter summary
    (a line "bytes_per_launch[<kernel>]: N" per kernel), or None when the summary is
    missing, does not cover the kernel, or the kernel source changed since the
    counters were taken."""
    import hashlib
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if ":" in line and not line.startswith(" ") and not line.startswith("|"):
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    src = os.path.join(ROOT, "paper_2507_14222_amd", "csrc", "subset.hip")
    now = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
    if vals.get("kernel_source_sha256_16") != now:
        return None
    v = vals.get("bytes_per_launch[%s]" % kernel)
    return int(v) if v else None


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

    slices = tune.slices_by_memory(probs)
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


def pruned_work(model, flows, nbins):
    """Pattern-flow tests of pruned scoring, from the model's bucket sizes and the
    flows' tokens: the tests it makes and those its padded tiles execute."""
    import numpy as np
    off = np.concatenate([[0], np.cumsum(nbins.astype(np.int64))])
    F = np.zeros(int(off[-1]), np.int64)
    for f in range(flows.shape[1]):
        np.add.at(F, off[f] + flows[:, f].astype(np.int64), 1)
    tests = ex = 0
    for c in (0, 1):
        P = model.bucket_sizes(c).astype(np.int64)
        tests += int((P * F).sum())
        ex += int((((P + 31) // 32) * 32 * ((F + 255) // 256) * 256).sum())
    return {"tests": tests, "exec_tests": ex}


def scoring_modes(model, d_flows, out, reps=5):
    """Device time of one scoring launch, pruned and dense (HIP events on the stream)."""
    import numpy as np
    import torch

    from paper_2507_14222_amd import ig
    res = {}
    for mode in ("pruned", "dense"):
        ts = []
        for _ in range(reps + 1):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            ig.score(model, d_flows, out=out, mode=mode)
            e1.record()
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1))
        res[mode + "_ms"] = float(np.median(ts[1:]))
    res["speedup"] = res["dense_ms"] / res["pruned_ms"]
    return res


def detection(model, d_train, d_train_labels, d_flows, truth, r=0.568):
    """Regulations 1-3 (Regulation 3 with mu_N, sigma_N of the normal training
    records and r = 0.568) on the held-out flows, and the metrics of Table 2."""
    import time as _t

    import torch

    from paper_2507_14222_amd import ig
    torch.cuda.synchronize()
    a = _t.perf_counter()
    tr = ig.score(model, d_train)
    mo = ig.normal_moments(tr, d_train_labels)
    T = ig.r3_threshold(mo, r)
    te = ig.score(model, d_flows)
    lab, _ = ig.classify(te, T)
    mt = ig.detection_metrics(te, lab, truth)
    torch.cuda.synchronize()
    out = mt.as_dict()
    out.update({"r": r, "r3_threshold": T, "wall_s": _t.perf_counter() - a})
    return out


def evidence_time(model, d_flows, k):
    import torch

    from paper_2507_14222_amd import ig
    ig.evidence(model, d_flows[:8], k)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    ig.evidence(model, d_flows, k)
    e1.record()
    torch.cuda.synchronize()
    return {"flows": int(d_flows.shape[0]), "k": k, "ms": e0.elapsed_time(e1)}


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def measured_peaks():
    """fp4 matrix-core and HBM copy rates measured on this device (best of 3)."""
    import torch

    from paper_2507_14222_amd import ig

    mf = max(ig.probe_mfma_fp4(20000)[0] for _ in range(3))
    src = torch.empty(1 << 32, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    src.fill_(1)
    hbm = max(ig.probe_hbm_copy(src, dst)[0] for _ in range(3))
    del src, dst
    torch.cuda.synchronize()
    return {"fp4_mfma_ops_per_s": mf, "hbm_copy_bytes_per_s": hbm,
            "fp4_mfma_frac_of_vendor": mf / MFMA_FP4_PEAK_OPS, "hbm_frac_of_vendor": hbm / (HBM_PEAK_GBS * 1e9)}


def fit_wall(codes, labels, nbins, d_codes, d_labels, reps=3):
    """Median wall time of ig_fit alone (device inputs, returns with the model
    complete) and of the whole fit from host arrays plus the export of both
    sorted pattern sets to the host."""
    import numpy as np
    import torch

    from paper_2507_14222_amd import ig

    dev, host = [], []
    for _ in range(reps):
        torch.cuda.synchronize()
        a = time.perf_counter()
        m = ig.fit(d_codes, d_labels, nbins)
        dev.append(time.perf_counter() - a)
        del m
        torch.cuda.synchronize()
        a = time.perf_counter()
        m = ig.fit(codes, labels, nbins)
        m.export(0)
        m.export(1)
        host.append(time.perf_counter() - a)
        del m
    return float(np.median(dev)), float(np.median(host))


def cpu_baseline(w, n_records, n_flows, n_records_1t):
    """The oracle as it stands, compiled for this host (-O3 -march=native), timed
    on a bounded sample of the 15k workload with all host threads, and on a
    smaller sample with one thread; value in subset tests/s."""
    import tempfile

    import oracle
    from oracle import build_oracle

    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    tmp = tempfile.mkdtemp(prefix="igoracle")
    oracle.use_library(build_oracle.build_native(tmp))

    def run(ns, nf):
        a = time.perf_counter()
        om = oracle.fit(w.codes[:ns], w.labels[:ns], w.nbins)
        oracle.score(om, w.test_codes[:nf], w.nbins)
        dt = time.perf_counter() - a
        tests = sum(om.stats["tests"]) + sum(p.shape[0] * n for p, n in zip(om.patterns, om.stats["n_class"])) \
            + sum(p.shape[0] for p in om.patterns) * nf
        return tests / dt, dt

    threads = oracle.max_threads()
    log("cpu oracle on", n_records, "records,", n_flows, "flows,", threads, "threads")
    v, dt = run(n_records, n_flows)
    oracle.set_threads(1)
    log("cpu oracle on", n_records_1t, "records, 1 thread")
    v1, dt1 = run(n_records_1t, n_flows // 3)
    oracle.set_threads(threads)
    oracle.use_library(None)
    return {"value": v, "unit": "subset tests/s", "cores": threads, "kind": "oracle", "seconds": dt,
            "sample": f"oracle fit of the first {n_records} training records of the 15k workload "
                      f"+ scoring {n_flows} held-out flows",
            "build": "gcc -O3 -march=native -fopenmp, built on this host", "cpu_model": model,
            "one_thread": {"value": v1, "seconds": dt1,
                           "sample": f"first {n_records_1t} training records + {n_flows // 3} flows"}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-148k", action="store_true", help="skip the 148k fit wall time")
    ap.add_argument("--no-serve", action="store_true", help="skip the served-scoring measurement")
    ap.add_argument("--no-batch", action="store_true", help="skip the 64-problem batched fit")
    ap.add_argument("--no-peaks", action="store_true", help="skip the measured-peak probes")
    ap.add_argument("--serve-seconds", type=float, default=2.0, help="offered load duration per rate")
    ap.add_argument("--cpu-records", type=int, default=8000, help="training records in the oracle sample")
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
    # each step's model replaces the previous one (freed once the next fit has
    # synchronised the stream, so its scoring is done); the stats are kept
    fit_stats = []
    t0 = time.perf_counter()
    for i in range(args.steps):
        m = step()
        fit_stats.append(m.stats())
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    log("timed steps done: %.2f ms/step" % ms_per_step)

    st = fit_stats[-1]
    npat = m.n_patterns()
    K = m.K
    n_flows = w.test_codes.shape[0]
    # the method's subset tests: sum of t(b) in input order (from one untimed fit on the
    # early-exit path), |P^c| * n_c support tests and |P| * n_flows scoring tests
    ref = ig.fit(d_codes, d_labels, w.nbins, kernels="valu", stream=stream)
    coh_tests = sum(ref.stats().tests)
    del ref
    n_class = list(st.n_class)
    sup_tests = npat[0] * n_class[0] + npat[1] * n_class[1]   # Eq. 2: every pattern against its class
    score_tests = (npat[0] + npat[1]) * n_flows
    tests_per_step = coh_tests + sup_tests + score_tests
    value = tests_per_step / (ms_per_step / 1e3)
    dense = st.distinct[0] * n_class[1] + st.distinct[1] * n_class[0]   # every (candidate, record) pair
    info = m.info()
    on_mfma = info.fit_words > 0             # the matrix-core kernels ran (no early exit)
    buckets = bool(info.flags & ig.IG_MODEL_FIT_BUCKETS)
    # pairs the contractions examined: all of them, or those of each candidate's bucket
    exec_coh, exec_sup = sum(st.tests), sum(st.support_tests)
    L_mfma = int(info.fit_tokens)            # tokens per operand row of the fit's contractions
    W_mfma = int(info.fit_words)             # 64-token words they occupy
    L_score = int(info.mfma_tokens)          # tokens per row of the scoring operands
    W_score = int(info.mfma_words)
    # per-kernel device time: event pairs around each launch on its stream; two
    # launches (one per class) of each contraction per fit, one scoring launch per step
    kcoh_ms = sum(fs.kernel_ms[0] for fs in fit_stats) / len(fit_stats)
    ksup_ms = sum(fs.kernel_ms[1] for fs in fit_stats) / len(fit_stats)
    score_ms = sum(a.elapsed_time(b) for a, b in score_ev[-len(fit_stats):]) / len(fit_stats)
    peaks = None if args.no_peaks else measured_peaks()
    if peaks:
        log("measured peaks", peaks)
    kernels = {}
    if on_mfma and buckets:
        # token buckets: a launch examines the pairs of each candidate with the records
        # holding its bucket token (the padding of buckets to whole tiles not counted)
        kernels["k_contain_mfma_pruned[coherence]"] = dict(ms=kcoh_ms, launches=2, tests=exec_coh,
                                                           exec_tests=exec_coh, tok=L_mfma, words=W_mfma)
        kernels["k_contain_mfma_pruned[support]"] = dict(ms=ksup_ms, launches=2, tests=exec_sup,
                                                         exec_tests=exec_sup, tok=L_mfma, words=W_mfma)
    elif on_mfma:
        # coherence: the method's tests are sum t(b); the launch executes every pair
        kernels["k_contain_mfma[coherence]"] = dict(ms=kcoh_ms, launches=2, tests=coh_tests, exec_tests=dense,
                                                    tok=L_mfma, words=W_mfma)
        kernels["k_contain_mfma[support]"] = dict(ms=ksup_ms, launches=2, tests=sup_tests, exec_tests=sup_tests,
                                                  tok=L_mfma, words=W_mfma)
    pruned = None
    if m.score_on_matrix_cores and m.bucketed:
        # pruned scoring (the default): each flow meets the buckets of its tokens only.
        # Its work is sum over (class, bucket u) of |P^c_u| * F_u pattern-flow tests
        # (F_u = test flows holding token u); the tiles execute ceil(|P^c_u| / 32) * 32
        # rows against ceil(F_u / 256) * 256 columns.
        pruned = pruned_work(m, w.test_codes, w.nbins)
        kernels["k_score_mfma_pruned"] = dict(ms=score_ms, launches=1, tests=pruned["tests"],
                                              exec_tests=pruned["exec_tests"], tok=L_score, words=W_score)
    elif m.score_on_matrix_cores:
        kernels["k_score_mfma"] = dict(ms=score_ms, launches=1, tests=score_tests, exec_tests=score_tests,
                                       tok=L_score, words=W_score)
    for k, v in kernels.items():
        v["bound"] = "mfma"
        v["unit"] = "TFLOP/s (fp4 dense)"
        v["ops"] = 2.0 * v["tok"] * v["tests"]                     # the method's operations
        v["exec_ops"] = 2.0 * 64 * v["words"] * v["exec_tests"]     # what the padded tiles execute
        sec = v["ms"] / 1e3
        v["avg_ms"] = v["ms"] / v["launches"]
        v["achieved"] = v["ops"] / sec / 1e12
        v["frac"] = v["ops"] / sec / MFMA_FP4_PEAK_OPS
        v["frac_dense"] = 2.0 * v["tok"] * v["exec_tests"] / sec / MFMA_FP4_PEAK_OPS
        v["frac_executed"] = v["exec_ops"] / sec / MFMA_FP4_PEAK_OPS
        if peaks:
            v["frac_of_measured_peak"] = v["ops"] / sec / peaks["fp4_mfma_ops_per_s"]
    res = {
        "metric": METRIC, "value": value, "unit": "subset tests/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "fp4(e2m1)->fp32 and int8->int32, exact integers",
        "data": "synthetic",
        "config": {"workload": w.name, "n_train": int(w.n), "n_flows": int(n_flows), "d": int(w.d),
                   "L": int(w.L), "K": int(K), "fit_tokens": L_mfma, "fit_words": W_mfma,
                   "score_tokens": L_score, "score_words": W_score},
        "tests_per_step": {"coherence": coh_tests, "coherence_dense": dense, "coherence_executed": exec_coh,
                           "support": sup_tests, "support_executed": exec_sup, "scoring": score_tests,
                           "scoring_executed": pruned["tests"] if pruned else score_tests},
        "fit_token_buckets": buckets,
        "patterns": list(npat), "distinct": list(st.distinct),
        "stage_ms": {k: round(v, 3) for k, v in zip(
            ["pack", "pairs", "sort", "dedup", "coherence", "order", "support", "fit_total"], st.ms)},
    }
    if kernels:
        dom = max(kernels, key=lambda k: kernels[k]["ms"])
        d = kernels[dom]
        res["roofline"] = {"bound": d["bound"], "kernel": dom, "achieved": d["achieved"],
                           "peak": MFMA_FP4_PEAK_OPS / 1e12, "unit": d["unit"], "frac": d["frac"],
                           "traffic": counted_traffic(args.traffic, dom), "avg_ms": d["avg_ms"],
                           "launches_per_step": d["launches"],
                           "tokens_per_test": d["tok"], "tests_per_launch": d["tests"] / d["launches"],
                           "frac_dense": d["frac_dense"], "frac_executed": d["frac_executed"],
                           "frac_of_measured_peak": d.get("frac_of_measured_peak")}
        res["kernels"] = {k: {x: (round(v[x], 4) if isinstance(v[x], float) else v[x])
                              for x in ("avg_ms", "launches", "achieved", "frac", "frac_dense", "frac_executed",
                                        "frac_of_measured_peak") if x in v}
                          for k, v in kernels.items()}
    if peaks:
        res["measured_peaks"] = peaks
    del m
    torch.cuda.synchronize()
    # fit alone, and from host arrays with the export; scoring alone
    res["fit_wall_s_15k"], res["fit_wall_s_15k_host_export"] = fit_wall(
        w.codes, w.labels, w.nbins, d_codes, d_labels)
    m = ig.fit(d_codes, d_labels, w.nbins)
    sw = []
    for _ in range(5):
        torch.cuda.synchronize()
        a = time.perf_counter()
        ig.score(m, d_flows, out=out)
        torch.cuda.synchronize()
        sw.append(time.perf_counter() - a)
    res["score_wall_s_15k"] = float(np.median(sw))
    res["scoring_15k"] = scoring_modes(m, d_flows, out)
    res["detection_15k"] = detection(m, d_codes, d_labels, d_flows, w.test_labels)
    res["evidence_15k"] = evidence_time(m, d_flows[:512], 16)
    log("15k scoring", res["scoring_15k"], "detection", res["detection_15k"], "evidence", res["evidence_15k"])
    del m
    log("15k fit %.1f ms (device inputs), %.1f ms (host arrays + export), score %.1f ms" % (
        res["fit_wall_s_15k"] * 1e3, res["fit_wall_s_15k_host_export"] * 1e3, res["score_wall_s_15k"] * 1e3))
    if not args.no_148k:
        w2 = synth.make_148k()
        log("148k workload", w2.codes.shape)
        dc2 = torch.from_numpy(w2.codes.view(np.int16)).cuda()
        dl2 = torch.from_numpy(w2.labels).cuda()
        m2 = ig.fit(dc2, dl2, w2.nbins)   # warm (allocations, code load)
        del m2
        res["fit_wall_s_148k"], res["fit_wall_s_148k_host_export"] = fit_wall(
            w2.codes, w2.labels, w2.nbins, dc2, dl2)
        m2 = ig.fit(dc2, dl2, w2.nbins)
        st2 = m2.stats()
        res["fit_148k"] = {"n_train": int(w2.n), "patterns": list(m2.n_patterns()), "tests_executed": list(st2.tests),
                           "coherence_kernel_ms": st2.kernel_ms[0], "support_kernel_ms": st2.kernel_ms[1]}
        d_f2 = torch.from_numpy(w2.test_codes.view(np.int16)).cuda()
        out2 = torch.empty((w2.test_codes.shape[0], 2), dtype=torch.int64, device="cuda")
        ig.score(m2, d_f2, out=out2)
        torch.cuda.synchronize()
        a = time.perf_counter()
        ig.score(m2, d_f2, out=out2)
        torch.cuda.synchronize()
        res["score_wall_s_148k"] = time.perf_counter() - a
        res["fit_148k"]["score_tests"] = sum(m2.n_patterns()) * int(w2.test_codes.shape[0])
        res["scoring_148k"] = scoring_modes(m2, d_f2, out2, reps=2)
        res["detection_148k"] = detection(m2, dc2, dl2, d_f2, w2.test_labels)
        log("148k scoring", res["scoring_148k"], "detection", res["detection_148k"])
        del m2, d_f2, out2
        log("148k fit %.1f ms, score of %d flows %.1f ms" % (res["fit_wall_s_148k"] * 1e3, w2.test_codes.shape[0],
                                                             res["score_wall_s_148k"] * 1e3))
    if not args.no_serve:
        res["serve"] = measure_serving(args.serve_seconds)
    if not args.no_cpu:
        res["cpu_baseline"] = cpu_baseline(w, min(args.cpu_records, w.n), 300, 2500)
    if not args.no_batch:
        torch.cuda.synchronize()
        res["batch"] = measure_batch()
        log("batch", res["batch"])
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
