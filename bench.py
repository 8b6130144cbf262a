#!/usr/bin/env python3
"""Benchmark of the multi-component progressive codec on one MI355X.

One step = the whole hot path over one field: range (tau_0, Sec. 5.1), Alg. 1
compression into n components (Sec. 4.1), then Alg. 2 retrieval at every
k = 1..n from scratch (Sec. 4.2).  Default workload: 512^3 float32 spectral
field (E(k) ~ k^-5/3, normalised to [-1, 1]), 8 components, tau_i = 2^-3i.

value = raw field bytes pushed through the codec per second:
        N*s * (1 compression + n retrievals) / step time   [GB/s]

Prints ONE JSON line on stdout; progress goes to stderr.
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


WORKLOADS = {
    # name: (shape, dtype, seed, n, tau(i, range), noise)
    "bulk_512_f32": ((512, 512, 512), np.float32, 1, 8, lambda i, r: 2.0 ** (-3 * i), 0.0),
    "bulk_256_f64": ((256, 256, 256), np.float64, 2, 8, lambda i, r: 2.0 ** (-3 * i), 0.0),
    "small_64_f64": (None, np.float64, 0, 4, lambda i, r: r * 10.0 ** -i, 0.0),
    "largest_1024_f32": ((1024, 1024, 1024), np.float32, 3, 12, lambda i, r: 2.0 ** (-2 * i), 1e-4),
    "largest_768_f64": ((768, 768, 768), np.float64, 4, 10, lambda i, r: 2.0 ** (-2 * i), 1e-4),
    "batched_256": None,
    "served_64": None,
}
TAU_TEXT = {"bulk_512_f32": "2^-3i", "bulk_256_f64": "2^-3i", "small_64_f64": "range*10^-i",
            "largest_1024_f32": "2^-2i", "largest_768_f64": "2^-2i"}


def make_field(name):
    from paper_2308_11759_amd import inputs
    shape, dt, seed, n, taufn, noise = WORKLOADS[name]
    if shape is None:
        return inputs.blobs_field(64, seed=seed, dtype=dt)
    return inputs.spectral_field(shape, seed=seed, dtype=dt, noise_rel=noise)


def source_sha():
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_2308_11759_amd", "csrc")
    for f in sorted(os.listdir(d)):
        if f.endswith((".hip", ".hpp", ".cpp")):
            h.update(open(os.path.join(d, f), "rb").read())
    return h.hexdigest()[:16]


def load_traffic(kernel, workload):
    """HBM bytes per launch measured by rocprofv3 --pmc (FETCH_SIZE, WRITE_SIZE),
    committed under profiles/; null when the kernel sources changed since."""
    p = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(p):
        return None
    try:
        t = json.load(open(p))
    except ValueError:
        return None
    e = t.get(workload, {}).get(kernel)
    if not e or e.get("source_sha") != source_sha():
        return None
    return e.get("bytes_per_launch")


# vector ALU issue rate: 1024 SIMDs (256 CUs x 4), one wave64 instruction per
# SIMD every 4 cycles at 2.4 GHz
VALU_WAVE_INSTR_PER_S = 1024 * 2.4e9 / 4


def load_valu_instructions(kernel, workload):
    """VALU wave-instructions per launch counted by rocprofv3 --pmc
    (SQ_INSTS_VALU), committed under profiles/; null when the kernel sources
    changed since."""
    p = os.path.join(ROOT, "profiles", "instructions.json")
    if not os.path.exists(p):
        return None
    try:
        t = json.load(open(p))
    except ValueError:
        return None
    e = t.get(workload, {}).get(kernel)
    if not e or e.get("source_sha") != source_sha():
        return None
    return e.get("valu_instr_per_launch")


def cpu_baseline(x, taus, planes, pool_planes):
    """The oracle as it stands on a z-slab of the same field: on all host
    cores (its serial driver over independent chunk-aligned sub-slabs on a
    thread pool, the unchanged serial code per sub-slab) and on one core.
    Work per value is the bench step's: compress n components, retrieve
    k = 1..n from scratch."""
    from oracle import driver, pool
    n = len(taus)

    def one(xs):
        comps, meta = driver.compress(xs, taus)
        for k in range(1, n + 1):
            driver.reconstruct(comps, k, xs.shape, xs.dtype)

    res = None
    if pool_planes > 0:
        xs = np.ascontiguousarray(x[:pool_planes])
        sub = pool.slab_planes(xs.shape)
        parts = pool.slabs(xs.shape, sub)
        cores = min(os.cpu_count() or 1, len(parts))
        from concurrent.futures import ThreadPoolExecutor
        t0 = time.perf_counter()
        with ThreadPoolExecutor(max_workers=cores) as ex:
            list(ex.map(lambda zz: one(np.ascontiguousarray(xs[zz[0]:zz[1]])), parts))
        dt = time.perf_counter() - t0
        res = {"value": xs.nbytes * (1 + n) / dt / 1e9, "unit": "GB/s", "cores": cores, "kind": "oracle",
               "sample": "z-slab %dx%dx%d of the same field (%d values) as %d independent %d-plane slabs on %d "
                         "threads, compress %d components + retrieve k=1..%d, %.1f s" %
                         (xs.shape[0], xs.shape[1], xs.shape[2], xs.size, len(parts), sub, cores, n, n, dt)}
    if planes > 0:
        xs = np.ascontiguousarray(x[:planes])
        t0 = time.perf_counter()
        one(xs)
        dt = time.perf_counter() - t0
        single = {"value": xs.nbytes * (1 + n) / dt / 1e9, "unit": "GB/s", "cores": 1, "kind": "oracle",
                  "sample": "z-slab %dx%dx%d of the same field (%d values), compress %d components + retrieve "
                            "k=1..%d, %.1f s" % (xs.shape[0], xs.shape[1], xs.shape[2], xs.size, n, n, dt)}
        if res is None:
            return single
        res["single_core"] = single
    return res


def batched_measure(ctx, nfields, steps, warmup):
    """256 fields, edges log-uniform in [16, 256] per axis, f32/f64 alternating,
    6 components, tau_i = range_f * 4^-i: one tuned graph per call vs a loop
    of single-field compressions (the same kernels, one pmc_compress each)."""
    import torch
    from paper_2308_11759_amd import inputs
    dev = ctx.device
    shapes = inputs.batched_shapes(nfields)
    log("batched: generating %d fields" % len(shapes))
    xs, taus = [], []
    for f, (shape, is32) in enumerate(shapes):
        xh = inputs.spectral_field(shape, seed=100 + f, dtype=np.float32 if is32 else np.float64)
        r = float(xh.max()) - float(xh.min())
        xs.append(torch.from_numpy(xh).to(dev))
        taus.append([r * 4.0 ** -i for i in range(1, 7)])
    total = sum(x.numel() * x.element_size() for x in xs)
    nval = sum(x.numel() for x in xs)
    batch = ctx.batch([(tuple(x.shape), x.dtype) for x in xs], taus)
    streams = torch.empty_like(batch.streams)
    log("batched: tuning (12 schedules)")
    gm, order, tms = batch.tune(xs)
    log("batched: tuned grid x%d, order %d, graph %.3f ms" % (gm, order, tms))
    for _ in range(warmup):
        batch.compress(xs, streams=streams)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        stores = batch.compress(xs, streams=streams)
    torch.cuda.synchronize()
    t_batch = (time.perf_counter() - t0) / steps
    outs = [torch.empty(ctx.compress_sizes(x, 6)[1] * 6, dtype=torch.uint8, device=dev) for x in xs]
    for x, t, o in zip(xs, taus, outs):
        ctx.compress(x, t, streams=o)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        singles = [ctx.compress(x, t, streams=o) for x, t, o in zip(xs, taus, outs)]
    torch.cuda.synchronize()
    t_loop = (time.perf_counter() - t0) / steps
    same = all(bool(torch.equal(a.stream(i), b.stream(i))) for a, b in zip(stores, singles) for i in range(6))
    sbytes = sum(m["bytes"] for st in stores for m in st.info)
    res = {"fields": len(xs), "values": nval, "bytes": total, "components": 6, "steps": steps,
           "schedule": {"grid_mult": gm, "order": order}, "tuned_graph_ms": tms,
           "ms_per_call": t_batch * 1e3, "gbs": total / t_batch / 1e9,
           "per_field_loop_ms": t_loop * 1e3, "per_field_loop_gbs": total / t_loop / 1e9,
           "speedup_vs_loop": t_loop / t_batch, "identical_to_single_field": same,
           "rate_bits_per_value": 8.0 * sbytes / nval}
    del stores, singles, outs, streams, batch, xs
    return res


def bench_batched(args):
    from paper_2308_11759_amd import pmc
    ctx = pmc.Context(0)
    b = batched_measure(ctx, args.fields, args.steps, args.warmup)
    rec = {"metric": "batched compress GB/s (256 mixed fields, 6 comps)", "value": b["gbs"],
           "unit": "GB/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": b["ms_per_call"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f32+f64", "data": "synthetic",
           "config": {"workload": "batched_256", "fields": b["fields"], "values": b["values"], "components": 6,
                      "schedule": b["schedule"]},
           "per_field_loop_gbs": b["per_field_loop_gbs"], "speedup_vs_loop": b["speedup_vs_loop"],
           "identical_to_single_field": b["identical_to_single_field"],
           "rate_bits_per_value": b["rate_bits_per_value"]}
    print(json.dumps(rec))


def build_served_store(ctx):
    """64 stored fields: cubic, edge log-uniform in [64, 384], f32/f64
    alternating, 10 components, tau_i = range * 10^(-i/2)."""
    import torch
    from paper_2308_11759_amd import inputs
    shapes = inputs.served_shapes(64)
    stores, ranges, nbytes = [], [], []
    log("served: building the store of %d fields" % len(shapes))
    for f, (shape, is32) in enumerate(shapes):
        xh = inputs.spectral_field(shape, seed=200 + f, dtype=np.float32 if is32 else np.float64)
        r = float(xh.max()) - float(xh.min())
        x = torch.from_numpy(xh).to(ctx.device)
        taus = [r * 10.0 ** (-i / 2.0) for i in range(1, 11)]
        stores.append(ctx.compress(x, taus))
        ranges.append(r)
        nbytes.append(x.numel() * x.element_size())
        del x, xh
        if f % 16 == 15:
            log("served:   %d fields stored" % (f + 1))
    torch.cuda.synchronize()
    return stores, ranges, nbytes


def served_measure(ctx, stores, ranges, nbytes, lam, nqueries, arena_gb):
    """One open-loop Poisson trace (field uniform, tolerance log-uniform in
    [1e-5, 1e-1] * range) replayed twice on the same GPU.  Served: the
    library's request loop (continuous batching, device partial-sum cache,
    HBM budget = arena).  Plain: first come first served, one Alg. 2 retrieval
    from scratch per query.  Both latencies run from the trace's scheduled
    arrival on the library's clock to completion, so a submitter running late
    counts against both forms alike."""
    import threading
    import torch
    from paper_2308_11759_amd import inputs, pmc
    trace = inputs.query_trace(len(stores), lam, nqueries, seed=7 + lam)
    trace = [(t, f, rel * ranges[f]) for t, f, rel in trace]
    out_bytes = sum(nbytes[f] for _, f, _ in trace)
    # served
    srv = pmc.Server(ctx, arena_bytes=arena_gb << 30, budget_bytes=arena_gb << 30, max_batch=64)
    for st in stores:
        srv.add(st)
    tickets = [None] * len(trace)
    lat = [None] * len(trace)
    t0 = pmc.clock() + 0.05

    def submitter():
        for i, (ta, f, tol) in enumerate(trace):
            d = t0 + ta - pmc.clock()
            if d > 0:
                time.sleep(d)
            tickets[i] = srv.submit(f, tol, arrival=t0 + ta)

    th = threading.Thread(target=submitter)
    th.start()
    outstanding = set()
    nsub = 0
    done = 0
    while done < len(trace):
        while nsub < len(trace) and tickets[nsub] is not None:
            outstanding.add(nsub)
            nsub += 1
        finished = []
        for i in outstanding:
            d, st, l = srv.poll(tickets[i])
            if d:
                assert st == pmc.OK, st
                lat[i] = l
                srv.release(tickets[i])
                finished.append(i)
        for i in finished:
            outstanding.discard(i)
        done += len(finished)
        if not finished:
            time.sleep(0.0005)
    th.join()
    makespan = pmc.clock() - t0
    sstats = srv.stats()
    srv.close()
    served = {"p50_ms": 1e3 * float(np.percentile(lat, 50)), "p99_ms": 1e3 * float(np.percentile(lat, 99)),
              "gbs": out_bytes / makespan / 1e9, "makespan_s": makespan,
              "hits": sstats["hits"], "partial": sstats["partial"], "misses": sstats["misses"],
              "steps": sstats["steps"], "max_queue": sstats["max_queue"]}
    # plain: FIFO, one retrieval from scratch per query
    outs = [torch.empty(st.shape, dtype=st.dtype, device=ctx.device) for st in stores]
    plat = []
    torch.cuda.synchronize()
    t0 = pmc.clock() + 0.05
    for ta, f, tol in trace:
        d = t0 + ta - pmc.clock()
        if d > 0:
            time.sleep(d)
        k = stores[f].select_k(tol)
        ctx.retrieve(stores[f], k, out=outs[f])
        torch.cuda.synchronize()
        plat.append(pmc.clock() - (t0 + ta))
    pmake = pmc.clock() - t0
    plain = {"p50_ms": 1e3 * float(np.percentile(plat, 50)), "p99_ms": 1e3 * float(np.percentile(plat, 99)),
             "gbs": out_bytes / pmake / 1e9, "makespan_s": pmake}
    del outs
    log("served %d QPS, %d queries: served p50 %.3f ms p99 %.3f ms | plain p50 %.3f ms p99 %.3f ms" %
        (lam, nqueries, served["p50_ms"], served["p99_ms"], plain["p50_ms"], plain["p99_ms"]))
    return {"rate_qps": lam, "queries": nqueries, "latency_from": "scheduled arrival", "served": served,
            "plain": plain}


def bench_served(args):
    from paper_2308_11759_amd import pmc
    ctx = pmc.Context(0)
    stores, ranges, nbytes = build_served_store(ctx)
    rates = [int(v) for v in args.rates.split(",")]
    results = {}
    for lam in rates:
        results[str(lam)] = served_measure(ctx, stores, ranges, nbytes, lam, args.queries, args.arena_gb)
    top = results[str(rates[-1])]
    rec = {"metric": "query p99 latency, served vs plain (64 fields, 10 comps)",
           "value": top["served"]["p99_ms"], "unit": "ms", "n_gpus": 1, "steps": args.queries, "warmup": 0,
           "ms_per_step": None, "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
           "dtype": "f32+f64", "data": "synthetic",
           "config": {"workload": "served_64", "queries_per_rate": args.queries, "rates_qps": rates,
                      "budget_gb": args.arena_gb},
           "plain_p99_ms": top["plain"]["p99_ms"], "per_rate": results}
    print(json.dumps(rec))


def rate_distortion(ctx, xd, rng, depth, out):
    """Sec. 5.1's rate-distortion comparison on one field: multi-component
    stores at granularity Delta in {4, 6, 8} (tau_i = 2^(-Delta i) * range, i = 1
    .. depth / Delta) against single-component compressions at
    tau = 2^(-2j) * range (Delta = 2), each run from scratch.  Per point: the
    rate in bits/value (cumulative for a store), the accuracy gain of Sec.
    5.1.1 and the measured max error over tau; and for each store point the
    extra bits/value it spends over the single-component run at the same tau."""
    N = xd.numel()

    def points(store):
        res = {"rate": [], "gain": [], "err_over_tau": []}
        bits = 0
        for k in range(1, store.n + 1):
            m = store.info[k - 1]
            bits += 8 * m["bytes"]
            ctx.retrieve(store, k, out=out)
            _, _, g = ctx.accuracy_gain(xd, out, bits / N)
            res["rate"].append(round(bits / N, 4))
            res["gain"].append(round(g, 4))
            res["err_over_tau"].append(round(m["linf"] / m["tau"], 4))
        return res

    rd = {"depth_bits": depth}
    single = {"rate": [], "gain": [], "err_over_tau": []}
    for j in range(1, depth // 2 + 1):
        st = ctx.compress(xd, [rng * 2.0 ** (-2 * j)])
        p = points(st)
        for key in single:
            single[key] += p[key]
        del st
    rd["single_delta2"] = single
    for delta in (4, 6, 8):
        st = ctx.compress(xd, [rng * 2.0 ** (-delta * i) for i in range(1, depth // delta + 1)])
        p = points(st)
        del st
        # tau_i of the store equals tau_j of the single runs at j = Delta i / 2
        p["overhead_bits"] = [round(r - single["rate"][delta * i // 2 - 1], 4)
                              for i, r in enumerate(p["rate"], start=1)]
        rd["multi_delta%d" % delta] = p
    return rd


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="bulk_512_f32", choices=sorted(WORKLOADS))
    ap.add_argument("--cpu-planes", type=int, default=16, help="z-planes of the one-core oracle sample (0 = skip)")
    ap.add_argument("--cpu-pool-planes", type=int, default=64,
                    help="z-planes of the all-cores oracle sample (0 = skip)")
    ap.add_argument("--literal", action="store_true", help="one decode pass per component (literal Alg. 2)")
    ap.add_argument("--refine-reps", type=int, default=3,
                    help="repetitions of the incremental refine chain k = 1..n timed after the steps (0 = skip)")
    ap.add_argument("--fields", type=int, default=256, help="batched workload: number of fields")
    ap.add_argument("--queries", type=int, default=10000, help="served workload: queries per arrival rate")
    ap.add_argument("--rates", default="200,500,1000,2000", help="served workload: arrival rates (QPS)")
    ap.add_argument("--arena-gb", type=int, default=64, help="served workload: cache arena and budget")
    ap.add_argument("--served-rate", type=int, default=2000,
                    help="default workload: arrival rate of the served sub-measurement (0 = skip)")
    ap.add_argument("--batched-fields", type=int, default=256,
                    help="default workload: fields of the batched sub-measurement (0 = skip)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run three 512 MiB device-to-device copies (scale for rocprofv3 byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: there is no multi-GPU path (a field would be split into "
              "z-slabs, one per GPU, with only the range and the stream sizes exchanged).", file=sys.stderr)
        sys.exit(2)

    if args.workload == "batched_256":
        return bench_batched(args)
    if args.workload == "served_64":
        return bench_served(args)

    import torch
    from paper_2308_11759_amd import inputs, pmc

    shape, dt, seed, n, taufn, noise = WORKLOADS[args.workload]
    log("generating %s" % args.workload)
    x = make_field(args.workload)
    rng = float(x.max()) - float(x.min())
    taus = [taufn(i, rng) for i in range(1, n + 1)]
    dev = torch.device("cuda", 0)
    xd = torch.from_numpy(x).to(dev)
    N, s = x.size, x.itemsize
    ctx = pmc.Context(0)
    if args.literal:
        ctx.set_option(pmc.OPT_FUSED_DECODE, 0)
    ws_bytes, cap1 = ctx.compress_sizes(xd, n)
    streams = torch.empty(cap1 * n, dtype=torch.uint8, device=dev)
    out = torch.empty_like(xd)
    log("field %s %s, %d components, ws %.2f GB, stream cap %.2f GB" %
        (x.shape, x.dtype, n, ws_bytes / 1e9, streams.numel() / 1e9))

    def step():
        ctx.range(xd)
        st = ctx.compress(xd, taus, streams=streams)
        for k in range(1, n + 1):
            ctx.retrieve(st, k, out=out)
        return st

    store = None
    for w in range(args.warmup):
        store = step()
        torch.cuda.synchronize()
        log("warmup %d done" % w)
    if store is None:
        store = ctx.compress(xd, taus, streams=streams)
    # parity probe at full size: Eq. (1) for every k, on the device; and the
    # accuracy gain of each x~_k at its cumulative rate (Sec. 5.1.1)
    gain = {"sigma": None, "rate_bits_per_value": [], "rmse": [], "gain": []}
    bits = 0
    for k in range(1, n + 1):
        ctx.retrieve(store, k, out=out)
        err = float((xd.double() - out.double()).abs().max())
        assert err <= taus[k - 1], (k, err, taus[k - 1])
        assert err == store.info[k - 1]["linf"], (k, err, store.info[k - 1]["linf"])
        bits += 8 * store.info[k - 1]["bytes"]
        sigma, rmse, g = ctx.accuracy_gain(xd, out, bits / x.size)
        gain["sigma"] = sigma
        gain["rate_bits_per_value"].append(round(bits / x.size, 4))
        gain["rmse"].append(rmse)
        gain["gain"].append(round(g, 4))
    torch.cuda.synchronize()

    ctx.set_option(pmc.OPT_PROFILE, 1)
    ctx.prof_read(reset=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for i in range(args.steps):
        store = step()
    ev1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_step = ev0.elapsed_time(ev1) / args.steps
    prof = ctx.prof_read(reset=True)
    ctx.set_option(pmc.OPT_PROFILE, 0)
    log("timed %d steps: %.3f ms/step (wall %.3f s)" % (args.steps, ms_step, wall))

    info = store.info
    nchunks = ((x.shape[2] + 3) // 4 * ((x.shape[1] + 3) // 4) * ((x.shape[0] + 3) // 4) + 15) // 16
    payload = [(m["bytes"] - 64 - 4 * nchunks) for m in info]
    # algorithmic bytes per step for each kernel
    enc_bytes = sum(N * s * (1 + (i > 0) + (i < n - 1)) + payload[i] + 4 * nchunks for i in range(n))
    if args.literal:
        dec_bytes = sum(sum(info[i]["bytes"] + (N * s if i > 0 else 0) + N * s for i in range(k))
                        for k in range(1, n + 1))
    else:
        dec_bytes = sum(sum(info[i]["bytes"] for i in range(k)) + N * s for k in range(1, n + 1))
    tname = "f32" if dt == np.float32 else "f64"
    kern = {}
    for name, (launches, ms) in prof.items():
        kern[name] = {"launches_per_step": launches / args.steps, "ms_per_step": ms / args.steps,
                      "avg_launch_ms": ms / max(launches, 1)}
    algo = {"k_encode_" + tname: enc_bytes, "k_decode_" + tname: dec_bytes}
    for name, b in algo.items():
        if name in kern:
            kern[name]["algorithmic_gb_per_step"] = b / 1e9
            kern[name]["achieved_gbs"] = b / 1e9 / (kern[name]["ms_per_step"] / 1e3)
    dom = max(algo, key=lambda k: kern.get(k, {}).get("ms_per_step", 0.0))
    dk = kern[dom]
    launches = dk["launches_per_step"]
    achieved = dk["achieved_gbs"]
    traffic = load_traffic(dom, args.workload)
    roofline = {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                "traffic_gbs": traffic / 1e9 / (dk["avg_launch_ms"] / 1e3) if traffic else None,
                "traffic_frac": traffic / 1e9 / (dk["avg_launch_ms"] / 1e3) / HBM_PEAK_GBS if traffic else None,
                "algorithmic_bytes_per_launch": algo[dom] / launches, "avg_launch_ms": dk["avg_launch_ms"]}
    # the vector ALUs' share of the launch: counted VALU instructions at the
    # issue rate over the live launch time (the kernels are VALU-bound below
    # the HBM roof)
    vi = load_valu_instructions(dom, args.workload)
    roofline["valu_issue_frac"] = vi / VALU_WAVE_INSTR_PER_S / (dk["avg_launch_ms"] / 1e3) if vi else None

    comp_ms = sum(kern.get(k, {}).get("ms_per_step", 0.0) for k in
                  ("k_encode_" + tname, "k_scan", "k_pack_" + tname))
    dec_ms = kern.get("k_decode_" + tname, {}).get("ms_per_step", 0.0)
    value = N * s * (1 + n) / (ms_step / 1e3) / 1e9

    # incremental refine (Alg. 2 continued from x~_{k-1}): one component per
    # call, k = 1..n, reported beside the from-scratch retrievals of the step
    refine_ms = None
    if args.steps > 0 and args.refine_reps > 0:
        ev2, ev3 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        reps = args.refine_reps
        ev2.record()
        for _ in range(reps):
            ctx.retrieve(store, 1, out=out)
            for k in range(2, n + 1):
                ctx.refine(store, k - 1, k, out)
        ev3.record()
        torch.cuda.synchronize()
        refine_ms = ev2.elapsed_time(ev3) / reps
        err = float((xd.double() - out.double()).abs().max())
        assert err == store.info[n - 1]["linf"], (err, store.info[n - 1]["linf"])

    # region retrieval (Sec. 6.1): x~_n on a 64^3 box (or the whole field if
    # smaller), decoding only the blocks that meet it
    region = None
    if args.steps > 0 and args.refine_reps > 0:
        edge = [min(64, d) for d in x.shape[::-1]]  # x, y, z
        lo = [(d - e) // 2 for d, e in zip(x.shape[::-1], edge)]
        hi = [l + e for l, e in zip(lo, edge)]
        box = ctx.retrieve_box(store, n, lo, hi)
        torch.cuda.synchronize()
        ev4, ev5 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev4.record()
        for _ in range(5):
            ctx.retrieve_box(store, n, lo, hi, out=box)
        ev5.record()
        torch.cuda.synchronize()
        full = ctx.retrieve(store, n)
        assert torch.equal(box, full[lo[2]:hi[2], lo[1]:hi[1], lo[0]:hi[0]])
        del full
        region = {"box_lo_xyz": lo, "box_hi_xyz": hi, "k": n, "ms": ev4.elapsed_time(ev5) / 5,
                  "box_fraction": float(np.prod(edge)) / x.size}

    # lossless limit (Sec. 5.1.3): the bench's schedule, then steps of 2^-16
    # down to 2^-152, below every float32 difference; report the first k with
    # x~_k == x bit for bit, and the ratio there
    lossless = None
    if args.steps > 0 and args.refine_reps > 0 and dt == np.float32 and args.workload.startswith("bulk"):
        ltaus = list(taus) + [taus[-1] * 2.0 ** (-16 * j) for j in range(1, 9)]
        lws, lcap = ctx.compress_sizes(xd, len(ltaus))
        lstreams = torch.empty(lcap * len(ltaus), dtype=torch.uint8, device=dev)
        lstore = ctx.compress(xd, ltaus, streams=lstreams)
        first = None
        for k in range(1, len(ltaus) + 1):
            if torch.equal(ctx.retrieve(lstore, k, out=out), xd):  # zero error (the sign of zero is not kept)
                first = k
                break
        if first is not None:
            nbytes = sum(m["bytes"] for m in lstore.info[:first])
            lossless = {"components": len(ltaus), "first_exact_k": first, "tau_first_exact": ltaus[first - 1],
                        "bytes": nbytes, "ratio": N * s / nbytes}
        del lstore, lstreams
        # a schedule aimed at the lossless end: three components, the last
        # below every float32 difference (2^-150), the middle one where the
        # residual is left with few bits (picked on an oracle sample of the
        # same field from 2^-a, 2^-b with a in 8..14, b in 26..36)
        ttaus = [2.0 ** -8, 2.0 ** -32, 2.0 ** -150]
        lws, lcap = ctx.compress_sizes(xd, 3)
        lstreams = torch.empty(lcap * 3, dtype=torch.uint8, device=dev)
        tstore = ctx.compress(xd, ttaus, streams=lstreams)
        exact = bool(torch.equal(ctx.retrieve(tstore, 3, out=out), xd))
        tbytes = sum(m["bytes"] for m in tstore.info)
        targeted = {"taus": ttaus, "exact_at_3": exact, "bytes": tbytes, "ratio": N * s / tbytes,
                    "rates_bits_per_value": [round(8.0 * m["bytes"] / N, 3) for m in tstore.info]}
        if lossless is None:
            lossless = {}
        lossless["targeted_schedule"] = targeted
        del tstore, lstreams

    # the second compressor (Sec. 3's float32 cast) on float64 fields: three
    # components, timed; x~_3 must equal x for normal values
    cast = None
    if args.steps > 0 and args.refine_reps > 0 and dt == np.float64:
        comps, clinf = ctx.cast_compress(xd, 3)
        torch.cuda.synchronize()
        ev6, ev7 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev6.record()
        for _ in range(5):
            comps, clinf = ctx.cast_compress(xd, 3)
        ev7.record()
        torch.cuda.synchronize()
        cms = ev6.elapsed_time(ev7) / 5
        exact = bool(torch.equal(ctx.cast_retrieve(comps, 3, out), xd))
        cast = {"components": 3, "ms": cms, "gbs": (N * s + 3 * N * 4) / (cms / 1e3) / 1e9,
                "linf": clinf, "exact_at_3": exact}
        del comps

    # rate-distortion of multi-component stores against single-component
    # runs (Sec. 5.1), over 24 bits of the range (float32) or 48 (float64)
    rdist = None
    if args.steps > 0 and args.refine_reps > 0 and args.workload.startswith("bulk"):
        rdist = rate_distortion(ctx, xd, rng, 24 if dt == np.float32 else 48, out)

    # the second codec (prediction and quantisation) behind the same driver,
    # on the same field and schedule: one step = compress + retrieve k = 1..n
    pred = None
    if args.steps > 0 and args.refine_reps > 0 and args.workload.startswith("bulk"):
        ctx.set_option(pmc.OPT_CODEC, pmc.CODEC_PREDICTION)
        pstreams = torch.empty(cap1 * n, dtype=torch.uint8, device=dev)
        pstore = ctx.compress(xd, taus, streams=pstreams)
        for k in range(1, n + 1):
            ctx.retrieve(pstore, k, out=out)
        torch.cuda.synchronize()
        err = float((xd.double() - out.double()).abs().max())
        assert err == pstore.info[n - 1]["linf"] <= taus[n - 1]
        reps = 5
        ctx.set_option(pmc.OPT_PROFILE, 1)
        ctx.prof_read(reset=True)
        ev8, ev9 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev8.record()
        for _ in range(reps):
            pstore = ctx.compress(xd, taus, streams=pstreams)
            for k in range(1, n + 1):
                ctx.retrieve(pstore, k, out=out)
        ev9.record()
        torch.cuda.synchronize()
        pprof = ctx.prof_read(reset=True)
        ctx.set_option(pmc.OPT_PROFILE, 0)
        ctx.set_option(pmc.OPT_CODEC, pmc.CODEC_TRANSFORM)
        pms = ev8.elapsed_time(ev9) / reps
        pk = {name: {"launches_per_step": l / reps, "ms_per_step": m / reps, "avg_launch_ms": m / max(l, 1)}
              for name, (l, m) in pprof.items()}
        penc = sum(pk.get(kk, {}).get("ms_per_step", 0.0) for kk in ("k_encode_pq_" + tname, "k_scan",
                                                                      "k_pack_" + tname))
        pdec = pk.get("k_decode_pq_" + tname, {}).get("ms_per_step", 0.0)
        pred = {"ms_per_step": pms, "gbs": N * s * (1 + n) / (pms / 1e3) / 1e9,
                "compress_gbs": N * s / (penc / 1e3) / 1e9 if penc else None,
                "retrieve_all_k_gbs": N * s * n / (pdec / 1e3) / 1e9 if pdec else None,
                "rates_bits_per_value": [round(8.0 * m["bytes"] / N, 3) for m in pstore.info],
                "linf": [m["linf"] for m in pstore.info],
                "escalated_blocks": [m["nesc"] for m in pstore.info], "raw_blocks": [m["nraw"] for m in pstore.info],
                "kernels": pk}
        del pstore, pstreams

    if args.copy_calibration:
        src = torch.empty(512 << 20, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    cpu = None
    if args.cpu_planes > 0 or args.cpu_pool_planes > 0:
        log("oracle baseline on %d z-planes (all cores) and %d (one core)" % (args.cpu_pool_planes, args.cpu_planes))
        cpu = cpu_baseline(x, taus, args.cpu_planes, args.cpu_pool_planes)

    # the other half of the headline metric, on the same GPU: many fields
    # coded in one captured launch (batched), and progressive-retrieval
    # queries served with continuous batching against plain retrieval
    batched = served = None
    if args.workload == "bulk_512_f32" and args.steps > 0 and (args.batched_fields > 0 or args.served_rate > 0):
        del store, streams, out
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
        if args.batched_fields > 0:
            batched = batched_measure(ctx, args.batched_fields, steps=5, warmup=2)
        if args.served_rate > 0:
            sstores, sranges, snbytes = build_served_store(ctx)
            served = served_measure(ctx, sstores, sranges, snbytes, args.served_rate, args.queries, args.arena_gb)
            served["fields"] = len(sstores)
            del sstores

    rec = {
        "metric": "compress/retrieve GB/s (%d^3 %s, %d comps)" % (x.shape[0], "f32" if dt == np.float32 else "f64", n),
        "value": value,
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if dt == np.float32 else "f64",
        "data": "synthetic",
        "config": {"workload": args.workload, "shape": list(x.shape), "components": n,
                   "tau": TAU_TEXT[args.workload],
                   "decode": "literal" if args.literal else "fused", "step": "range + compress + retrieve k=1..n"},
        "compress_gbs": N * s / (comp_ms / 1e3) / 1e9 if comp_ms else None,
        "retrieve_all_k_gbs": N * s * n / (dec_ms / 1e3) / 1e9 if dec_ms else None,
        "refine_chain_gbs": N * s * n / (refine_ms / 1e3) / 1e9 if refine_ms else None,
        "refine_chain_ms": refine_ms,
        "region_retrieval": region,
        "lossless": lossless,
        "cast_codec": cast,
        "prediction_codec": pred,
        "rate_distortion": rdist,
        "lag1_autocorrelation_xyz": [round(v, 4) for v in inputs.lag1_autocorrelation(x)],
        "rates_bits_per_value": [round(8.0 * m["bytes"] / N, 3) for m in info],
        "linf": [m["linf"] for m in info],
        "accuracy_gain": gain,
        "kernels": kern,
        "roofline": roofline,
        "cpu_baseline": cpu,
        "batched": batched,
        "served": served,
    }
    print(json.dumps(rec))


if __name__ == "__main__":
    main()
