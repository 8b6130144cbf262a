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
}


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


def cpu_baseline(x, taus, planes):
    """The oracle as it stands, single-threaded, on a z-slab of the same field."""
    from oracle import driver
    xs = np.ascontiguousarray(x[:planes])
    n = len(taus)
    t0 = time.perf_counter()
    comps, meta = driver.compress(xs, taus)
    for k in range(1, n + 1):
        driver.reconstruct(comps, k, xs.shape, xs.dtype)
    dt = time.perf_counter() - t0
    gbs = xs.nbytes * (1 + n) / dt / 1e9
    return {"value": gbs, "unit": "GB/s", "cores": 1, "kind": "oracle",
            "sample": "z-slab %dx%dx%d of the same field (%d values), compress %d components + retrieve "
                      "k=1..%d, %.1f s" % (xs.shape[0], xs.shape[1], xs.shape[2], xs.size, n, n, dt)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="bulk_512_f32", choices=sorted(WORKLOADS))
    ap.add_argument("--cpu-planes", type=int, default=8, help="z-planes of the oracle sample (0 = skip)")
    ap.add_argument("--literal", action="store_true", help="one decode pass per component (literal Alg. 2)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path (the field would be split "
              "into z-slabs, one per GPU; see DESIGN.md).", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2308_11759_amd import pmc

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

    for w in range(args.warmup):
        store = step()
        torch.cuda.synchronize()
        log("warmup %d done" % w)
    # parity probe at full size: Eq. (1) for every k, on the device
    for k in range(1, n + 1):
        ctx.retrieve(store, k, out=out)
        err = float((xd.double() - out.double()).abs().max())
        assert err <= taus[k - 1], (k, err, taus[k - 1])
        assert err == store.info[k - 1]["linf"], (k, err, store.info[k - 1]["linf"])
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
                "algorithmic_bytes_per_launch": algo[dom] / launches, "avg_launch_ms": dk["avg_launch_ms"]}

    comp_ms = sum(kern.get(k, {}).get("ms_per_step", 0.0) for k in
                  ("k_encode_" + tname, "k_scan", "k_pack_" + tname))
    dec_ms = kern.get("k_decode_" + tname, {}).get("ms_per_step", 0.0)
    value = N * s * (1 + n) / (ms_step / 1e3) / 1e9

    cpu = None
    if args.cpu_planes > 0:
        log("oracle baseline on %d z-planes" % args.cpu_planes)
        cpu = cpu_baseline(x, taus, args.cpu_planes)

    rec = {
        "metric": "compress/retrieve GB/s (512^3 f32, 8 comps)",
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
                   "tau": "2^-3i" if args.workload.startswith("bulk") else "see DESIGN.md",
                   "decode": "literal" if args.literal else "fused", "step": "range + compress + retrieve k=1..n"},
        "compress_gbs": N * s / (comp_ms / 1e3) / 1e9 if comp_ms else None,
        "retrieve_all_k_gbs": N * s * n / (dec_ms / 1e3) / 1e9 if dec_ms else None,
        "rates_bits_per_value": [round(8.0 * m["bytes"] / N, 3) for m in info],
        "linf": [m["linf"] for m in info],
        "kernels": kern,
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(rec))


if __name__ == "__main__":
    main()
