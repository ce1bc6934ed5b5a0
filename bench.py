"""Throughput of one rBKI-TK decomposition step on one MI355X.

A step is one full pass of the hot path over the resident input tensor: for
every mode the sketch and Gram products, the block Krylov basis, the
projected eigenproblem and the factor; then the core by a chain of mode
products and the explicit reconstruction error (Alg. 2).

    python bench.py [--steps K] [--warmup W] [--workload NAME] [--precision P]

Prints one JSON line.  `value` is the executed (algorithmic) TFLOP/s of the
whole step; `roofline` reports the Gram/sketch kernel (the dominant launch)
against the MFMA peak of its arithmetic type, timed with HIP events on the
stream it runs on; `cpu_baseline` times the FP64 oracle on a bounded slab of
the same input.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_TFLOPS = {"bf16": 2500.0, "fp8": 5000.0, "f32": 157.3, "f64": 78.6}
HBM_GBPS = 8000.0


def mode_views(dims):
    out = []
    for n in range(len(dims)):
        A = 1
        for k in range(n):
            A *= dims[k]
        B = 1
        for k in range(n + 1, len(dims)):
            B *= dims[k]
        out.append((A, dims[n], B))
    return out


def step_flops(dims, ranks, p, q, variant="krylov"):
    """Executed flops of the Gram route: per mode the symmetric Gram matrix
    and the sketch in one pass over X, the float64 Krylov steps on the Gram
    matrix (products, two projections, CholeskyQR), Z and the factor; then the
    core chain and the reconstruction of the residual.  The power variant has
    no projections, and its basis is one block wide."""
    T = 1
    for d in dims:
        T *= d
    total = 0.0
    gram = []
    for (A, I, B), R in zip(mode_views(dims), ranks):
        J = A * B
        S = min(R + p, I, J)
        Sp = S if variant == "power" else S * (q + 1)
        g = I * (I + 1) * J + 2.0 * I * J * S           # symmetric Gram + sketch
        gram.append(g)
        kry = 0.0
        for j in range(1, q + 1):
            m = S * j
            proj = 0.0 if variant == "power" else 2 * (2.0 * S * m * I * 2)
            kry += 2.0 * I * I * S + proj + 4.0 * S * S * I
        kry += 2.0 * I * I * S + 2.0 * Sp * Sp * I + 2.0 * R * Sp * I
        total += g + kry
    # core chain: first product on the mode with the largest I/R, then ascending
    first = max(range(len(dims)), key=lambda n: (dims[n] / ranks[n], -n))
    cur = list(dims)
    order = [first] + [n for n in range(len(dims)) if n != first]
    for n in order:
        size = 1
        for d in cur:
            size *= d
        total += 2.0 * ranks[n] * size
        cur[n] = ranks[n]
    # reconstruction chain (modes 1..N-1) and the residual with U^(1)
    for n in range(1, len(dims)):
        size = 1
        for k, d in enumerate(cur):
            size *= d
        total += 2.0 * dims[n] * size
        cur[n] = dims[n]
    total += 2.0 * ranks[0] * T
    return total, gram


def source_hash():
    h = hashlib.sha256()
    for f in ("gram.hip", "gram_pipe.hip", "rbki_mma.h"):
        with open(os.path.join(ROOT, "paper_2211_14828_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def load_traffic(workload, precision):
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        rec = json.load(open(path)).get(f"gram/{workload}/{precision}")
    except (OSError, ValueError):
        return None
    if not rec or rec.get("source_hash") != source_hash():
        return None
    return rec.get("bytes_per_launch")


# torch.mul(src, 1.0, out=dst) on float32: reads and writes n*4 bytes
COPY_KERNEL = "AUnaryFunctor<float, float, float, at::native::binary_internal::MulFunctor<float> >"


def _pmc_rows(path, counter):
    import csv
    out = {}
    with open(path) as fh:
        for r in csv.DictReader(fh):
            if r.get("Counter_Name") != counter:
                continue
            d = int(r["Dispatch_Id"])
            out[d] = (r["Kernel_Name"], out.get(d, (None, 0.0))[1] + float(r["Counter_Value"]))
    return out


def traffic_from(fetch_csv, write_csv, workload, precision, copy_mib, command):
    """HBM bytes per Gram launch from two rocprofv3 --pmc runs (FETCH_SIZE, then
    WRITE_SIZE, KiB per dispatch), each scaled by what the same counter reads
    for the calibration copy of known size in the same program."""
    kernel = "gram_pipe_kernel" if precision in ("mixed_bf16", "mixed_fp8") else "gram_sketch_kernel"
    known = copy_mib * 1024 * 1024
    res = {}
    for name, path, counter in (("fetch", fetch_csv, "FETCH_SIZE"), ("write", write_csv, "WRITE_SIZE")):
        rows = _pmc_rows(path, counter)
        copies = [v * 1024 for k, v in rows.values() if COPY_KERNEL in k]
        grams = [v * 1024 for k, v in rows.values() if kernel in k]
        if not copies or not grams:
            raise SystemExit(f"{path}: no {COPY_KERNEL} or {kernel} dispatches with {counter}")
        scale = known / (sum(copies) / len(copies))
        res[name] = {"raw_bytes_per_launch": sum(grams) / len(grams), "copy_scale": scale,
                     "bytes_per_launch": sum(grams) / len(grams) * scale, "launches": len(grams)}
    path = os.path.join(ROOT, "profiles", "traffic.json")
    db = json.load(open(path)) if os.path.exists(path) else {}
    db[f"gram/{workload}/{precision}"] = {
        "kernel": kernel, "bytes_per_launch": res["fetch"]["bytes_per_launch"] + res["write"]["bytes_per_launch"],
        "fetch": res["fetch"], "write": res["write"], "copy_bytes": known,
        "source_hash": source_hash(), "command": command}
    with open(path, "w") as fh:
        json.dump(db, fh, indent=1, sort_keys=True)
        fh.write("\n")
    print(json.dumps(db[f"gram/{workload}/{precision}"]))


def cpu_baseline(X, w, target_s=20.0):
    """The FP64 oracle, as it stands, on a bounded slab X[..., :slab] of the
    same tensor: the whole decomposition (every mode's sketch, q Krylov steps
    in the streamed form, Z and its eigenvectors, the core and the explicit
    error).  A probe on a thin slab sizes the timed slab to about target_s
    seconds.  The value is in the unit of the GPU figure: the flops that the
    GPU route executes for the slab's shape (step_flops) per second of the
    oracle, so value_gpu / value_cpu is the speed ratio for equal work."""
    import numpy as np
    from oracle.rbki import rbki_tucker
    from oracle.trsvd import rbki_htr
    p, q, seed = w["p"], w["q"], w["seeds"][1]
    last = X.shape[-1]

    def run(slab):
        Xs = np.ascontiguousarray(X[..., :slab].double().cpu().numpy())
        ranks = tuple(min(R, d) for R, d in zip(w["ranks"], Xs.shape))
        t0 = time.perf_counter()
        if w["kind"] == "ring":
            rbki_htr(Xs, ranks, p, q, seed, w["tr_ranks"], explicit_error="core")
        else:
            rbki_tucker(Xs, ranks, p, q, seed)
        return time.perf_counter() - t0, Xs.shape, ranks

    # the probe slab: at most about 3e7 entries (a 64^5 tensor gives one
    # slice of its last mode)
    rest = X.numel() // last
    probe = max(1, min(last, 60, int(3e7 // rest)))
    dt, _, _ = run(probe)
    slab = int(min(last, max(probe, probe * target_s / max(dt, 1e-3))))
    dt, shape, ranks = run(slab)
    flops, _ = step_flops(shape, ranks, p, q)
    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 1) for i in threadpool_info() if i.get("user_api") == "blas"] or [1])
    except Exception:
        threads = os.cpu_count()
    return {"value": flops / dt / 1e12, "unit": "TFLOP/s", "cores": int(threads), "kind": "oracle",
            "sample": f"FP64 oracle (numpy/LAPACK, {threads} BLAS threads, host cpu_count={os.cpu_count()}): "
                      f"whole {'rBKI-TK-TR (Alg. 3)' if w['kind'] == 'ring' else 'rBKI-TK'} decomposition (Alg. 2: every mode's sketch, {q} Krylov steps in the "
                      f"streamed form, Z, eigenvectors, core, explicit error) of the slab X[..., :{slab}] "
                      f"({'x'.join(str(d) for d in shape)}, ranks {ranks}) of the same input, {dt:.2f} s; value = "
                      f"GPU-route flops of that shape ({flops:.3e}) / time"}


METRIC = "rBKI-TK TFLOP/s + rel err vs FP64 oracle; served solves/s, p50/p99 latency"


def load_golden(workload):
    path = os.path.join(ROOT, "tests", "golden", "full_size.json")
    try:
        with open(path) as f:
            return json.load(f).get(workload)
    except (OSError, ValueError):
        return None


def _pct(v, q):
    import numpy as np
    return float(np.percentile(np.asarray(v, dtype=np.float64), q)) if len(v) else None


def serving_leg(torch, rb, synth, count, slots, budget_gib, load, precision):
    """The served mix: `count` third-order requests (dims U{32..256}, ranks
    U{4..32} capped at dim/2, Gaussian core, orthonormal factors, SNR U[5,30]
    dB, bf16 storage, p = 5, q U{1,2,3}), all resident in HBM before timing.

    1. one-at-a-time: each request solved alone by the plain form on its
       float32 copy, in arrival order, one after the other; and the same on
       the bf16 tensors in the served precision (the same arithmetic as the
       server, so the two capacities separate batching from arithmetic);
    2. saturated: every request submitted to the request server at once
       (capacity in solves/s);
    3. the same Poisson arrivals (the recipe's exponential gaps) at one
       offered rate, `load` x the one-at-a-time float32 capacity, for the
       one-at-a-time float32 solver (a FIFO queue) and for the server;
    4. the server alone at `load` x its saturated rate.
    Latency is from the scheduled arrival to completion.  The served results'
    relative errors are compared with the plain ones."""
    import threading
    reqs = synth.served_requests(count=count)
    Xb, X32 = [], []
    for i, w in enumerate(reqs):
        x = synth.make_device(w)
        Xb.append(x)
        X32.append(x.float())
        if (i + 1) % 500 == 0:
            torch.cuda.synchronize()
            print(f"[serve] generated {i + 1}/{count} requests", file=sys.stderr, flush=True)
    torch.cuda.synchronize()

    def args_of(w):
        return dict(p=w["p"], q=w["q"], seed=w["seeds"][1])

    def one_at_a_time(xs, prec):
        for w, x in list(zip(reqs, xs))[:8]:
            rb.tucker(x, w["ranks"], precision=prec, **args_of(w))
        torch.cuda.synchronize()
        lat, err = [], []
        t0 = time.perf_counter()
        for w, x in zip(reqs, xs):
            t = time.perf_counter()
            _, _, e = rb.tucker(x, w["ranks"], precision=prec, **args_of(w))
            lat.append((time.perf_counter() - t) * 1e3)
            err.append(e)
        return count / (time.perf_counter() - t0), lat, err

    def fifo(xs, prec, rate):
        # one solver, requests taken in arrival order: a request waits for the
        # ones before it
        arrivals = [w["arrival"] / rate for w in reqs]
        lat = []
        t0 = time.perf_counter()
        for w, x, a in zip(reqs, xs, arrivals):
            d = t0 + a - time.perf_counter()
            if d > 0:
                time.sleep(d)
            rb.tucker(x, w["ranks"], precision=prec, **args_of(w))
            lat.append((time.perf_counter() - t0 - a) * 1e3)
        return lat

    def served_poisson(sv, rate):
        arrivals = [w["arrival"] / rate for w in reqs]
        lat = [None] * count
        lag = [0.0] * count
        done_at = [0.0] * count
        tick = [None] * count
        ready = threading.Semaphore(0)

        def collect():
            for i in range(count):
                ready.acquire()
                r = sv.wait(tick[i])
                done_at[i] = time.perf_counter()
                lat[i] = lag[i] + r[3]

        th = threading.Thread(target=collect)
        th.start()
        t0 = time.perf_counter()
        for i, (w, x) in enumerate(zip(reqs, Xb)):
            d = t0 + arrivals[i] - time.perf_counter()
            if d > 0:
                time.sleep(d)
            lag[i] = (time.perf_counter() - t0 - arrivals[i]) * 1e3
            tick[i] = sv.submit(x, w["ranks"], precision=precision, **args_of(w))
            ready.release()
        th.join()
        return lat, count / (max(done_at) - t0)

    plain_rate, lat_plain, err_plain = one_at_a_time(X32, "plain")
    print(f"[serve] one-at-a-time plain f32: {plain_rate:.1f} solves/s", file=sys.stderr, flush=True)
    same_rate = load * plain_rate
    lat_fifo = fifo(X32, "plain", same_rate)
    print(f"[serve] one-at-a-time plain f32 at {same_rate:.1f}/s offered: p50 {_pct(lat_fifo, 50):.3f} ms "
          f"p99 {_pct(lat_fifo, 99):.3f} ms", file=sys.stderr, flush=True)
    del X32
    torch.cuda.empty_cache()
    prec_rate, _, _ = one_at_a_time(Xb, precision)
    print(f"[serve] one-at-a-time {precision} on bf16: {prec_rate:.1f} solves/s", file=sys.stderr, flush=True)

    budget = int(budget_gib * (1 << 30))
    with rb.Server(budget, slots=slots) as sv:
        for w, x in list(zip(reqs, Xb))[:2 * slots]:
            sv.wait(sv.submit(x, w["ranks"], precision=precision, **args_of(w)))
        t0 = time.perf_counter()
        tickets = [sv.submit(x, w["ranks"], precision=precision, **args_of(w)) for w, x in zip(reqs, Xb)]
        res = [sv.wait(t) for t in tickets]
        sat_rate = count / (time.perf_counter() - t0)
        err_served = [r[2] for r in res]
        print(f"[serve] saturated: {sat_rate:.1f} solves/s", file=sys.stderr, flush=True)
        del res
        lat_same, _ = served_poisson(sv, same_rate)
        print(f"[serve] served at {same_rate:.1f}/s offered: p50 {_pct(lat_same, 50):.3f} ms "
              f"p99 {_pct(lat_same, 99):.3f} ms", file=sys.stderr, flush=True)
        rate = load * sat_rate
        lat, achieved = served_poisson(sv, rate)
    ex = [(a - b) / b for a, b in zip(err_served, err_plain) if b > 0]
    out = {"requests": count, "mix": "3rd-order, dims U{32..256}, ranks U{4..32} capped at dim/2, bf16, p=5, "
                                      "q U{1,2,3}, SNR U[5,30] dB",
           "precision": precision, "slots": slots, "hbm_budget_gib": budget_gib,
           "solves_per_s": round(sat_rate, 2),
           "plain_one_at_a_time_solves_per_s": round(plain_rate, 2),
           "speedup_vs_plain": round(sat_rate / plain_rate, 3),
           "same_precision_one_at_a_time_solves_per_s": round(prec_rate, 2),
           "speedup_vs_same_precision": round(sat_rate / prec_rate, 3),
           "same_offered_rate": {"offered_rate": round(same_rate, 2),
                                 "served_p50_ms": round(_pct(lat_same, 50), 4),
                                 "served_p99_ms": round(_pct(lat_same, 99), 4),
                                 "plain_fifo_p50_ms": round(_pct(lat_fifo, 50), 4),
                                 "plain_fifo_p99_ms": round(_pct(lat_fifo, 99), 4)},
           "offered_rate": round(rate, 2), "achieved_rate": round(achieved, 2),
           "p50_ms": round(_pct(lat, 50), 4), "p99_ms": round(_pct(lat, 99), 4),
           "plain_p50_ms": round(_pct(lat_plain, 50), 4), "plain_p99_ms": round(_pct(lat_plain, 99), 4),
           "excess_vs_plain_median": _pct(ex, 50), "excess_vs_plain_max": max(ex) if ex else None}
    print(f"[serve] {out}", file=sys.stderr, flush=True)
    del Xb
    torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="tucker1000_f32",
                    help="tucker1000_f32, tucker400_f32, tucker64_f64 (Alg. 2) or ring64x5_f32 (Alg. 3)")
    ap.add_argument("--data", default="host", choices=["host", "device"],
                    help="host: the bytes of synth.make_host, whose float64 oracle error is stored in "
                         "tests/golden/full_size.json; device: a seeded torch generator on the GPU (faster, "
                         "no oracle reference)")
    ap.add_argument("--precision", default="mixed_fp8")
    ap.add_argument("--variant", default="krylov", choices=["krylov", "power"],
                    help="subspace of each factor: the block Krylov space (Alg. 1) or power iteration (Sec. 3.1)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-compare", action="store_true",
                    help="skip the FP64 and plain-form runs that follow the timed region")
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="run a plain copy of MIB MiB first (the reference for PMC byte counters)")
    ap.add_argument("--traffic-from", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="write profiles/traffic.json from two rocprofv3 --pmc counter CSVs and exit")
    ap.add_argument("--traffic-command", default="")
    ap.add_argument("--serve-requests", type=int, default=2000,
                    help="requests of the served mix (0: skip the serving leg)")
    ap.add_argument("--serve-slots", type=int, default=16)
    ap.add_argument("--serve-hw-queues", type=int, default=0,
                    help="hardware queues of the process (default: one per slot, at most 32)")
    ap.add_argument("--serve-budget-gib", type=float, default=16.0)
    ap.add_argument("--serve-load", type=float, default=0.7,
                    help="Poisson arrival rate as a fraction of a capacity: of the one-at-a-time float32 rate for "
                         "the same-rate comparison, and of the saturated rate for the served run")
    ap.add_argument("--serve-precision", default="plain")
    ap.add_argument("--serve-only", action="store_true")
    args = ap.parse_args()
    if args.traffic_from:
        traffic_from(args.traffic_from[0], args.traffic_from[1], args.workload, args.precision,
                     args.calibrate_copy, args.traffic_command)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path (the per-GPU slab of a sharded "
              "run is the same kernel at a smaller shape); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    # one hardware queue per server slot: with fewer, the slots' streams share
    # queues and their solves run one after the other.  The HIP runtime reads
    # this when it starts, so it is set before torch is imported.
    if args.serve_requests > 0:
        os.environ["GPU_MAX_HW_QUEUES"] = str(max(4, min(args.serve_hw_queues or args.serve_slots, 32)))
    import torch
    import paper_2211_14828_amd as rb
    import synth

    rb.load_library(build_if_missing=True)
    if args.serve_only:
        print(json.dumps({"serving": serving_leg(torch, rb, synth, args.serve_requests, args.serve_slots,
                                                 args.serve_budget_gib, args.serve_load, args.serve_precision)}),
              flush=True)
        return
    w = synth.WORKLOADS[args.workload]
    dims, ranks, p, q = tuple(w["dims"]), tuple(w["ranks"]), w["p"], w["q"]
    htr = w["kind"] == "ring"
    gold = load_golden(args.workload)
    oracle_err = None
    if args.data == "host":
        # the bytes the stored oracle result was computed on
        print(f"[bench] generating {args.workload} {dims} on the host", file=sys.stderr, flush=True)
        Xh, _ = synth.make_host(w)
        if gold is not None and synth.same_fingerprint(synth.fingerprint(Xh), gold["fingerprint"]):
            oracle_err = gold["htr"]["rel_err"] if htr else gold["oracle"]["rel_err"]
        else:
            print("[bench] no stored oracle result for these bytes", file=sys.stderr, flush=True)
        X = torch.from_numpy(Xh).to("cuda")
        del Xh
    else:
        print(f"[bench] generating {args.workload} {dims} on the device", file=sys.stderr, flush=True)
        X = synth.make_device(w)
    torch.cuda.synchronize()
    seed = w["seeds"][1]

    if args.calibrate_copy:
        n = args.calibrate_copy * 1024 * 1024 // 4
        src = torch.ones(n, device="cuda", dtype=torch.float32)
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.mul(src, 1.0, out=dst)
        torch.cuda.synchronize()
        del src, dst

    def step(Xin=X, precision=args.precision):
        if htr:
            # Alg. 3: the Tucker step with the compress sizes, TR-SVD of the core
            cores, e = rb.htr(Xin, ranks, w["tr_ranks"], p=p, q=q, seed=seed, precision=precision,
                              out_dtype=torch.float32)
            return cores, None, e
        return rb.tucker(Xin, ranks, p=p, q=q, seed=seed, precision=precision, out_dtype=torch.float32,
                         variant=args.variant)

    for i in range(args.warmup):
        _, _, e = step()
        print(f"[bench] warmup {i} rel_err {e:.8f}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    rb.profile_reset()
    rb.profile_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        _, _, e = step()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    rb.profile_enable(False)
    ms = dt / args.steps * 1e3
    flops, gram_flops = step_flops(dims, ranks, p, q, args.variant)
    tflops = flops / (dt / args.steps) / 1e12
    nlaunch, gram_ms = rb.profile_read("gram")
    avg_gram_ms = gram_ms / max(nlaunch, 1)
    alg_gram = sum(gram_flops) / len(gram_flops)       # per launch (one launch per mode)
    achieved = alg_gram / (avg_gram_ms * 1e-3) / 1e12
    in_dt = {"float32": "f32", "float64": "f64", "bfloat16": "bf16"}[w["dtype"]]
    gram_dtype = {"plain": in_dt, "mixed_bf16": "bf16", "mixed_fp8": "fp8"}[args.precision]
    kernel = "gram_pipe_kernel" if gram_dtype in ("bf16", "fp8") else "gram_sketch_kernel"
    peak = PEAK_TFLOPS[gram_dtype]
    stages = {}
    for k in ("omega", "gram", "chain", "eig", "ttm", "error", "convert"):
        n, t = rb.profile_read(k)
        if n:
            stages[k] = round(t / args.steps, 4)
    print(f"[bench] {args.steps} steps, {ms:.3f} ms/step, rel_err {e:.8f}, stage ms/step {stages}",
          file=sys.stderr, flush=True)

    compare = {}
    if oracle_err is not None:
        # the float64 oracle's error on the same bytes, stored by
        # tests/golden/make_full_size.py
        compare["rel_err_oracle"] = oracle_err
        compare["excess_vs_oracle"] = (e - oracle_err) / oracle_err
    if not args.no_compare:
        # outside the timed region: the FP64 form on the same values (parity-pinned
        # to the oracle) gives the reference error; the plain form gives the wall
        # time the mixed form is compared with
        X64 = X.double()
        _, _, e64 = step(X64, "plain")
        del X64
        torch.cuda.empty_cache()
        compare["rel_err_gpu_f64"] = e64
        compare["excess_vs_gpu_f64"] = (e - e64) / e64 if e64 > 0 else None
        if args.precision != "plain":
            step(X, "plain")
            torch.cuda.synchronize()
            n_plain = max(1, min(3, args.steps))
            t1 = time.perf_counter()
            for _ in range(n_plain):
                step(X, "plain")
            torch.cuda.synchronize()
            compare["plain_ms_per_step"] = round((time.perf_counter() - t1) / n_plain * 1e3, 4)
        print(f"[bench] compare {compare}", file=sys.stderr, flush=True)

    serving = None
    if args.serve_requests > 0:
        serving = serving_leg(torch, rb, synth, args.serve_requests, args.serve_slots, args.serve_budget_gib,
                              args.serve_load, args.serve_precision)

    cpu = None
    if not args.no_cpu_baseline:
        print("[bench] timing the CPU oracle on a slab", file=sys.stderr, flush=True)
        cpu = cpu_baseline(X, w, args.cpu_seconds)
    rec = {
        "metric": METRIC,
        "value": round(tflops, 4),
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": gram_dtype,
        "data": "synthetic",
        "config": {"workload": args.workload, "dims": list(dims), "ranks": list(ranks), "p": p, "q": q,
                   "precision": args.precision, "variant": args.variant, "input_dtype": w["dtype"], "rel_err": e,
                   **compare, "stage_ms_per_step": stages,
                   "flops_per_step": flops},
        "roofline": {"bound": "mfma", "achieved": round(achieved, 3), "peak": peak, "unit": "TFLOP/s",
                     "frac": round(achieved / peak, 5), "traffic": load_traffic(args.workload, args.precision),
                     "kernel": kernel, "avg_launch_ms": round(avg_gram_ms, 5),
                     "launches": nlaunch, "alg_flops_per_launch": alg_gram},
        "cpu_baseline": cpu,
        "serving": serving,
    }
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
