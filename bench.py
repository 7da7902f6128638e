#!/usr/bin/env python3
"""Benchmark of the Lazy SPCA hot path on one MI355X.

One step = one Lazy SPCA fit of X (Algorithm 2: Omega, Y = X Omega, G, F,
the small FP64 stage) followed by the projection Z = X V of the same X.
Workload (default): X 1,000,000 x 4,096 FP32 low-rank-plus-noise (rank-256
signal, sigma_i = i^-1/2, noise N(0, 0.05^2)), Gaussian Omega, k = 256.

Printed: one JSON line with the X-stream throughput of the step (bytes of X
the step streams, 2 |X|: once for the fit, once for the projection, over the
step time), the per-phase device times, the dominant kernel's roofline and
the FP64 CPU oracle timed on a bounded row sample.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAKS = {  # MI355X published dense peaks
    "hbm_GBs": 8000.0,
    "fp32_mfma_TFs": 157.3,
    "fp64_mfma_TFs": 78.6,
    "bf16_mfma_TFs": 2500.0,
    "fp16_mfma_TFs": 2500.0,
}


# HBM bytes per launch of the sketch kernel, from rocprofv3 FETCH_SIZE and
# WRITE_SIZE (one counter per run) scaled by the counters' reading for a
# reference op of known traffic (the profiles/*.md summaries give the
# commands and figures). A figure holds only for the kernel source it was measured on:
# when the sources' hash differs, traffic is reported as null.
MEASURED_TRAFFIC = {
    ("f32", 1_000_000, 4096, 256, "gaussian"): {
        "sources": ["paper_1709_07175_amd/csrc/gemm.hip", "paper_1709_07175_amd/csrc/common.h"],
        "sha256": "ea4b9a73560b99c7b7d05b8fbe0a5b2e7a19206a842869ac504688c63414e46f",
        "bytes": 1.8462e+10,
    },
    ("bf16", 1_000_000, 4096, 256, "sparse"): {
        "sources": ["paper_1709_07175_amd/csrc/sparse.hip", "paper_1709_07175_amd/csrc/philox.h",
                    "paper_1709_07175_amd/csrc/common.h"],
        "sha256": "ab8e6665aa1ef24a584ced86975937ec90dd83eb330ffea79a741092a49755c4",
        "bytes": 9.2164e+09,
    },
    ("f16", 4_600_000, 2048, 128, "gaussian"): {
        "sources": ["paper_1709_07175_amd/csrc/gemm16.hip", "paper_1709_07175_amd/csrc/common.h"],
        "sha256": "07454a9563b9283d1daa4f734fe3102f5bb7c7f66bb19a1d0f4f274007ccbc78",
        "bytes": 2.1740e+10,
    },
    ("csr", 131_072, 98_450, 500, "sparse"): {   # k_csc_block, per row-block launch
        "sources": ["paper_1709_07175_amd/csrc/csr.hip", "paper_1709_07175_amd/csrc/common.h"],
        "sha256": "f6d727e531aef2c0c468ea327e50865dfeffc5dc130c8022b748346f3e3ab814",
        "bytes": 6.3321e+09,
    },
}


def measured_traffic_rec(rec):
    import hashlib
    h = hashlib.sha256()
    for f in rec["sources"]:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest() == rec["sha256"]


def measured_traffic(cfg, m):
    rec = MEASURED_TRAFFIC.get((cfg["dtype"], m, cfg["n"], cfg["k"], cfg["kind"]))
    if rec is None:
        return None
    return rec["bytes"] if measured_traffic_rec(rec) else None


def roofline(cfg, m, n, k, xbytes, esz, sketch_ms):
    """The sketch Y = X Omega (one launch per fit). FP32/FP64 with a Gaussian
    Omega: 2 m n k flop on the matrix cores, the bound. 16-bit data (the
    MFMA peak is 16x FP32's) and the very sparse Omega (gather-adds, no MFMA):
    the X stream is the bound, algorithmic bytes = X + Omega + Y once."""
    alg_bytes = xbytes + (esz * n * k if cfg["kind"] == "gaussian" else 0) + 4 * m * k
    if cfg["dtype"] in ("f32", "f64") and cfg["kind"] == "gaussian":
        flops = 2.0 * m * n * k
        peak = PEAKS["fp32_mfma_TFs"] if cfg["dtype"] == "f32" else PEAKS["fp64_mfma_TFs"]
        achieved = flops / (sketch_ms * 1e-3) / 1e12
        name = ("k_nt32s (sketch Y = X Omega; persistent, operands copied straight into LDS)"
                if cfg["dtype"] == "f32" else "k_nt (sketch Y = X Omega)")
        return {"kernel": name, "bound": "mfma", "achieved": round(achieved, 3),
                "peak": peak, "unit": "TFLOP/s", "frac": round(achieved / peak, 4),
                "traffic": measured_traffic(cfg, m),
                "algorithmic": f"2 m n k = {flops:.4g} flop per launch", "algorithmic_bytes": alg_bytes}
    achieved = alg_bytes / (sketch_ms * 1e-3) / 1e9
    name = ("k_sparse_sketch (gather-adds)" if cfg["kind"] == "sparse"
            else "k_nt16v2 (sketch Y = X Omega; persistent, operands copied straight into LDS)")
    return {"kernel": name, "bound": "hbm", "achieved": round(achieved, 3), "peak": PEAKS["hbm_GBs"],
            "unit": "GB/s", "frac": round(achieved / PEAKS["hbm_GBs"], 4),
            "traffic": measured_traffic(cfg, m),
            "algorithmic": f"X + Omega + Y = {alg_bytes:.4g} bytes per launch", "algorithmic_bytes": alg_bytes}


def pass_rooflines(cfg, m, n, k, xbytes, esz, phases):
    """Every kernel phase of the step against its bound (device times from the
    library's events, averaged over the timed steps): the sketch, F = Y^T X,
    the small FP64 stage (latency-bound: time only) and the projection."""
    dt = cfg["dtype"]

    def avg(key, which=0):
        return sum(p[which][key] for p in phases) / len(phases)

    h16 = dt in ("bf16", "f16")
    mfma_peak = {"f64": PEAKS["fp64_mfma_TFs"], "f32": PEAKS["fp32_mfma_TFs"]}.get(dt, PEAKS["bf16_mfma_TFs"])
    res = {"sketch": roofline(cfg, m, n, k, xbytes, esz, avg("sketch_ms"))}
    f_ms = avg("factor_ms")
    # F: one product per element for FP32/FP64, two for 16-bit data (the
    # split sketch, Y_hi and Y_lo); the fits here ask for no Sigma^s, so the
    # pass forms no G
    flops = 2.0 * m * n * k * (2 if h16 else 1)
    ybytes = m * k * (8 if dt == "f64" else 4)   # Y (FP64, FP32, or the two 16-bit parts)
    f_bytes = xbytes + ybytes
    tf = flops / (f_ms * 1e-3) / 1e12
    if dt == "f32":
        fname = "k_tn32s (F = Y^T X, operands copied straight into LDS)"
    elif not h16:
        fname = "k_tn (F = Y^T X)"
    elif dt == "f16" and cfg["kind"] == "gaussian":
        fname = "k_tn16 (F = Y_hi^T X + Y_lo^T X, Y split from the FP32 sketch as loaded)"
    else:
        fname = "k_tn16v2 (F = Y_hi^T X + Y_lo^T X, operands copied straight into LDS)"
    res["F"] = {"kernel": fname,
                "ms": round(f_ms, 4), "flop": flops, "TFLOPs": round(tf, 2),
                "mfma_peak_TFs": mfma_peak, "mfma_frac": round(tf / mfma_peak, 4),
                "hbm_bytes_algorithmic": f_bytes,
                "hbm_frac": round(f_bytes / (f_ms * 1e-3) / 1e9 / PEAKS["hbm_GBs"], 4)}
    res["small_fp64"] = {"ms": round(avg("small_ms"), 4), "bound": "latency"}
    t_ms = avg("transform_ms", 1)
    tflops = 2.0 * m * n * k * (2 if h16 else 1)
    tbytes = xbytes + m * k * (8 if dt == "f64" else 4)
    if h16:
        pname = "k_nt16 (Z = X V_hi + X V_lo)"
    elif dt == "f32":
        pname = "k_nt32s (Z = X V; persistent, operands copied straight into LDS)"
    else:
        pname = "k_nt (Z = X V)"
    res["projection"] = {"kernel": pname,
                         "ms": round(t_ms, 4), "flop": tflops,
                         "mfma_frac": round(tflops / (t_ms * 1e-3) / 1e12 / mfma_peak, 4),
                         "hbm_frac": round(tbytes / (t_ms * 1e-3) / 1e9 / PEAKS["hbm_GBs"], 4)}
    # the bound of the whole fit by the method's own work: X read once, the
    # two products at the matrix-core peak (16-bit: with the refinement)
    t_hbm = xbytes / (PEAKS["hbm_GBs"] * 1e9)
    t_mfma = (2.0 * m * n * k + flops) / (mfma_peak * 1e12)
    if cfg["kind"] == "sparse":
        t_mfma = flops / (mfma_peak * 1e12)
    bound_ms = max(t_hbm, t_mfma) * 1e3
    res["fit_bound"] = {"ms": round(bound_ms, 4), "hbm_ms": round(t_hbm * 1e3, 4),
                        "mfma_ms": round(t_mfma * 1e3, 4),
                        "frac_fit": round(bound_ms / avg("total_ms"), 4),
                        "frac_pass": round(bound_ms / (avg("sketch_ms") + f_ms + avg("reduce_ms") +
                                                       avg("layout_ms")), 4)}
    return res


# The paper's own timings (context, not the target): the largest analysis of
# Experiment 1 (Sec. I and Sec. IV-A), on one CPU machine.
PAPER_CONTEXT = {
    "spca_hours": 43.7, "lazy_spca_hours": 9.9, "speedup": round(43.7 / 9.9, 2),
    "hardware": "one Amazon EC2 r3.8xlarge instance: 16 physical cores (32 hyperthreads), 244 GB RAM; "
                "Julia v0.3.8, sparse products and QR in Intel MKL",
    "workload": "sparse malware feature matrix, 4,608,517 samples x 98,450 features, mean density "
                "0.0244, FP32 values, very sparse Omega; the k of the largest run is not stated "
                "(k up to 20,000 in that experiment)",
    "source": "Sec. I and Sec. IV-A of arXiv 1709.07175",
}


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def cpu_baseline(cfg, X_dev, budget_s=20.0):
    """FP64 oracle (numpy, BLAS threads) on a bounded row sample of the same
    X: one fit plus one projection, scaled to X-stream GB/s."""
    import numpy as np
    from oracle import lspca_oracle as O
    from oracle import philox as P
    try:
        from threadpoolctl import threadpool_info
        cores = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:  # pragma: no cover
        cores = os.cpu_count()
    n, k = cfg["n"], cfg["k"]
    om = P.omega(n, k, cfg["kind"], cfg["omega_seed"], cfg.get("p", 64), dtype=cfg["dtype"])
    m = X_dev.shape[0]

    def one(rows):
        Xh = X_dev[:rows].double().cpu().numpy()
        t0 = time.perf_counter()
        fit = O.streaming_lazy_fit(Xh, om, k, S=max(1, rows // 65536))
        O.transform(Xh, fit["V"])
        return time.perf_counter() - t0

    # grow the row sample while the next size stays within the budget, then
    # repeat that size until at least 10 s of oracle work is timed
    rows = min(m, 4096)
    dt = one(rows)
    while rows < m and dt * 2.2 <= budget_s:
        rows = min(m, rows * 2)
        dt = one(rows)
    times = [dt]
    while sum(times) < 10.0 and len(times) < 2000:
        times.append(one(rows))
    total = sum(times)
    esz = X_dev.element_size()
    gbs = 2 * rows * n * esz * len(times) / total / 1e9
    return {"value": round(gbs, 4), "unit": "GB/s", "cores": int(cores), "kind": "oracle",
            "cpu_model": cpu_model(), "host_cpus": os.cpu_count(),
            "sample": f"first {rows} rows of the same X (of {m}): FP64 oracle fit (Algorithm 2, "
                      f"numpy/BLAS) plus Z = X V, timed {len(times)}x, {total:.2f} s in all"}


def serving(lib, V, Xsrc, levels, counts, modes, seed=7175 + 5, log_every=500):
    """Projection serving at Poisson arrivals (one level after another).

    Requests: r rows, log-uniform on [1, 65,536], of BF16 rows drawn from the
    fitted workload (a pool of the first rows of X, cast to BF16); V resident
    in the server. Mode "device": payloads pre-staged in HBM; mode "host":
    payloads and results in pinned host memory (H2D and D2H included).
    Latency is the server's own (submit to completion seen). Returns a dict
    per mode and level."""
    import threading
    import numpy as np
    import torch
    from synth import request_sizes

    sys.setswitchinterval(1e-4)
    n, k = V.shape
    max_rows = 65_536
    pool_rows = min(Xsrc.shape[0], max_rows + 16_384)
    pool = Xsrc[:pool_rows].to(torch.bfloat16).contiguous()
    out = {}
    for mode in modes:
        host = mode == "host"
        Q = 16 if host else 64
        if host:
            Xp = pool.cpu().pin_memory()
            Zring = torch.empty((Q, max_rows, k), dtype=torch.float32).pin_memory()
            arena = 6 * (max_rows * n * 2 + max_rows * k * 4)
        else:
            Xp = pool
            Zring = torch.empty((Q, max_rows, k), dtype=torch.float32, device=pool.device)
            arena = 0
        torch.cuda.synchronize()
        res = {}
        with lib.Server(V, lib.BF16, arena_bytes=arena, max_inflight=64) as srv:
            # warm-up: a few requests of each size class
            for r in (1, 300, 5000, max_rows):
                srv.wait(srv.submit_ptr(Xp.data_ptr(), r, Zring[0].data_ptr()))
            xrow = n * Xp.element_size()
            zslot = max_rows * k * 4
            for li, qps in enumerate(levels):
                N = counts[li]
                rng = np.random.default_rng(seed + 1000 * li + (7 if host else 0))
                sizes = request_sizes(N, seed + li)
                offs = rng.integers(0, pool_rows - sizes + 1)
                gaps = rng.exponential(1.0 / qps, size=N)
                lat = [None] * N
                done = [threading.Event() for _ in range(N)]
                tickets = [None] * N
                have = [threading.Event() for _ in range(N)]

                def waiter():
                    for i in range(N):
                        have[i].wait()
                        lat[i] = srv.wait(tickets[i])
                        done[i].set()

                th = threading.Thread(target=waiter)
                th.start()
                t0 = time.perf_counter()
                target = t0
                for i in range(N):
                    target += gaps[i]
                    if i >= Q:
                        done[i - Q].wait()        # its result slot is free again
                    while True:
                        dt = target - time.perf_counter()
                        if dt <= 0:
                            break
                        if dt > 3e-4:
                            time.sleep(dt - 2e-4)
                    tickets[i] = srv.submit_ptr(Xp.data_ptr() + int(offs[i]) * xrow, int(sizes[i]),
                                                Zring.data_ptr() + (i % Q) * zslot)
                    have[i].set()
                    if log_every and (i + 1) % log_every == 0:
                        log(f"serving {mode} {qps} QPS: {i + 1}/{N} submitted")
                th.join()
                wall = time.perf_counter() - t0
                a = np.array(lat)
                rows = int(sizes.sum())
                res[str(qps)] = {"requests": N, "p50_ms": round(float(np.percentile(a, 50)), 4),
                                 "p99_ms": round(float(np.percentile(a, 99)), 4),
                                 "mean_ms": round(float(a.mean()), 4), "max_ms": round(float(a.max()), 4),
                                 "offered_qps": qps, "achieved_qps": round(N / wall, 2),
                                 "rows_per_s": round(rows / wall, 1),
                                 "payload_GBs": round(rows * (xrow + 4 * k) / wall / 1e9, 3)}
                log(f"serving {mode} {qps} QPS: p50 {res[str(qps)]['p50_ms']} ms, "
                    f"p99 {res[str(qps)]['p99_ms']} ms")
            st = srv.stats()
        res["server"] = {key: st[key] for key in ("launches", "max_requests_per_launch",
                                                  "max_concurrent_launches", "arena_peak_bytes")}
        c = max(1, st["completed"])
        res["server"]["mean_us"] = {"queue": round(st["queue_ns"] / c / 1e3, 2),
                                    "enqueue": round(st["enqueue_ns"] / c / 1e3, 2),
                                    "device": round(st["device_ns"] / c / 1e3, 2)}
        out[mode] = res
        del Zring, Xp
        torch.cuda.synchronize()
    return out


# Gather bound of the sparse column sums: each XCD's L2 serves 16 channels x
# 128 B per clock (the CDNA3 L2 design), 8 XCDs at 2.4 GHz.
L2_GBs = 8 * 16 * 128 * 2.4


def calibrate(torch, dev, gib):
    """y = 2 x over `gib` GiB of FP32: a reference op of known HBM traffic
    (reads and writes gib GiB once) for the byte counters."""
    cnt = int(gib * 2 ** 30) // 4
    a = torch.ones(cnt, dtype=torch.float32, device=dev)
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    torch.mul(a, 2.0, out=b)
    torch.cuda.synchronize()
    del a, b


def csr_block_launches(rows, n, esz):
    """Row blocks of one stripe (the library's csc_shape): one k_csc_block
    launch each."""
    slice_cols = 128 if esz == 4 else 64                 # columns per XCD slice
    rb_l2 = (4 << 20) // (slice_cols * esz)
    nb = -(-rows // rb_l2)
    nb = max(1, min(nb, max(1, (1 << 26) // n)))
    rb = -(-rows // nb)
    return -(-rows // rb)


def csr_roofline(c, nnz, m, esz, launches, factor_ms):
    """The column sums F += Y^T X (k_csc_block, one launch per row block of a
    stripe). Per launch (the pass's totals over its launches): gathered bytes
    = entries x k x value size (one sketch-row segment per entry and column
    slice); algorithmic HBM bytes = the entries (row index + value) once, the
    sketch rows once, F read and written once."""
    n, k = c["n"], c["k"]
    gathered = nnz * k * esz / launches
    alg = (nnz * (4 + esz) + m * k * esz + 2 * k * n * 8) / launches
    t = factor_ms / launches * 1e-3
    achieved = gathered / t / 1e9
    rec = MEASURED_TRAFFIC.get(("csr", m, n, k, c["kind"]))
    traffic = None
    if rec is not None and measured_traffic_rec(rec):
        traffic = rec["bytes"]
    return {"kernel": "k_csc_block (F += Y^T X, one row block)", "bound": "l2",
            "achieved": round(achieved, 3), "peak": L2_GBs, "unit": "GB/s",
            "frac": round(achieved / L2_GBs, 4), "traffic": traffic,
            "algorithmic": f"gathered: entries x k x {esz} B = {gathered:.4g} bytes per launch "
                           f"({launches} launches per fit)",
            "algorithmic_bytes": gathered,
            "hbm_algorithmic_bytes": alg,
            "hbm_GBs": round(alg / t / 1e9, 3)}


def csr_cpu_baseline(c, rph, cih, vvh, budget_s=20.0):
    """FP64 oracle on a bounded row sample of the same CSR X: the dense
    matrix of those rows (oracle.csr_dense), one Lazy SPCA fit plus Z = X V,
    scaled to CSR-stream GB/s."""
    import numpy as np
    from oracle import lspca_oracle as O
    from oracle import philox as P
    try:
        from threadpoolctl import threadpool_info
        cores = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:  # pragma: no cover
        cores = os.cpu_count()
    n, k = c["n"], c["k"]
    om = P.omega(n, k, c["kind"], c["omega_seed"], c["p"], dtype=c["dtype"])

    def one(rows):
        t0 = time.perf_counter()
        Xd = O.csr_dense(rph[:rows + 1], cih, vvh, n)
        fit = O.lazy_fit(Xd, om, k)
        O.transform(Xd, fit["V"])
        return time.perf_counter() - t0

    rows = k
    dt = one(rows)
    cap = min(len(rph) - 1, 8192)                   # dense rows of the sample: <= 8192 x n FP64
    while rows < cap and dt * 2.2 <= budget_s:
        rows = min(cap, rows * 2)
        dt = one(rows)
    times = [dt]
    while sum(times) < 10.0 and len(times) < 200:
        times.append(one(rows))
    total = sum(times)
    nbytes = 2 * (8 * (rows + 1) + int(rph[rows]) * (4 + vvh.itemsize))
    return {"value": round(nbytes * len(times) / total / 1e9, 4), "unit": "GB/s", "cores": int(cores),
            "kind": "oracle", "cpu_model": cpu_model(), "host_cpus": os.cpu_count(),
            "sample": f"first {rows} rows of the same CSR X: FP64 oracle fit (dense rows, numpy/BLAS) "
                      f"plus Z = X V, timed {len(times)}x, {total:.2f} s in all"}


def csr_main(args, lib, torch):
    """One step = lspca_fit_csr + lspca_transform_csr over the whole CSR X
    (resident on the device). Value: bytes of the CSR arrays the step streams
    (twice: fit and projection) over the step time."""
    from synth import CSR_CONFIG, csr_torch
    c = dict(CSR_CONFIG)
    if args.m:
        c["m"] = args.m
    if args.k:
        c["k"] = args.k
    m, n, k = c["m"], c["n"], c["k"]
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    log(f"generating CSR X {m}x{n} at density {c['density']} (seed {c['data_seed']})")
    t0 = time.time()
    rp, ci, vv = csr_torch(m, n, c["density"], c["data_seed"], c["alpha"], c["binary"], c["dtype"],
                           device=dev)
    torch.cuda.synchronize()
    X = lib.CSR(rp, ci, vv, n)
    log(f"generated in {time.time() - t0:.1f}s: nnz {X.nnz}")
    xbytes = rp.numel() * 8 + X.nnz * (4 + vv.element_size())
    stream = torch.cuda.current_stream()
    if args.calib_gib > 0:
        calibrate(torch, dev, args.calib_gib)

    def step(timing):
        V, s = lib.fit_csr(X, k, c["kind"], c["omega_seed"], timing=timing, sparse_p=c["p"])
        tf = lib.last_timings() if timing else None
        Z = lib.transform_csr(X, V, timing=timing)
        tt = lib.last_timings() if timing else None
        return V, Z, tf, tt

    for i in range(args.warmup):
        step(False)
        torch.cuda.synchronize()
        log(f"warmup {i + 1}/{args.warmup} done")
    phases = []
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    for i in range(args.steps):
        _, _, tf, tt = step(True)
        phases.append((tf, tt))
    ev1.record(stream)
    torch.cuda.synchronize()
    ms_step = ev0.elapsed_time(ev1) / args.steps
    log(f"timed {args.steps} steps: {ms_step:.3f} ms/step")

    def avg(key, which=0):
        return sum(p[which][key] for p in phases) / len(phases)

    # stripes of the pass (the library's plan: entries per stripe <= 2^28 on
    # 64-row boundaries, rows <= the 4 GiB sketch budget)
    rph = rp.cpu().numpy()
    esz = vv.element_size()
    starts, r0 = [0], 0
    rows_cap = min((4 << 30) // (k * esz), 1 << 24)
    while r0 < m:
        r1 = r0 + 64
        while r1 < m and r1 + 64 - r0 <= rows_cap and rph[min(r1 + 64, m)] - rph[r0] <= (1 << 28):
            r1 += 64
        r0 = min(r1, m)
        starts.append(r0)
    nstripes = len(starts) - 1
    launches = sum(csr_block_launches(starts[t + 1] - starts[t], n, esz) for t in range(nstripes))
    fit_ms, tr_ms = avg("total_ms", 0), avg("transform_ms", 1)
    value = 2 * xbytes / (ms_step * 1e-3) / 1e9
    out = {
        "metric": "X-stream GB/s (% HBM/MFMA roofline) per Lazy SPCA fit vs SPCA; projection p99 ms",
        "value": round(value, 3), "unit": "GB/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_step, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": c["dtype"], "data": "synthetic",
        "config": {"workload": f"lazy-spca fit+projection, sparse X (CSR) {m}x{n} density {c['density']} "
                               f"{c['dtype']} values, {c['kind']} Omega, k={k}",
                   "m": m, "n": n, "k": k, "nnz": X.nnz, "x_bytes": xbytes, "stripes": nstripes,
                   "parallelism": "single-gpu"},
        "phases_ms": {"fit_total": round(fit_ms, 4), "omega": round(avg("omega_ms"), 4),
                      "sketch": round(avg("sketch_ms"), 4), "csc_build": round(avg("layout_ms"), 4),
                      "factor_F": round(avg("factor_ms"), 4), "reduce": round(avg("reduce_ms"), 4),
                      "small_fp64": round(avg("small_ms"), 4), "transform": round(tr_ms, 4)},
        "roofline": csr_roofline(c, X.nnz, m, esz, launches, avg("factor_ms")),
    }
    if not args.no_spca and k <= 256:
        # Algorithm 1 on the same CSR X (the GPU tall-skinny QR holds k <= 256)
        lib.spca_fit_csr(X, k, c["kind"], c["omega_seed"], sparse_p=c["p"])
        torch.cuda.synchronize()
        sp = []
        for _ in range(2):
            lib.spca_fit_csr(X, k, c["kind"], c["omega_seed"], timing=True, sparse_p=c["p"])
            sp.append(lib.last_timings())
        sp_ms = sum(t["total_ms"] for t in sp) / len(sp)
        out["spca"] = {"fit_ms": round(sp_ms, 3),
                       "phases_ms": {key: round(sum(t[key + "_ms"] for t in sp) / len(sp), 4)
                                     for key in ("omega", "sketch", "qr", "layout", "pass2", "reduce", "small")},
                       "lazy_fit_speedup": round(sp_ms / fit_ms, 3)}
        log(f"spca_fit_csr {sp_ms:.2f} ms vs lazy {fit_ms:.2f} ms")
    if not args.no_cpu:
        log("cpu baseline (oracle on a row sample)")
        out["cpu_baseline"] = csr_cpu_baseline(c, rph, ci.cpu().numpy(), vv.cpu().numpy())
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", type=int, default=2)
    ap.add_argument("--m", type=int, default=0, help="override rows (smaller runs)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-spca", action="store_true")
    ap.add_argument("--spca-steps", type=int, default=3)
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-plain", action="store_true",
                    help="skip the fit of an FP32 copy of 16-bit X (the plain FP32 path)")
    ap.add_argument("--no-host", action="store_true",
                    help="skip the fit of the same X from pinned host memory (Algorithm 4 streamed)")
    ap.add_argument("--serve-counts", type=str, default="1000,2000,4000",
                    help="requests at 50,200,800 QPS")
    ap.add_argument("--also", type=str, default="1,3,4",
                    help="other workloads measured after the headline one (sub-objects of the line); "
                         "empty for none")
    ap.add_argument("--also-steps", type=int, default=5)
    ap.add_argument("--serve-modes", type=str, default="device,host")
    ap.add_argument("--csr", action="store_true",
                    help="the sparse-X workload instead: CSR X 131,072 x 98,450 at density 0.0244 "
                         "(Experiment 1's feature matrix shape), very sparse Omega, k = 500")
    ap.add_argument("--k", type=int, default=0, help="override k (sparse-X workload)")
    ap.add_argument("--calib-gib", type=float, default=0.0,
                    help="run y = 2 x over this many GiB (FP32) before timing: a reference of "
                         "known traffic for HBM byte counters")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import torch
    import paper_1709_07175_amd as lib
    from synth import config

    lib.load()
    if args.csr:
        return csr_main(args, lib, torch)
    cfg = config(args.config)
    if args.m:
        cfg["m"] = args.m
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    out, X = dense_run(args, lib, torch, cfg, args.steps, args.warmup, headline=True)
    m, n, k = cfg["m"], cfg["n"], cfg["k"]
    if not args.no_serve and n == 4096 and k == 256:
        # projection serving with the fitted V (the 4,096 x 256 map of this workload)
        levels = (50, 200, 800)
        counts = [int(c) for c in args.serve_counts.split(",")]
        V, _ = lib.fit(X, k, cfg["kind"], cfg["omega_seed"], sparse_p=cfg.get("p", 64))
        sv = serving(lib, V, X, levels, counts, args.serve_modes.split(","))
        out["serving"] = sv
        if "device" in sv:
            out["projection_p99_ms"] = {q: sv["device"][q]["p99_ms"] for q in map(str, levels)}
    if not args.no_cpu:
        log("cpu baseline (oracle on a row sample)")
        out["cpu_baseline"] = cpu_baseline(cfg, X)
    del X
    torch.cuda.empty_cache()
    # the other workloads, each at its full size, fits and projections timed
    # the same way (lighter: fewer steps, no serving, host or CPU legs)
    extra = [int(c) for c in args.also.split(",") if c.strip()] if args.also else []
    if extra:
        out["workloads"] = {}
    for cid in extra:
        if cid == args.config:
            continue
        c2 = config(cid)
        try:
            sub, Xc = dense_run(args, lib, torch, c2, args.also_steps, 1, headline=False)
            del Xc
        except (RuntimeError, lib.LspcaError) as e:     # e.g. out of memory on a smaller device
            sub = {"error": str(e)}
        torch.cuda.empty_cache()
        out["workloads"][str(cid)] = sub
    out["paper_context"] = PAPER_CONTEXT
    print(json.dumps(out), flush=True)


def dense_run(args, lib, torch, cfg, steps, warmup, headline):
    """One dense workload: `steps` timed steps (lspca_fit then lspca_transform
    of the same X, inputs resident in HBM), the SPCA baselines on the same X
    and, for 16-bit X, the plain FP32 path. Returns (record, X)."""
    from synth import lowrank_torch
    m, n, k = cfg["m"], cfg["n"], cfg["k"]
    dev = torch.device("cuda:0")
    log(f"generating X {m}x{n} {cfg['dtype']} (seed {cfg['data_seed']})")
    t0 = time.time()
    X = lowrank_torch(m, n, cfg["r"], cfg["spectrum"], cfg["s"], cfg["data_seed"], cfg["dtype"],
                      device=dev)
    torch.cuda.synchronize()
    log(f"generated in {time.time() - t0:.1f}s")
    xbytes = X.numel() * X.element_size()
    stream = torch.cuda.current_stream()
    if headline and args.calib_gib > 0:
        calibrate(torch, dev, args.calib_gib)
    sp = cfg.get("p", 64)

    def step(timing):
        V, s = lib.fit(X, k, cfg["kind"], cfg["omega_seed"], timing=timing, sparse_p=sp)
        tf = lib.last_timings() if timing else None
        Z = lib.transform(X, V, timing=timing)
        tt = lib.last_timings() if timing else None
        return V, s, Z, tf, tt

    for i in range(warmup):
        step(False)
        torch.cuda.synchronize()
        log(f"warmup {i + 1}/{warmup} done")

    phases = []
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    t0 = time.perf_counter()
    for i in range(steps):
        _, _, _, tf, tt = step(True)
        phases.append((tf, tt))
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_step = ev0.elapsed_time(ev1) / steps
    log(f"timed {steps} steps: {ms_step:.3f} ms/step (wall {wall / steps * 1e3:.3f})")

    def avg(key, which=0):
        return sum(p[which][key] for p in phases) / len(phases)

    fit_ms = avg("total_ms", 0)
    tr_ms = avg("transform_ms", 1)
    sketch_ms = avg("sketch_ms", 0)
    factor_ms = avg("factor_ms", 0)
    small_ms = avg("small_ms", 0)
    pass_ms = sketch_ms + factor_ms + avg("reduce_ms") + avg("layout_ms")
    workload = (f"lazy-spca fit+projection, X {m}x{n} {cfg['dtype']} low-rank+noise, "
                f"{cfg['kind']} Omega, k={k}")
    out = {
        "metric": "X-stream GB/s (% HBM/MFMA roofline) per Lazy SPCA fit vs SPCA; projection p99 ms",
        "value": round(xbytes / (fit_ms * 1e-3) / 1e9, 3),
        "unit": "GB/s",
        "value_basis": "bytes of X / device time of one whole lspca_fit (Omega, pass, small FP64 stage), "
                       "averaged over the timed steps; each step also runs lspca_transform of the same X",
        "n_gpus": 1,
        "steps": steps,
        "warmup": warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"f64": "f64", "f32": "f32", "bf16": "bf16", "f16": "f16"}[cfg["dtype"]],
        "data": "synthetic",
        "config": {"workload": workload, "m": m, "n": n, "k": k, "x_bytes": xbytes,
                   "parallelism": "single-gpu"},
        "phases_ms": {"fit_total": round(fit_ms, 4), "omega": round(avg("omega_ms"), 4),
                      "sketch": round(sketch_ms, 4), "layout": round(avg("layout_ms"), 4),
                      "factor_F_G": round(factor_ms, 4),
                      "reduce": round(avg("reduce_ms"), 4), "small_fp64": round(small_ms, 4),
                      "transform": round(tr_ms, 4)},
        "fit_ms": round(fit_ms, 4),
        "fit_x_stream_GBs": round(xbytes / (fit_ms * 1e-3) / 1e9, 3),
        "fit_pass_x_stream_GBs": round(xbytes / (pass_ms * 1e-3) / 1e9, 3),
        "step_x_stream_GBs": round(2 * xbytes / (ms_step * 1e-3) / 1e9, 3),
        "transform_x_stream_GBs": round(xbytes / (tr_ms * 1e-3) / 1e9, 3),
        "roofline": roofline(cfg, m, n, k, xbytes, X.element_size(), sketch_ms),
        "kernels": pass_rooflines(cfg, m, n, k, xbytes, X.element_size(), phases),
    }
    if not headline:
        out = {key: out[key] for key in ("value", "unit", "value_basis", "ms_per_step", "steps", "dtype",
                                         "config", "phases_ms", "fit_ms", "fit_x_stream_GBs",
                                         "fit_pass_x_stream_GBs", "step_x_stream_GBs",
                                         "transform_x_stream_GBs", "roofline", "kernels")}
    spca_steps = args.spca_steps if headline else 2
    if not args.no_spca:
        # the non-lazy baseline on the same X: Algorithm 1 with the GPU
        # tall-skinny Householder QR (two passes over X)
        try:
            lib.spca_fit(X, k, cfg["kind"], cfg["omega_seed"], sparse_p=sp)
            torch.cuda.synchronize()
            sps = []
            for _ in range(spca_steps):
                lib.spca_fit(X, k, cfg["kind"], cfg["omega_seed"], timing=True, sparse_p=sp)
                sps.append(lib.last_timings())
            sp_ms = sum(t["total_ms"] for t in sps) / len(sps)
            out["spca"] = {
                "fit_ms": round(sp_ms, 4),
                "fit_x_stream_GBs": round(xbytes / (sp_ms * 1e-3) / 1e9, 3),
                "phases_ms": {key: round(sum(t[key + "_ms"] for t in sps) / len(sps), 4)
                              for key in ("omega", "sketch", "qr", "pass2", "reduce", "small")},
                "lazy_fit_speedup": round(sp_ms / fit_ms, 3),
            }
            log(f"spca_fit {sp_ms:.3f} ms vs lazy fit {fit_ms:.3f} ms")
            # Algorithm 3: one pass with the R factor updated per stripe
            lib.spca_fit_stream(X, k, cfg["kind"], cfg["omega_seed"], sparse_p=sp)
            torch.cuda.synchronize()
            ss = []
            for _ in range(spca_steps):
                lib.spca_fit_stream(X, k, cfg["kind"], cfg["omega_seed"], timing=True, sparse_p=sp)
                ss.append(lib.last_timings())
            ss_ms = sum(t["total_ms"] for t in ss) / len(ss)
            out["spca_stream"] = {
                "fit_ms": round(ss_ms, 4),
                "fit_x_stream_GBs": round(xbytes / (ss_ms * 1e-3) / 1e9, 3),
                "phases_ms": {key: round(sum(t[key + "_ms"] for t in ss) / len(ss), 4)
                              for key in ("omega", "sketch", "qr", "factor", "reduce", "pass2", "small")},
                "lazy_fit_speedup": round(ss_ms / fit_ms, 3),
            }
            log(f"spca_fit_stream {ss_ms:.3f} ms")
        except lib.LspcaError as e:
            out["spca"] = {"error": str(e)}
    if not args.no_plain and cfg["dtype"] in ("bf16", "f16"):
        # the same values as FP32 through the plain FP32 path (exact copy)
        log("fit of an FP32 copy of X (plain FP32 path)")
        X32 = X.float()
        lib.fit(X32, k, cfg["kind"], cfg["omega_seed"], sparse_p=sp)
        torch.cuda.synchronize()
        pts = []
        for _ in range(2):
            lib.fit(X32, k, cfg["kind"], cfg["omega_seed"], timing=True, sparse_p=sp)
            pts.append(lib.last_timings())
        p_ms = sum(t["total_ms"] for t in pts) / len(pts)
        out["fp32_plain"] = {"fit_ms": round(p_ms, 3),
                             "x_bytes": X32.numel() * 4,
                             "phases_ms": {key: round(sum(t[key + "_ms"] for t in pts) / len(pts), 4)
                                           for key in ("omega", "sketch", "factor", "reduce", "small")},
                             "lazy_16bit_speedup": round(p_ms / fit_ms, 3)}
        log(f"FP32 copy: fit {p_ms:.2f} ms vs {fit_ms:.2f} ms")
        del X32
        torch.cuda.empty_cache()
    if headline and not args.no_host:
        # Algorithm 4 with X in pinned host memory (the out-of-core regime):
        # host-to-device copies of stripes overlapped with the pass
        log("copying X to pinned host memory")
        Xh = torch.empty(X.shape, dtype=X.dtype, pin_memory=True)
        Xh.copy_(X)
        torch.cuda.synchronize()
        lib.fit_host(Xh, k, cfg["kind"], cfg["omega_seed"], sparse_p=sp)
        hts = []
        for _ in range(2):
            lib.fit_host(Xh, k, cfg["kind"], cfg["omega_seed"], timing=True, sparse_p=sp)
            hts.append(lib.last_timings())
        h_ms = sum(t["total_ms"] for t in hts) / len(hts)
        out["fit_host"] = {"fit_ms": round(h_ms, 3), "x_stream_GBs": round(xbytes / (h_ms * 1e-3) / 1e9, 3),
                           "pass_ms": round(sum(t["factor_ms"] for t in hts) / len(hts), 3),
                           "note": "X in pinned host memory; stripes copied host-to-device while the "
                                   "previous stripe is processed (PCIe-inclusive, not the headline value)"}
        log(f"fit from host memory: {h_ms:.1f} ms")
        del Xh
    return out, X


if __name__ == "__main__":
    main()
