"""Throughput benchmark of the adaptive H2-matrix product on one MI355X.

One step = one complete h2_mul (exact product in the induced tree, coarsening,
adaptive row and column bases, couplings) on operands already resident in HBM
with the product plan cached.  Default workload: unit sphere from an
icosahedron refined 5 times (n = 20480 triangle centroids), single-layer
kernel 1/(4 pi |x-y|) with the row-nearfield-mean diagonal, leaf size 64,
eta = 1, tensor Chebyshev order 4 (k = 64), A*A at eps = 1e-6.

The headline leg is plain FP64 at the workload's eps.  The library runs the
FP32 bulk only for eps >= 1e-5 (below that its rounding would exceed the
coarsening tolerance), so the FP32-bulk / FP64-recompression form is timed
against plain FP64 on the same operands at eps = 1e-4 (`modes`: products/s,
precision used and roofline of each leg).

Timing: `value`, ms_per_step and the latencies come from the timed steps
without instrumentation (each product replays its HIP graph, captured in
the warm-up). The same number of products then runs again with
HIP events around every kernel launch, on the stream of the launch (timing
mode 2): that pass gives the per-kernel device times of the roofline; the
dominant kernel is the one with the largest device time.  Its algorithmic flops (or bytes) per
launch come from one untimed counting call (timing mode 3: the QR and SVD
kernels report the sizes they factored).  achieved = algorithmic work per
launch / average launch duration.

cpu_baseline: the FP64 oracle (test infrastructure) on one host core (its many
small factorizations run fastest single-threaded), on a bounded sample: the
full oracle product of the same construction one refinement level lower
(n = 5120), scaled to the timed workload by the oracle's own time ratio of
the two products, both measured in full once on one host core
(`--oracle-scaling`, recorded in profiles/oracle_icosphere5_slp.md); for the
small grid workload the full product itself.

global_error (untimed): the relative spectral error of one product, both
norms estimated by ten device power-iteration steps, with the storage of the
product.  --sweep LEVELS instead times G*G, G*K and K*K over icosphere levels, and
--sweep-cube M K*K on the cube surface with m x m squares per face, at eps
1e-4, and reports time per degree of freedom, storage and error per n.

--workload batch64 times a batch of 64 independent products submitted at once
(overlapping on the context's lanes) against the same products one at a
time (run it with GPU_MAX_HW_QUEUES=16 in the environment: 4 lanes of 3
streams each share the default 4 in-order hardware queues otherwise); --serve serves a seeded Poisson stream of requests on resident operands
and reports throughput and p50/p99 latency.

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "H² products/s + roofline fraction at stated eps vs plain FP64; p50/p99 latency"
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6     # 256 CUs x 2.4 GHz x 128 FP64 flop/clk/CU (vector FMA and MFMA alike)
ALU_KERNELS = ("qr_kernel", "svd_kernel", "svd_narrow_kernel", "chol_kernel")

WORKLOADS = {
    "grid32": dict(desc="32x32 grid in [0,1]^2, -log|x-y| (diag 0), leaf 32, eta 1/2, Chebyshev order 3 (k=9), "
                    "A*A, eps 1e-4",
               eps=1e-4, geom=("grid", 32), kernel=0, leaf=32, order=3, eta=0.5, diag=0, sample=None),
    "icosphere5_slp": dict(desc="icosphere level 5 (n=20480 centroids), 1/(4 pi |x-y|) (diag = row nearfield mean), leaf 64, "
                    "eta 1, Chebyshev order 4 (k=64), A*A, eps 1e-6",
               eps=1e-6, geom=("ico", 5), kernel=1, leaf=64, order=4, eta=1.0, diag=1, sample=("ico", 4),
               cmp_eps=1e-4),
    "icosphere6_slp_dlp": dict(desc="icosphere level 6 (n=81920 centroids), single layer 1/(4 pi |x-y|) times double layer "
                    "(x-y).n_y/(4 pi |x-y|^3), leaf 64, eta 1, Chebyshev order 4 (k=64), eps 1e-4",
               eps=1e-4, geom=("ico", 6), kernel=1, leaf=64, order=4, eta=1.0, diag=1, dlp=True,
               sample=("ico", 4)),
}


def geometry(g):
    from paper_2403_01566_amd import workloads as W
    if g[0] == "grid":
        return W.grid2d(g[1]), None
    return W.icosphere(g[1])


def build(h2, ctx, cfg, geom=None):
    P, nrm = geometry(geom or cfg["geom"])
    T = h2.Tree(ctx, P, cfg["leaf"])
    A = h2.Matrix.interpolated(ctx, T, T, cfg["kernel"], cfg["order"], cfg["eta"], cfg["diag"], nrm)
    B = h2.Matrix.interpolated(ctx, T, T, h2.KERNEL_LAPLACE_DLP, cfg["order"], cfg["eta"], 0, nrm) \
        if cfg.get("dlp") else A
    return T, A, B


def say(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def run_mode(h2, ctx, A, B, eps, prec, steps, warmup):
    nk = h2.NKERNEL
    for _ in range(warmup):
        C, _ = h2.mul(ctx, A, B, eps, h2.default_options(precision=prec, graph=1))  # also captures the graph
        del C
    # untimed: algorithmic work of every kernel from the sizes the kernels report
    C, cnt = h2.mul(ctx, A, B, eps, h2.default_options(precision=prec, timing=3))
    del C
    # throughput and latency: plain products, no instrumentation
    lat = []
    t0 = time.perf_counter()
    for _ in range(steps):
        t1 = time.perf_counter()
        C, st = h2.mul(ctx, A, B, eps, h2.default_options(precision=prec, graph=1))  # returns when the device is done
        lat.append(time.perf_counter() - t1)
        del C
    total = time.perf_counter() - t0
    # the same number of products again with HIP events around every kernel
    # launch (on the stream of the launch): per-kernel device time for the roofline
    opt = h2.default_options(precision=prec, timing=2)
    t_k, l_k, phase = [0.0] * nk, [0] * nk, [0.0] * 8
    t0 = time.perf_counter()
    for _ in range(steps):
        C, st = h2.mul(ctx, A, B, eps, opt)
        del C
        for i in range(nk):
            t_k[i] += st["t_kernel"][i]
            l_k[i] += st["launches_kernel"][i]
        for i in range(8):
            phase[i] += st["t_phase"][i]
    total_events = time.perf_counter() - t0
    return dict(total=total, total_events=total_events, lat=lat, st=st, cnt=cnt, t_k=t_k, l_k=l_k,
                phase=[p / steps for p in phase])


def measured_traffic(workload, kernel):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary (FETCH_SIZE and WRITE_SIZE, scaled by a copy-kernel calibration),
    or None when there is none or the kernels or the planner changed since."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"counters_{workload}.json")
    if not os.path.exists(path):
        return None
    data = json.load(open(path))
    h = hashlib.sha256()
    for f in ("h2_kernels.hip", "h2_plan.cpp"):  # the kernels and the launches they receive
        h.update(open(os.path.join(ROOT, "paper_2403_01566_amd", "csrc", f), "rb").read())
    if data.get("source_sha256") != h.hexdigest():
        return None
    k = data.get("kernels", {}).get(kernel)
    return None if k is None else k["hbm_bytes_per_launch"]


COUNTER_FILES = {"icosphere5_slp": "icosphere5_slp"}


def roofline(names, r, steps, workload):
    t_k, l_k, cnt = r["t_k"], r["l_k"], r["cnt"]
    dom = max(range(len(names)), key=lambda i: t_k[i])
    name = names[dom]
    launches = cnt["launches_kernel"][dom]
    avg_launch_s = max(1e-12, t_k[dom] / max(1, l_k[dom]) * 1e-3)
    alu = name.startswith(ALU_KERNELS)
    per_launch = (cnt["flops_kernel"][dom] if alu else cnt["bytes_kernel"][dom]) / max(1, launches)
    if alu:
        achieved = per_launch / avg_launch_s / 1e12
        roof = {"bound": "alu", "achieved": achieved, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": achieved / FP64_PEAK_TFLOPS, "traffic": None}
    else:
        achieved = per_launch / avg_launch_s / 1e9
        roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": None}
    tr = measured_traffic(COUNTER_FILES[workload], name) if workload in COUNTER_FILES else None
    roof["traffic"] = tr
    roof["traffic_unit"] = "HBM bytes per launch"
    roof.update({"kernel": name, "launches_per_step": launches, "ms_per_launch": avg_launch_s * 1e3,
                 "units_per_launch": cnt["units_kernel"][dom] / max(1, launches),
                 "algorithmic_per_launch": per_launch,
                 "share_of_device_time": t_k[dom] / max(1e-30, sum(t_k))})
    return roof


ORACLE_SCALING = os.path.join(ROOT, "profiles", "oracle_icosphere5_slp.md")


def _oracle_time(cfg, geom, threads=1):
    """Seconds of one full oracle product (test infrastructure, untuned) of
    the workload's construction on `geom`, with `threads` BLAS threads."""
    import oracle as O
    from threadpoolctl import threadpool_limits
    P, nrm = geometry(geom)
    T = O.ClusterTree(P, cfg["leaf"])
    A = O.build_interpolated(T, cfg["kernel"], cfg["order"], cfg["eta"], diag=cfg["diag"], normals=nrm)
    B = O.build_interpolated(T, O.KERNEL_DLP, cfg["order"], cfg["eta"], normals=nrm) if cfg.get("dlp") else A
    with threadpool_limits(limits=threads, user_api="blas"):
        t0 = time.perf_counter()
        O.mul(A, B, cfg["eps"])
        return time.perf_counter() - t0, len(P)


def _oracle_scaling():
    """The oracle's own ratio of its time on the timed workload to its time on
    the sample, measured once in full on one core (bench.py --oracle-scaling),
    as recorded in the profiles folder (a JSON line)."""
    try:
        for line in open(ORACLE_SCALING):
            line = line.strip()
            if line.startswith("{") and '"t_full_s"' in line:
                return json.loads(line)
    except OSError:
        pass
    return None


def cpu_baseline(cfg, workload):
    """The oracle (test infrastructure, untuned) on the host, one BLAS thread
    (its many small factorizations run fastest that way), on a bounded sample:
    the full oracle product of the same construction one refinement level
    lower, scaled to the timed workload by the oracle's own measured time
    ratio between the two (recorded from a full run of both on one core);
    the small grid workload runs in full."""
    geom = cfg["sample"] or cfg["geom"]
    dt, n = _oracle_time(cfg, geom)
    if not cfg["sample"]:
        return {"value": 1.0 / dt, "unit": "products/s", "cores": 1, "kind": "oracle",
                "sample": f"full oracle product of the timed workload, {dt:.1f} s", "seconds": dt}
    rec = _oracle_scaling() if workload == "icosphere5_slp" else None
    if rec is None:
        return {"value": None, "unit": "products/s", "cores": 1, "kind": "oracle",
                "sample": f"full oracle product at icosphere level {geom[1]} (n={n}), {dt:.1f} s; no recorded "
                          f"scaling to the timed workload", "seconds": dt}
    ratio = rec["t_full_s"] / rec["t_sample_s"]
    return {"value": 1.0 / (dt * ratio), "unit": "products/s", "cores": 1, "kind": "oracle",
            "sample": f"full oracle product of the same construction at icosphere level {geom[1]} (n={n}), "
                      f"{dt:.1f} s on one core, scaled by the oracle's own time ratio {ratio:.1f} of the timed "
                      f"workload to this sample (both measured in full on one core of {rec['host_cpu']}: "
                      f"{rec['t_full_s']:.0f} s and {rec['t_sample_s']:.1f} s)",
            "seconds": dt, "full_product_seconds_recorded": rec["t_full_s"]}


def hbm_probe(gib=4, reps=20):
    """Rates that plain torch kernels reach on this device: a copy (read and
    write), a sum (read) and a fill (write) of `gib` GiB of float64, each the
    mean of `reps` launches after 3 untimed ones.  Context for the GEMM's
    fraction of the HBM peak."""
    import torch
    n = gib << 30
    a = torch.ones(n // 8, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    out = {"bytes": n}
    for name, fn, moved in (("copy", lambda: b.copy_(a), 2 * n), ("sum", lambda: a.sum(), n),
                            ("fill", lambda: b.fill_(1.0), n)):
        for _ in range(3):
            fn()
        torch.cuda.synchronize()
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        out[name] = {"ms": ms, "GB_per_s": moved / ms / 1e6}
        say(f"{name}: {ms:.3f} ms, {moved / ms / 1e9:.2f} TB/s")
    return out


def global_error(h2, ctx, A, B, n, eps, prec, iters=10):
    """Relative spectral error ||AB - C||_2 / ||AB||_2 of one product C, both
    norms estimated by `iters` power-iteration steps on the device from a
    seeded start vector (the error column of the paper's experiments).
    Untimed: it runs after the timed steps."""
    from paper_2403_01566_amd import workloads as W
    C, _ = h2.mul(ctx, A, B, eps, h2.default_options(precision=prec))
    z0 = W.start_vector(n, 2403)
    t0 = time.perf_counter()
    err, nxy = h2.product_error(A, B, C, z0, iters)
    dt = time.perf_counter() - t0
    return {"rel_spectral": err / nxy, "abs": err, "norm_product": nxy, "power_steps": iters,
            "seconds": dt, "storage_mb": C.storage_bytes() / 1e6}


SWEEP = {
    "slp": dict(x=(1, 1), y=(1, 1), desc="G*G, G = single layer 1/(4 pi |x-y|) (diag = row nearfield mean)"),
    "slp_dlp": dict(x=(1, 1), y=(2, 0), desc="G*K, K = double layer (x-y).n_y/(4 pi |x-y|^3)"),
    "dlp": dict(x=(2, 0), y=(2, 0), desc="K*K"),
}


def sweep(h2, ctx, jobs, steps, eps):
    """Time per degree of freedom over n (the runtime plot of the paper's
    experiments), with the storage and the relative spectral error of each
    product (the columns of its tables).  jobs: (operator, geometry, size)
    with geometry "ico" (icosphere level) or "cube" (m x m squares per face
    of [-1,1]^3); leaf 64, eta 1, Chebyshev order 4, the given eps.  A product
    that the library rejects (a rank cap, memory) is reported with its error."""
    from paper_2403_01566_amd import workloads as W
    rows = []
    for kind, geo, size in jobs:
        kc = SWEEP[kind]
        P, nrm = W.icosphere(size) if geo == "ico" else W.cube_surface(size)
        T = h2.Tree(ctx, P, 64)
        row = {"operator": kind, "geometry": geo, "size": size, "n": int(T.n)}
        try:
            A = h2.Matrix.interpolated(ctx, T, T, kc["x"][0], 4, 1.0, kc["x"][1], nrm)
            B = h2.Matrix.interpolated(ctx, T, T, kc["y"][0], 4, 1.0, kc["y"][1], nrm) if kc["y"] != kc["x"] else A
            t0 = time.perf_counter()
            C, st0 = h2.mul(ctx, A, B, eps)   # first call: host plan + device run
            first = time.perf_counter() - t0
            del C
            ts = []
            for _ in range(steps):
                t1 = time.perf_counter()
                C, st = h2.mul(ctx, A, B, eps)
                ts.append(time.perf_counter() - t1)
                del C
            ts.sort()
            med = ts[len(ts) // 2]
            ge = global_error(h2, ctx, A, B, int(T.n), eps, st["prec_used"])
            row.update({"ms": med * 1e3, "us_per_dof": med * 1e6 / T.n, "first_call_ms": first * 1e3,
                        "plan_ms": st0["t_plan_ms"], "storage_mb": ge["storage_mb"],
                        "rel_error": ge["rel_spectral"], "precision_used": st["prec_used"],
                        "rank_max": [st["rank_max_row"], st["rank_max_col"]], "n_adm": st["n_adm"],
                        "n_inadm": st["n_inadm"]})
            say(f"sweep {kind} {geo} {size} n={T.n}: {row['ms']:.1f} ms, {row['us_per_dof']:.3f} us/DOF, "
                f"{row['storage_mb']:.1f} MB, rel. error {row['rel_error']:.2e}")
            del A, B
        except h2.H2Error as e:
            row["error"] = str(e)
            say(f"sweep {kind} {geo} {size} n={T.n}: {e}")
        rows.append(row)
        del T
    return {"sweep": rows, "eps": eps, "steps": steps,
            "config": {"geometry": {"ico": "icosphere (triangle centroids, outward normals)",
                                    "cube": "surface of [-1,1]^3, 12 m^2 triangle centroids, face normals"},
                       "leaf": 64, "eta": 1.0, "order": 4,
                       "operators": {k: v["desc"] for k, v in SWEEP.items()}}}


def run_batch64(h2, args):
    """Many independent products (64 instances, n log-uniform in [1024, 32768],
    orders 3..6, eps 1e-5, FP32 bulk): all submitted at once and overlapping
    on the context's lanes; one step = one batch.  The same products one after
    the other (h2_mul) are timed too."""
    from paper_2403_01566_amd import workloads as W
    ctx = h2.Context(0)
    h2.set_lanes(ctx, args.lanes)
    inst = W.batched_instances()
    say(f"building {len(inst)} operands")
    ops = []
    for q in inst:
        T = h2.Tree(ctx, W.uniform2d(q["n"], q["points_seed"]), q["leaf"])
        ops.append((T, h2.Matrix.interpolated(ctx, T, T, h2.KERNEL_NEG_LOG, q["order"], 0.5, h2.DIAG_ZERO)))
    eps = 1e-5
    opt = h2.default_options(precision=h2.PREC_FP32_BULK, graph=1)
    pairs = [(A, A) for _, A in ops]
    say("first batch (plans built on the host)")
    t0 = time.perf_counter()
    out = h2.mul_batch(ctx, pairs, eps, opt)
    t_first = time.perf_counter() - t0
    prec = [st["prec_used"] for _, st in out]
    del out
    for _ in range(args.warmup):
        h2.mul_batch(ctx, pairs, eps, opt)
    say(f"timing {args.steps} batches")
    t0 = time.perf_counter()
    for _ in range(args.steps):
        out = h2.mul_batch(ctx, pairs, eps, opt)
        del out
    total = time.perf_counter() - t0
    say("the same products one at a time")
    t0 = time.perf_counter()
    for A, B in pairs:
        C, _ = h2.mul(ctx, A, B, eps, opt)
        del C
    seq = time.perf_counter() - t0
    ms = 1000.0 * total / args.steps
    return {
        "metric": "batched H2 products/s (64 independent products)",
        "value": len(pairs) * args.steps / total,
        "unit": "products/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "strong",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic (seeded uniform points, operands built by interpolation on the host, resident on the device)",
        "config": {"workload": "64 products A_i A_i, n_i log-uniform in [1024, 32768] (PCG64 seed 2403), uniform "
                               "points in [0,1]^2, -log|x-y|, Chebyshev order 3..6, leaf 32 (order <= 4) or 64, "
                               "eta 1/2, eps 1e-5, FP32 bulk", "lanes": args.lanes, "total_n": sum(T.n for T, _ in ops),
                   "fp32_bulk_products": int(sum(1 for x in prec if x == h2.PREC_FP32_BULK))},
        "sequential_products_per_s": len(pairs) / seq,
        "overlap_speedup": seq / (total / args.steps),
        "first_batch_s": t_first,
    }


def run_serve(h2, args):
    """Serving: a seeded Poisson stream of product requests on resident
    operands.  Requests are admitted on arrival while fewer than 2 x lanes
    products are in flight and overlap on the lanes.  Each product's plan is
    resident, so its workspace is already held by the lane arenas; a request
    whose submission still runs out of device memory (its result, or an arena
    that must grow) waits until products in flight have finished, and is
    refused only if it fails with none in flight.  Latency = result ready -
    arrival."""
    from collections import deque
    from paper_2403_01566_amd import workloads as W
    nreq = args.serve_requests + args.serve_warmup
    reqs = W.serving_requests(nreq, rate=args.serve_rate, m_range=(12, args.serve_mmax))
    ctx = h2.Context(0)
    h2.set_lanes(ctx, args.lanes)
    ops = {}
    for r in reqs:
        key = (r["geometry"], r["m"], r["order"])
        if key in ops:
            continue
        P, nrm = W.serving_points(r["geometry"], r["m"])
        if r["geometry"] == "2d":
            T = h2.Tree(ctx, P, 32 if r["order"] ** 2 <= 32 else 64)
            A = h2.Matrix.interpolated(ctx, T, T, h2.KERNEL_NEG_LOG, r["order"], 0.5, h2.DIAG_ZERO)
        else:
            T = h2.Tree(ctx, P, 32 if r["order"] ** 3 <= 32 else 64)
            A = h2.Matrix.interpolated(ctx, T, T, h2.KERNEL_LAPLACE_SLP, r["order"], 1.0, h2.DIAG_ROW_NEARFIELD_MEAN,
                                       nrm)
        ops[key] = (T, A)
    def options(eps):
        return h2.default_options(precision=h2.PREC_FP32_BULK if eps >= 1e-5 else h2.PREC_FP64, graph=1)
    say(f"{len(ops)} operands; planning every (operand, precision) class once")
    seen, rejected_cls = set(), {}
    for r in reqs:
        k = (r["geometry"], r["m"], r["order"], r["eps"])
        if k not in seen:
            seen.add(k)
            if len(seen) % 10 == 0:
                say(f"  {len(seen)} request classes ready")
            try:
                C, _ = h2.mul(ctx, ops[k[:3]][1], ops[k[:3]][1], r["eps"], options(r["eps"]))
                del C
            except h2.H2Error as e:  # e.g. a rank cap: the library refuses, the server reports it
                rejected_cls[k] = str(e)
    if rejected_cls:
        say(f"{len(rejected_cls)} request classes refused by the library: {sorted(set(rejected_cls.values()))}")
    cap = 2 * args.lanes
    say(f"serving {nreq} requests at {args.serve_rate}/s, at most {cap} in flight")
    pending = deque(reqs)
    inflight = []
    done, refused = [], []
    refused_reasons = set(rejected_cls.values())
    memory_waits = 0
    t_start = time.perf_counter()
    while pending or inflight:
        now = time.perf_counter() - t_start
        progressed = False
        while pending and pending[0]["t"] <= now and len(inflight) < cap:
            r = pending.popleft()
            progressed = True
            if (r["geometry"], r["m"], r["order"], r["eps"]) in rejected_cls:
                refused.append(r)
                continue
            A = ops[(r["geometry"], r["m"], r["order"])][1]
            try:
                inflight.append((r, h2.submit(ctx, A, A, r["eps"], options(r["eps"]))))
            except h2.H2Error as e:
                if e.code == h2.H2_ERR_OUT_OF_MEMORY and inflight:
                    # memory held by products in flight: admit it once some have finished
                    pending.appendleft(r)
                    memory_waits += 1
                    break
                refused.append(r)
                refused_reasons.add(str(e))
        still = []
        for r, j in inflight:
            if j.poll():
                try:
                    C, st = j.wait()
                    del C
                    done.append((r, time.perf_counter() - t_start))
                except h2.H2Error:
                    refused.append(r)
                j.close()
                progressed = True
                if (len(done) + len(refused)) % 50 == 0:
                    say(f"  {len(done)} served, {len(refused)} refused, {len(pending)} not yet admitted at "
                        f"t = {time.perf_counter() - t_start:.1f} s")
            else:
                still.append((r, j))
        inflight = still
        if not progressed:
            time.sleep(0.0002)
    order = {id(r): i for i, r in enumerate(reqs)}
    measured = [(r, t) for r, t in done if order[id(r)] >= args.serve_warmup]
    lat = sorted(1000.0 * (t - r["t"]) for r, t in measured)
    t_first = min(r["t"] for r, _ in measured)
    t_last = max(t for _, t in measured)
    pct = lambda q: lat[min(len(lat) - 1, int(math.ceil(q * len(lat))) - 1)]
    return {
        "metric": "served H2 products/s and latency (Poisson stream)",
        "value": len(measured) / (t_last - t_first),
        "unit": "products/s",
        "n_gpus": 1,
        "higher_is_better": True,
        "offered_rate": args.serve_rate,
        "requests": len(measured),
        "warmup_requests": args.serve_warmup,
        "refused_requests": sum(1 for r in refused if order[id(r)] >= args.serve_warmup),
        "refused_reasons": sorted(refused_reasons),
        "admissions_deferred_for_memory": memory_waits,
        "latency_ms": {"p50": pct(0.5), "p99": pct(0.99), "max": lat[-1]},
        "saturated": len(measured) / (t_last - t_first) < 0.9 * args.serve_rate,
        "dtype": "f32+f64",
        "data": "synthetic (seeded request stream and operands)",
        "config": {"workload": f"Poisson arrivals {args.serve_rate}/s (PCG64 seed 2404); geometry 2D uniform or "
                               f"Fibonacci sphere, n = 2^m, m in 12..{args.serve_mmax}, order 2D 3..8 / sphere "
                               f"3..4, eps in 1e-4, 1e-6, 1e-8 (FP32 bulk at eps >= 1e-5)",
                   "operands": len(ops), "request_classes": len(seen), "lanes": args.lanes,
                   "max_in_flight": cap},
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="icosphere5_slp", choices=sorted(WORKLOADS) + ["batch64"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--oracle-scaling", action="store_true",
                    help="time the full oracle product on the sample and on the workload (one core), print "
                         "the JSON line the cpu_baseline scaling reads, and exit (takes minutes)")
    ap.add_argument("--fp64-only", action="store_true")
    ap.add_argument("--no-global-error", action="store_true",
                    help="skip the untimed power-iteration error (profiled runs: only the products' kernels)")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only copy MIB MiB device-to-device once (HBM counter calibration)")
    ap.add_argument("--hbm-probe", action="store_true",
                    help="only time plain device copy, sum and fill over 4 GiB (practical HBM rates)")
    ap.add_argument("--sweep", default="", metavar="LEVELS",
                    help="comma-separated icosphere levels: time per DOF, storage and error per n, then exit")
    ap.add_argument("--sweep-cube", default="", metavar="M",
                    help="comma-separated squares per cube edge: K*K on the cube surface (n = 12 m^2)")
    ap.add_argument("--sweep-eps", type=float, default=1e-4)
    ap.add_argument("--lanes", type=int, default=4, help="lanes (streams) for batched and served products")
    ap.add_argument("--serve", action="store_true", help="serve a Poisson stream of requests instead")
    ap.add_argument("--serve-requests", type=int, default=1000)
    ap.add_argument("--serve-warmup", type=int, default=50)
    ap.add_argument("--serve-rate", type=float, default=200.0)
    ap.add_argument("--serve-mmax", type=int, default=15,
                    help="largest m (n = 2^m); the workload names 17, whose plans exceed the memory here")
    args = ap.parse_args()
    if args.copy_probe:
        import torch
        a = torch.ones(args.copy_probe * 131072, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": a.numel() * 8}), flush=True)
        return
    if args.hbm_probe:
        print(json.dumps(hbm_probe()), flush=True)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print(json.dumps({"error": "the product runs on one GPU; --gpus above 1 is not supported",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    if args.oracle_scaling:
        import platform
        cfg = WORKLOADS[args.workload]
        ts, ns = _oracle_time(cfg, cfg["sample"])
        say(f"oracle sample (n={ns}): {ts:.1f} s")
        tf, nf = _oracle_time(cfg, cfg["geom"])
        say(f"oracle full workload (n={nf}): {tf:.1f} s")
        model = platform.machine()
        try:
            model = next(l.split(":", 1)[1].strip() for l in open("/proc/cpuinfo") if l.startswith("model name"))
        except (OSError, StopIteration):
            pass
        print(json.dumps({"workload": args.workload, "t_sample_s": ts, "n_sample": ns, "t_full_s": tf, "n_full": nf,
                          "blas_threads": 1, "host_cpu": model, "host_cpus_visible": os.cpu_count()}), flush=True)
        return
    from paper_2403_01566_amd import h2
    if args.serve:
        print(json.dumps(run_serve(h2, args)), flush=True)
        return
    if args.workload == "batch64":
        print(json.dumps(run_batch64(h2, args)), flush=True)
        return
    if args.sweep or args.sweep_cube:
        ctx = h2.Context(0)
        jobs = [(k, "ico", int(x)) for k in ("slp", "slp_dlp", "dlp") for x in args.sweep.split(",") if x]
        jobs += [("dlp", "cube", int(x)) for x in args.sweep_cube.split(",") if x]
        print(json.dumps(sweep(h2, ctx, jobs, max(1, args.steps), args.sweep_eps)), flush=True)
        return
    names = h2.kernel_names()
    cfg = WORKLOADS[args.workload]
    eps = cfg["eps"]
    ctx = h2.Context(0)
    say(f"building operands: {cfg['desc']}")
    T, A, B = build(h2, ctx, cfg)
    # headline: plain FP64 at the workload's eps.  The library runs the FP32
    # bulk only at eps >= 1e-5, so the FP32-bulk / FP64-recompression form is
    # compared with plain FP64 on the same operands at a looser eps.
    modes = [("fp64", h2.PREC_FP64, eps)]
    cmp_eps = cfg.get("cmp_eps")
    if not args.fp64_only:
        if cmp_eps:
            modes += [("fp64_cmp", h2.PREC_FP64, cmp_eps), ("fp32_bulk_cmp", h2.PREC_FP32_BULK, cmp_eps)]
        else:
            modes += [("fp32_bulk", h2.PREC_FP32_BULK, eps)]
    res = {}
    for name, prec, e in modes:
        say(f"timing {name} (eps {e}): {args.warmup} warmup + {args.steps} steps")
        res[name] = run_mode(h2, ctx, A, B, e, prec, args.steps, args.warmup)
        res[name]["eps"] = e
        say(f"{name}: {1000.0 * res[name]['total'] / args.steps:.1f} ms per product")
    head = "fp32_bulk" if "fp32_bulk" in res and res["fp32_bulk"]["st"]["prec_used"] == h2.PREC_FP32_BULK else "fp64"
    r = res[head]
    st = r["st"]
    ms = 1000.0 * r["total"] / args.steps
    lat_ms = sorted(1000.0 * x for x in r["lat"])
    p50 = lat_ms[len(lat_ms) // 2]
    p99 = lat_ms[min(len(lat_ms) - 1, int(math.ceil(0.99 * len(lat_ms))) - 1)]
    out = {
        "metric": METRIC,
        "value": 1000.0 / ms,
        "unit": "products/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "strong",
        "vs_baseline": None,
        "dtype": "f32+f64" if head == "fp32_bulk" else "f64",
        "data": "synthetic (seeded geometry, operands built by interpolation on the host, resident on the device)",
        "config": {"workload": cfg["desc"], "n": int(T.n), "eps": eps, "n_adm": st["n_adm"],
                   "n_inadm": st["n_inadm"], "rank_max": [st["rank_max_row"], st["rank_max_col"]]},
        "latency_ms": {"p50": p50, "p99": p99},
        "instrumented_ms_per_step": 1000.0 * r["total_events"] / args.steps,
        "roofline": roofline(names, r, args.steps, args.workload),
        "phase_ms": {k: v for k, v in zip(["prep", "exact", "leaf", "coarsen", "bases", "-", "couple", "total"],
                                           r["phase"]) if k != "-"},
        # per kernel: device time per product (events, on the launch's stream),
        # algorithmic work per product and the rates they give
        "kernels": {names[i]: {"ms_per_step": r["t_k"][i] / args.steps,
                               "launches_per_step": r["cnt"]["launches_kernel"][i],
                               "units_per_step": r["cnt"]["units_kernel"][i],
                               "gflop_per_step": r["cnt"]["flops_kernel"][i] * 1e-9,
                               "gbyte_per_step": r["cnt"]["bytes_kernel"][i] * 1e-9,
                               "achieved_gbs": r["cnt"]["bytes_kernel"][i] * 1e-9
                               / max(1e-12, r["t_k"][i] / args.steps * 1e-3),
                               "achieved_tflops": r["cnt"]["flops_kernel"][i] * 1e-12
                               / max(1e-12, r["t_k"][i] / args.steps * 1e-3)}
                    for i in range(len(names)) if r["cnt"]["launches_kernel"][i]},
        "headline_mode": head,
        "modes": {name: {"eps": x["eps"], "products_per_s": args.steps / x["total"],
                         "ms_per_step": 1000.0 * x["total"] / args.steps,
                         "precision_used": "fp32_bulk" if x["st"]["prec_used"] == h2.PREC_FP32_BULK else "fp64",
                         "rank_max": [x["st"]["rank_max_row"], x["st"]["rank_max_col"]],
                         "roofline": roofline(names, x, args.steps, args.workload if name == head else None)}
                  for name, x in res.items()},
    }
    if not args.no_global_error:
        say("global error of one product (10 power-iteration steps, untimed)")
        out["global_error"] = global_error(h2, ctx, A, B, int(T.n), eps, st["prec_used"])
    if not args.no_cpu_baseline:
        say("oracle on the host (bounded sample)")
        out["cpu_baseline"] = cpu_baseline(cfg, args.workload)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
