#!/usr/bin/env python3
"""Throughput benchmark of contour-guided demons registration on one MI355X.

One step = one full registration (Algorithm A: pyramid set-up, coarse demons levels,
finest-level CG-DIR loop) of the synthetic workload, through the C-ABI, with the inputs
already resident in HBM.  value = voxel-iterations per second, sum over levels of
(voxels x iterations) / wall time per step.

Also reported on the same JSON line:
  roofline      the dominant kernel (finest-level step or smooth) -- algorithmic bytes per launch
                (bytes per voxel x voxels) over its average launch duration, from HIP
                events on the library's stream during a profiled pass of the same steps;
                traffic = HBM bytes per launch from the rocprofv3 FETCH_SIZE / WRITE_SIZE
                summary in profiles/, when it was taken on the current kernel source.
  cpu_baseline  the FP64 oracle on a bounded sample of the same workload (rank 0 only).
  served        with --serve: open-loop Poisson arrivals, p50/p99 latency.
"""
import argparse
import hashlib
import json
import math
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

# algorithmic bytes per voxel of each finest-level kernel (fields FP32 SoA, mask bit-planes
# one byte per voxel per side).  step (force, fluid smoothing, compose) reads the warped
# image I0~ (4), T0 (4), u (12) and, with contour terms, the stencil structure bits and the
# target bits (1 + 1), and, with the stopping metric, the UROI (1); it writes u_c (12).
# smooth (diffusion smoothing, then the warp of I0) reads u_c (12) and I0 (4, gathered about
# once) and writes u (12), I0~ (4) and, with contour terms, the structure bits (1).  The
# K_i~ values and moving-mask bits near structures are data dependent and left out.
def bytes_per_voxel(kernel, k, metric):
    if kernel == "step":
        return 4 + 4 + 12 + 12 + (2 if k else 0) + (1 if metric else 0)
    if kernel == "smooth":
        return 12 + 4 + 12 + 4 + (1 if k else 0)
    return None


KERNEL_SYMBOL = {"step": "k_step_batch", "smooth": "k_smooth_batch"}

WORKLOADS = {
    "pelvis": ("pelvis-like CT 512x512x128, 8 structures (+15 HU), 3 levels x 150 iterations, "
               "DVF sigma 1", lambda P: P.pelvis_pair()),
    "head_neck": ("head-and-neck-like CT 256x256x128, 5 structures (+10..30 HU), 3 levels x 100 "
                  "iterations, DVF sigma 1.5", lambda P: P.head_neck_pair()),
    "plain": ("nested-ellipsoid phantom 64x64x32, 1 structure, 1 level x 100 iterations",
              lambda P: P.plain_pair()),
    "pelvis_slab": ("one GPU's z-slab of the pelvis-like CT when one volume is split over 8 GPUs: "
                    "512x512x16 plus 4-plane halos (512x512x24), 8 structures, finest level x 150 "
                    "iterations, DVF sigma 1", lambda P: slab_of(P.pelvis_pair(), 16, 4)),
}


def slab_of(pair, planes, halo):
    """The middle z-slab of a pair (planes + halo on each side), finest level only: the shape
    one GPU would hold if the volume were split in z."""
    nz = pair.target.shape[0]
    z0 = max(0, (nz - planes) // 2 - halo)
    z1 = min(nz, z0 + planes + 2 * halo)
    sl = slice(z0, z1)
    pair.target = np.ascontiguousarray(pair.target[sl])
    pair.moving = np.ascontiguousarray(pair.moving[sl])
    pair.target_masks = np.ascontiguousarray(pair.target_masks[:, sl])
    pair.moving_masks = np.ascontiguousarray(pair.moving_masks[:, sl])
    pair.levels = 1
    pair.iters = (pair.iters[0],)
    pair.name = pair.name + "_slab"
    return pair


def copy_peak_gbs(torch, mib=1024, reps=10):
    """Device-to-device copy bandwidth (read + write bytes per second) with HIP events."""
    n = mib << 18
    src = torch.ones(n, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        dst.copy_(src)
    b.record()
    b.synchronize()
    ms = a.elapsed_time(b) / reps
    del src, dst
    return 2 * n * 4 / (ms * 1e-3) / 1e9


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def kernel_source_hash():
    with open(os.path.join(ROOT, "paper_1301_0970_amd", "csrc", "cgdir_kernels.hip"), "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def read_traffic(workload, kernel):
    """HBM bytes per launch from profiles/<kernel>_<workload>_pmc.md, if it was measured on
    the current kernel source (else None)."""
    path = os.path.join(ROOT, "profiles", "%s_%s_pmc.md" % (kernel, workload))
    if not os.path.exists(path):
        return None
    txt = open(path).read()
    m_hash = re.search(r"kernel_source_sha256_16:\s*([0-9a-f]+)", txt)
    m_bytes = re.search(r"hbm_bytes_per_launch:\s*([0-9.eE+]+)", txt)
    if not m_hash or not m_bytes or m_hash.group(1) != kernel_source_hash():
        return None
    return float(m_bytes.group(1))


def cpu_baseline(pair, target_vi=3.0e8):
    """The oracle's Algorithm A on the full-size inputs of the workload, with the same number
    of iterations at every level, as many as make about `target_vi` voxel-iterations (8 for
    the pelvis workload: 10-15 s of work on 16 cores), at most the workload's own count."""
    import oracle
    per_iter, dims = 0, pair.dims
    for _ in range(pair.levels):
        per_iter += dims[0] * dims[1] * dims[2]
        dims = tuple((n + 1) // 2 for n in dims)
    it = max(1, min(max(pair.iters), int(math.ceil(target_vi / per_iter))))
    prm = oracle.params_for(pair, iters=(it,) * pair.levels)
    t0 = time.time()
    oracle.register(pair.target, pair.moving, pair.target_masks, pair.moving_masks, prm)
    dt = time.time() - t0
    vi = 0
    dims = pair.dims
    for _ in range(pair.levels):
        vi += dims[0] * dims[1] * dims[2] * it
        dims = tuple((n + 1) // 2 for n in dims)
    cores = int(os.environ.get("OMP_NUM_THREADS") or os.cpu_count())
    return {"value": vi / dt, "unit": "voxel-iter/s", "cores": cores, "kind": "oracle",
            "sample": "FP64 oracle, Algorithm A on the full %dx%dx%d inputs with %d iterations per "
                      "level (%d levels, %.0f M voxel-iterations, %.1f s)"
                      % (pair.dims + (it, pair.levels, vi / 1e6, dt))}


def served(cgdir, P, torch, duration, rate, pool_bytes, distinct):
    """Open-loop Poisson arrivals; each request registers a pair drawn like the batched
    workload (a pool of `distinct` pre-generated pairs is cycled).  The same arrival schedule
    is replayed twice: with continuous batching (8 slots) and as a serial FIFO (1 slot)."""
    times, specs = P.serve_schedule(rate=rate, duration=duration)
    pool_specs = specs[:distinct]
    pairs = [P.from_spec(s) for s in pool_specs]
    dev = torch.device("cuda")
    items = [(torch.from_numpy(p.target).to(dev), torch.from_numpy(p.moving).to(dev),
              torch.from_numpy(p.target_masks).to(dev), torch.from_numpy(p.moving_masks).to(dev))
             for p in pairs]
    outs = [torch.empty((3,) + p.target.shape, device=dev) for p in pairs]
    prms = [cgdir.params_for_pair(p) for p in pairs]

    def replay(slots):
        lat = []
        with cgdir.Context(pool_bytes, max_slots=slots) as ctx:
            for it, pr, o in zip(items, prms, outs):   # warm-up: tile shapes tuned
                ctx.register(*it, pr, o)
            start = time.time()
            tickets = []
            for i, t in enumerate(times):
                now = time.time() - start
                if t > now:
                    time.sleep(t - now)
                j = i % len(items)
                # requests for the same pair share its output tensor: they carry the same
                # inputs, so whatever overlaps writes the same values
                tickets.append(ctx.submit(*items[j], prms[j], outs[j]))
            for t in tickets:
                rc = ctx.wait(t)
                if rc != cgdir.OK:
                    raise RuntimeError("served request failed: %s" % cgdir.strerror(rc))
            end = time.time()
            for t in tickets:
                st = ctx.poll(t)
                lat.append((st.t_done_ns - st.t_submit_ns) / 1e6)
        lat = np.array(lat)
        return {"slots": slots, "p50_ms": float(np.percentile(lat, 50)),
                "p99_ms": float(np.percentile(lat, 99)),
                "registrations_per_s": len(lat) / (end - start)}

    log("served: continuous batching")
    cont = replay(8)
    log("served: serial FIFO")
    fifo = replay(1)
    return {"requests": len(times), "rate_per_s": rate, "duration_s": duration,
            "distinct_pairs": len(items), "continuous_batching": cont, "serial_fifo": fifo}


def evaluated(cgdir, torch, pair, pool):
    """Section 2.3 metrics on the GPU for the workload registered with CG-DIR, with CG-DIR
    whose contour terms also act at the coarse levels, and with plain demons (contour terms
    off): the comparison the paper makes, on the synthetic pair."""
    dev = torch.device("cuda")
    t = torch.from_numpy(pair.target).to(dev)
    m = torch.from_numpy(pair.moving).to(dev)
    tm = torch.from_numpy(pair.target_masks).to(dev)
    mm = torch.from_numpy(pair.moving_masks).to(dev)
    out = {}
    with cgdir.Context(pool) as ctx:
        for name, mask in (("cg_dir", 1), ("cg_dir_all_levels", (1 << pair.levels) - 1), ("demons", 0)):
            prm = cgdir.params_for_pair(pair, contour_level_mask=mask)
            ctx.register(t, m, tm, mm, prm)             # warm-up (tile shapes)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            u = ctx.register(t, m, tm, mm, prm)
            torch.cuda.synchronize()
            reg_ms = (time.perf_counter() - t0) * 1e3
            ctx.evaluate(t, m, tm, mm, u)               # warm-up
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r = ctx.evaluate(t, m, tm, mm, u)
            ms = (time.perf_counter() - t0) * 1e3
            # one finest-level iteration: (150 iterations - 50 iterations) / 100, set-up cancelled
            fin = []
            for n in (50, 150, 50, 150):
                pf = cgdir.params_for_pair(pair, levels=1, iters=(n,), contour_level_mask=mask & 1)
                torch.cuda.synchronize()
                t1 = time.perf_counter()
                ctx.register(t, m, tm, mm, pf)
                torch.cuda.synchronize()
                fin.append((time.perf_counter() - t1) * 1e3)
            iter_ms = ((fin[1] - fin[0]) + (fin[3] - fin[2])) / 200.0
            st = r["structures"]
            out[name] = {"rms_id": r["whole"]["rms_id"], "cc": r["whole"]["cc"],
                         "rms_id_uroi": r["uroi"]["rms_id"], "cc_uroi": r["uroi"]["cc"],
                         "dsc": [round(x["dsc"], 4) for x in st],
                         "ssd_mean_mm": [round(x["ssd"]["mean"], 3) for x in st],
                         "ssd_p95_mm": [round(x["ssd"]["p95"], 3) for x in st],
                         "register_ms": reg_ms, "evaluate_ms": ms, "finest_iteration_ms": iter_ms}
        # before registration
        z = torch.zeros((3,) + tuple(pair.target.shape), device=dev)
        r = ctx.evaluate(t, m, tm, mm, z)
        out["unregistered"] = {"rms_id": r["whole"]["rms_id"], "cc": r["whole"]["cc"],
                               "rms_id_uroi": r["uroi"]["rms_id"], "cc_uroi": r["uroi"]["cc"],
                               "dsc": [round(x["dsc"], 4) for x in r["structures"]]}
    return out


def cold_start(cgdir, torch, pair, pool):
    """The first registration in a fresh context: with its tile shapes still to be tuned (the
    first launches of each group try candidate shapes), and with the groups imported from an
    earlier context's cgdir_tuning_export."""
    dev = torch.device("cuda")
    t = torch.from_numpy(pair.target).to(dev)
    m = torch.from_numpy(pair.moving).to(dev)
    tm = torch.from_numpy(pair.target_masks).to(dev)
    mm = torch.from_numpy(pair.moving_masks).to(dev)
    prm = cgdir.params_for_pair(pair)

    def first(text=None):
        with cgdir.Context(pool) as ctx:
            if text is not None:
                ctx.tuning_import(text)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ctx.register(t, m, tm, mm, prm)
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t0) * 1e3
            return ms, ctx.tuning_export()
    _, text = first()                                   # tunes; module loads happen here
    untuned, _ = first()
    imported, _ = first(text)
    return {"untuned_first_ms": untuned, "imported_first_ms": imported,
            "groups": len([l for l in text.splitlines() if l])}


def warm_start(cgdir, torch, pair, pool, iters=30):
    """Re-registration from an existing field (finest level only, no coarse demons) against
    the full pyramid: latency and the resulting overlap (device evaluation)."""
    dev = torch.device("cuda")
    t = torch.from_numpy(pair.target).to(dev)
    m = torch.from_numpy(pair.moving).to(dev)
    tm = torch.from_numpy(pair.target_masks).to(dev)
    mm = torch.from_numpy(pair.moving_masks).to(dev)
    out = {}
    with cgdir.Context(pool) as ctx:
        full = cgdir.params_for_pair(pair)
        ctx.register(t, m, tm, mm, full)                           # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        u = ctx.register(t, m, tm, mm, full)
        torch.cuda.synchronize()
        out["full_ms"] = (time.perf_counter() - t0) * 1e3
        out["full_dsc_mean"] = float(np.mean([s["dsc"] for s in ctx.evaluate(t, m, tm, mm, u)["structures"]]))
        # the previous field as the start of a finest-level-only run (e.g. the next fraction)
        warm = cgdir.params_for_pair(pair, levels=1, iters=(iters,))
        ctx.register(t, m, tm, mm, warm, initial=u)                # warm-up of the tile shapes
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        uw = ctx.register(t, m, tm, mm, warm, initial=u)
        torch.cuda.synchronize()
        out["warm_ms"] = (time.perf_counter() - t0) * 1e3
        out["warm_iters"] = iters
        out["warm_dsc_mean"] = float(np.mean([s["dsc"] for s in ctx.evaluate(t, m, tm, mm, uw)["structures"]]))
    return out


def batched(cgdir, P, torch, n_pairs):
    """The uneven batch (sizes and structure counts drawn per pair): all pairs in one
    cgdir_register_batch call vs the same pairs registered one at a time, both timed after a
    pass of each that lets the autotuner settle every tile-shape group they use."""
    specs = P.batch_specs(n_pairs)
    pairs = [P.from_spec(s) for s in specs]
    dev = torch.device("cuda")
    items = [(torch.from_numpy(p.target).to(dev), torch.from_numpy(p.moving).to(dev),
              torch.from_numpy(p.target_masks).to(dev), torch.from_numpy(p.moving_masks).to(dev))
             for p in pairs]
    prms = [cgdir.params_for_pair(p) for p in pairs]
    outs = [torch.empty((3,) + p.target.shape, device=dev) for p in pairs]
    vi = sum(p.voxel_iterations() for p in pairs)
    pool = sum(cgdir.footprint(*p.dims, p.k, pr) for p, pr in zip(pairs, prms)) + (256 << 20)
    with cgdir.Context(pool) as ctx:
        for it, pr, o in zip(items, prms, outs):        # warm-up: tile shapes of every pair
            ctx.register(*it, pr, o)
        ctx.register_batch(items, prms, outs)           # and of every batched launch group
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for it, pr, o in zip(items, prms, outs):
            ctx.register(*it, pr, o)
        torch.cuda.synchronize()
        serial = time.perf_counter() - t0
        time.sleep(0.05)   # an idle gap that marks the timed batched run in a kernel trace
        t0 = time.perf_counter()
        rc, st = ctx.register_batch(items, prms, outs)
        torch.cuda.synchronize()
        batch = time.perf_counter() - t0
        if rc != cgdir.OK:
            raise RuntimeError("batch failed: %s" % cgdir.strerror(rc))
    return {"pairs": n_pairs, "voxel_iterations": vi,
            "batched_value": vi / batch, "batched_ms": batch * 1e3,
            "one_at_a_time_value": vi / serial, "one_at_a_time_ms": serial * 1e3,
            "speedup": serial / batch, "unit": "voxel-iter/s",
            "sizes": [list(p.dims) for p in pairs], "structures": [p.k for p in pairs]}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="pelvis", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--serve", action="store_true", help="also run the served workload")
    ap.add_argument("--batch", type=int, default=0, metavar="PAIRS",
                    help="also run the uneven batched workload with this many pairs (32 in full)")
    ap.add_argument("--serve-seconds", type=float, default=30.0)
    ap.add_argument("--warm-start", action="store_true",
                    help="also time a finest-level re-registration started from the full result")
    ap.add_argument("--cold-start", action="store_true",
                    help="also time the first registration of a fresh context, untuned and with imported tile shapes")
    ap.add_argument("--evaluate", action="store_true",
                    help="also evaluate (section 2.3 metrics) CG-DIR, CG-DIR with contour terms at every level and plain demons on the workload")
    ap.add_argument("--serve-rate", type=float, default=4.0, help="Poisson arrivals per second")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run 5 plain device copies of MIB MiB (calibrates HBM byte counters)")
    args = ap.parse_args()

    if args.gpus != 1:
        print("bench.py measures one GPU only: registration pairs shard across GPUs with no "
              "exchange, so there is no multi-GPU path to time (asked for --gpus %d)" % args.gpus,
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1301_0970_amd import cgdir, phantom as P

    if args.copy_probe:
        n = args.copy_probe << 18   # float32 elements
        src = torch.ones(n, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes_read": n * 4, "copy_probe_bytes_written": n * 4}))
        return

    desc, make = WORKLOADS[args.workload]
    log("generating %s" % args.workload)
    pair = make(P)
    dev = torch.device("cuda", 0)
    t = torch.from_numpy(pair.target).to(dev)
    m = torch.from_numpy(pair.moving).to(dev)
    tm = torch.from_numpy(pair.target_masks).to(dev)
    mm = torch.from_numpy(pair.moving_masks).to(dev)
    prm = cgdir.params_for_pair(pair)
    out = torch.empty((3,) + pair.target.shape, device=dev)
    pool = cgdir.footprint(*pair.dims, pair.k, prm) + (64 << 20)
    vi = pair.voxel_iterations()

    with cgdir.Context(pool) as ctx:
        for i in range(args.warmup):
            log("warmup %d" % i)
            ctx.register(t, m, tm, mm, prm, out)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(args.steps):
            ctx.register(t, m, tm, mm, prm, out)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / args.steps
        log("timed %d steps: %.2f ms/step" % (args.steps, dt * 1e3))

    # profiled pass of the same steps: per-kernel HIP events on the library's stream
    with cgdir.Context(pool, profile=True) as ctx:
        ctx.register(t, m, tm, mm, prm, out)
        ctx.kernel_stats(reset=True)
        for i in range(args.steps):
            ctx.register(t, m, tm, mm, prm, out)
        torch.cuda.synchronize()
        stats = ctx.kernel_stats()
    finest = {s["name"].split("@")[0]: s for s in stats if s["name"].endswith("@L0")}
    dom = max((n for n in finest if n in KERNEL_SYMBOL), key=lambda n: finest[n]["total_ms"])
    s = finest[dom]
    bpv = bytes_per_voxel(dom, pair.k, prm.stop_mode != 0)
    per_launch_bytes = bpv * s["voxels"] / s["launches"]
    avg_ms = s["total_ms"] / s["launches"]
    achieved = per_launch_bytes / (avg_ms * 1e-3) / 1e9
    traffic = read_traffic(args.workload, dom)
    log("copy probe")
    copy_gbs = copy_peak_gbs(torch)
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "copy_measured_gbs": round(copy_gbs, 1),
                "kernel": "%s (%s), finest level" % (dom, KERNEL_SYMBOL[dom]),
                "avg_launch_ms": round(avg_ms, 5), "algorithmic_bytes_per_launch": per_launch_bytes,
                "bytes_per_voxel": bpv}
    per_kernel = {x["name"]: {"launches": x["launches"], "avg_ms": round(x["total_ms"] / x["launches"], 5)}
                  for x in stats}

    result = {
        "metric": "voxel-iterations/s + HBM GB/s vs roofline; served p50/p99 latency per registration",
        "value": vi / dt,
        "unit": "voxel-iter/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded phantom standing in for clinical CT)",
        "config": {"workload": desc, "dims": list(pair.dims), "structures": pair.k,
                   "levels": pair.levels, "iters": list(pair.iters), "voxel_iterations": vi},
        "roofline": roofline,
        "kernels": per_kernel,
    }
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        result["cpu_baseline"] = cpu_baseline(pair)
    if args.warm_start:
        log("warm start")
        result["warm_start"] = warm_start(cgdir, torch, pair, pool + (1 << 30))
    if args.cold_start:
        log("cold start")
        result["cold_start"] = cold_start(cgdir, torch, pair, pool + (1 << 30))
    if args.evaluate:
        log("evaluation")
        result["evaluation"] = evaluated(cgdir, torch, pair, pool + (1 << 30))
    if args.batch:
        log("batched workload")
        result["batched"] = batched(cgdir, P, torch, args.batch)
    if args.serve:
        log("served workload")
        result["served"] = served(cgdir, P, torch, args.serve_seconds, args.serve_rate,
                                  32 << 30, 16)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
