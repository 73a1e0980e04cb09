#!/usr/bin/env python3
"""Throughput benchmark of contour-guided demons registration on one MI355X.

One step = one full registration (Algorithm A: pyramid set-up, coarse demons levels,
finest-level CG-DIR loop) of the pelvis workload, through the C-ABI, with the inputs
already resident in HBM.  value = voxel-iterations per second, sum over levels of
(voxels x iterations) / wall time per step.

Also reported on the same JSON line:
  roofline      the finest-level iteration (the step launch plus the smoothing launch):
                algorithmic bytes of one iteration (u read and written, I0, T0, the mask
                bit-planes: 34 B per voxel with contour terms) over the summed average
                launch durations, from HIP events on the library's stream during a
                profiled pass of the same steps, against 8 TB/s; per-kernel shares of those
                bytes; the HBM bytes the counters measured (rocprofv3 FETCH_SIZE /
                WRITE_SIZE) and the VALU instructions (SQ_INSTS_VALU) per launch, read from
                the summaries in profiles/ when they were taken on the current kernel
                source; the VALU-issue ceiling those instructions imply; `bound` is the
                resource closer to its ceiling.
  cpu_baseline  the FP64 oracle on a bounded sample of the same workload, on all the host
                threads it is given and on one thread (rank 0 only).
  batched       the uneven batch of 32 pairs in one call against the same pairs one at a time.
  served        Poisson arrivals at 4 requests/s for 120 s (pairs drawn like the batch),
                continuous batching against a serial FIFO on the same schedule, and both again
                at 1.1 times the serial FIFO's capacity (the mean service time of the pairs
                alone).
"""
import argparse
import hashlib
import json
import math
import os
import re
import subprocess
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# VALU issue of MI355X without packed FP32: 256 compute units, each issuing one wave64 vector
# instruction per clock (four SIMDs of 16 lanes, four clocks per wave64 instruction), 2.4 GHz
VALU_WAVE_INSTS_PER_S = 256 * 2.4e9
VALU_LANE_OPS_PEAK = VALU_WAVE_INSTS_PER_S * 64


# Algorithmic bytes per voxel of one finest-level iteration (fields FP32 SoA, one mask
# bit-plane byte per voxel per side): u read and written (12 + 12), I0 (4, gathered about
# once: u is smooth), T0 (4), the moving and target bit-planes (1 + 1) with contour terms,
# the UROI (1) with the stopping metric.  Everything else the design moves (the composite
# update u_c, the warped image and its structure bits, K~) is a design intermediate.
def iteration_bytes_per_voxel(k, metric):
    return 32 + (2 if k else 0) + (1 if metric else 0)


# The same bytes split by kernel: the step kernel reads u, T0 and the bit-planes; the
# smoothing kernel gathers I0 and writes u.
def kernel_bytes_per_voxel(kernel, k, metric):
    if kernel == "step":
        return 12 + 4 + (2 if k else 0) + (1 if metric else 0)
    return 4 + 12


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


def _pair_from_spec(spec):
    from paper_1301_0970_amd import phantom as P
    return P.from_spec(spec)


def generate(specs, workers):
    """The pairs of a list of specs, drawn in parallel worker processes (numpy only; started
    before this process touches the GPU)."""
    if workers <= 1 or len(specs) <= 1:
        out = []
        for i, s in enumerate(specs):
            out.append(_pair_from_spec(s))
            log("  pair %d of %d" % (i + 1, len(specs)))
        return out
    import multiprocessing as mp
    with mp.get_context("spawn").Pool(min(workers, len(specs))) as pool:
        return pool.map(_pair_from_spec, specs, chunksize=1)


def host_threads():
    """Threads the oracle's OpenMP runtime uses (OMP_NUM_THREADS, else the CPUs this process
    may run on)."""
    env = os.environ.get("OMP_NUM_THREADS")
    if env and env.split(",")[0].isdigit():
        return int(env.split(",")[0])
    return len(os.sched_getaffinity(0))


def cpu_model():
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
    except Exception:
        return None
    info = {}
    for line in out.splitlines():
        if ":" in line:
            key, v = line.split(":", 1)
            info[key.strip()] = v.strip()
    return {"model": info.get("Model name"), "cpus": info.get("CPU(s)"),
            "sockets": info.get("Socket(s)"), "threads_per_core": info.get("Thread(s) per core")}


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


_START = time.time()


def log(msg):
    print("[%6.1f s] %s" % (time.time() - _START, msg), file=sys.stderr, flush=True)


def kernel_source_hash():
    """sha256 (16 hex digits) of the kernel sources with their comments and runs of blank space
    removed: the counter summaries under profiles/ stay attached to the code they measured when
    only a comment changes, and are set aside when the code does."""
    h = hashlib.sha256()
    for name in ("cgdir_kernels.hip", "cgdir_internal.h"):
        with open(os.path.join(ROOT, "paper_1301_0970_amd", "csrc", name)) as f:
            src = f.read()
        src = re.sub(r"/\*.*?\*/", " ", re.sub(r"//[^\n]*", " ", src), flags=re.S)
        h.update(re.sub(r"\s+", " ", src).strip().encode())
    return h.hexdigest()[:16]


def read_profile(workload, what):
    """Key/value lines `<name>: <number>` of profiles/iteration_<workload>_<what>.md when the
    summary was taken on the current kernel source (else None)."""
    path = os.path.join(ROOT, "profiles", "iteration_%s_%s.md" % (workload, what))
    if not os.path.exists(path):
        return None
    txt = open(path).read()
    m_hash = re.search(r"kernel_source_sha256_16:\s*([0-9a-f]+)", txt)
    if not m_hash or m_hash.group(1) != kernel_source_hash():
        return None
    return {m.group(1): float(m.group(2))
            for m in re.finditer(r"^([a-z_]+):\s*([-0-9.eE+]+)\s*$", txt, re.M)}


def roofline(stats, pair, metric, workload, copy_gbs):
    """The finest-level iteration against HBM bandwidth and VALU issue."""
    fin = {s["name"].split("@")[0]: s for s in stats if s["name"].endswith("@L0")}
    st, sm = fin["step"], fin["smooth"]
    n = st["voxels"] / st["launches"]
    t_step = st["total_ms"] / st["launches"]
    t_smooth = sm["total_ms"] / sm["launches"]
    t_iter = t_step + t_smooth
    bpv = iteration_bytes_per_voxel(pair.k, metric)
    alg = bpv * n
    achieved = alg / (t_iter * 1e-3) / 1e9
    out = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
           "kernel": "finest-level iteration: k_step_batch + k_smooth_batch (%d voxels)" % n,
           "bytes_per_voxel": bpv, "algorithmic_bytes_per_iteration": alg,
           "iteration_ms": round(t_iter, 5), "copy_measured_gbs": round(copy_gbs, 1)}
    per = {}
    for name, s, t in (("step", st, t_step), ("smooth", sm, t_smooth)):
        b = kernel_bytes_per_voxel(name, pair.k, metric) * n
        per[name] = {"avg_launch_ms": round(t, 5), "algorithmic_bytes": b,
                     "frac": round(b / (t * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
    hbm = read_profile(workload, "hbm")
    if hbm:
        traffic = hbm["step_hbm_bytes_per_launch"] + hbm["smooth_hbm_bytes_per_launch"]
        out["traffic"] = traffic
        out["traffic_over_algorithmic"] = round(traffic / alg, 3)
        out["measured_gbs"] = round(traffic / (t_iter * 1e-3) / 1e9, 1)
        for name in per:
            per[name]["hbm_bytes"] = hbm[name + "_hbm_bytes_per_launch"]
    sq = read_profile(workload, "valu")
    busy_hbm = (out["measured_gbs"] / copy_gbs) if hbm else None
    if sq:
        insts = sq["step_valu_insts_per_launch"] + sq["smooth_valu_insts_per_launch"]
        ceiling_ms = insts / VALU_WAVE_INSTS_PER_S * 1e3
        out["valu"] = {"wave_insts_per_iteration": insts,
                       "insts_per_voxel": round(64 * insts / n, 1),
                       "ceiling_ms": round(ceiling_ms, 5),
                       "achieved_lane_ops": round(64 * insts / (t_iter * 1e-3) / 1e12, 2),
                       "peak_lane_ops": round(VALU_LANE_OPS_PEAK / 1e12, 2),
                       "unit": "T lane-instructions/s",
                       "frac": round(ceiling_ms / t_iter, 4)}
        for name in per:
            v = sq[name + "_valu_insts_per_launch"]
            per[name]["valu_insts_per_voxel"] = round(64 * v / n, 1)
        if busy_hbm is None or out["valu"]["frac"] > busy_hbm:
            out["bound"] = "alu"
    out["bound_evidence"] = ("VALU issue %s of its ceiling, HBM traffic %s of the copy-measured rate"
                             % ("%.2f" % out["valu"]["frac"] if sq else "unmeasured",
                                "%.2f" % busy_hbm if busy_hbm is not None else "unmeasured"))
    if sq and "step_wait_any_over_wave_cycles" in sq:
        # neither near its ceiling: the waves wait (memory and LDS latency, barriers)
        out["wave_cycles_waiting"] = {name: round(sq[name + "_wait_any_over_wave_cycles"], 3) for name in per}
        out["bound_evidence"] += ("; waves waiting %.2f (step) and %.2f (smooth) of their cycles"
                                  % (out["wave_cycles_waiting"]["step"], out["wave_cycles_waiting"]["smooth"]))
    out["kernels"] = per
    return out


def cpu_baseline(pair, target_vi=3.0e8, one_thread_vi=4.0e7):
    """The oracle's Algorithm A on the full-size inputs of the workload, with the same number
    of iterations at every level: as many as make about `target_vi` voxel-iterations on all
    the host threads it is given (8 for the pelvis workload), and one iteration per level on
    one thread."""
    import ctypes
    import oracle
    per_iter, dims = 0, pair.dims
    for _ in range(pair.levels):
        per_iter += dims[0] * dims[1] * dims[2]
        dims = tuple((n + 1) // 2 for n in dims)

    def run(it):
        prm = oracle.params_for(pair, iters=(it,) * pair.levels)
        t0 = time.time()
        oracle.register(pair.target, pair.moving, pair.target_masks, pair.moving_masks, prm)
        return per_iter * it / (time.time() - t0), time.time() - t0

    it = max(1, min(max(pair.iters), int(math.ceil(target_vi / per_iter))))
    cores = host_threads()
    value, dt = run(it)
    res = {"value": value, "unit": "voxel-iter/s", "cores": cores, "kind": "oracle",
           "sample": "FP64 oracle, Algorithm A on the full %dx%dx%d inputs with %d iterations per "
                     "level (%d levels, %.0f M voxel-iterations, %.1f s on %d threads)"
                     % (pair.dims + (it, pair.levels, per_iter * it / 1e6, dt, cores)),
           "host": cpu_model()}
    # one thread: the OpenMP runtime the oracle links, asked for one thread for this call
    gomp = ctypes.CDLL("libgomp.so.1")
    gomp.omp_set_num_threads(1)
    try:
        it1 = max(1, int(round(one_thread_vi / per_iter)))
        v1, dt1 = run(it1)
    finally:
        gomp.omp_set_num_threads(cores)
    res["one_thread"] = {"value": v1, "unit": "voxel-iter/s", "cores": 1,
                         "sample": "%d iteration(s) per level, %.0f M voxel-iterations, %.1f s"
                                   % (it1, per_iter * it1 / 1e6, dt1)}
    return res


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


def batched(cgdir, torch, pairs, repeats=3):
    """The uneven batch (sizes and structure counts drawn per pair): all pairs in one
    cgdir_register_batch call vs the same pairs registered one at a time, both timed after a
    pass of each that lets the autotuner settle every tile-shape group they use, then timed
    `repeats` times in alternation; the medians are reported (one timing of the batch varies by
    a few per cent from the next)."""
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
        serials, batches = [], []
        for _ in range(repeats):
            time.sleep(0.05)   # idle gaps that mark each timed run (serial, then batched) in a trace
            t0 = time.perf_counter()
            for it, pr, o in zip(items, prms, outs):
                ctx.register(*it, pr, o)
            torch.cuda.synchronize()
            serials.append(time.perf_counter() - t0)
            time.sleep(0.05)
            t0 = time.perf_counter()
            rc, st = ctx.register_batch(items, prms, outs)
            torch.cuda.synchronize()
            batches.append(time.perf_counter() - t0)
            if rc != cgdir.OK:
                raise RuntimeError("batch failed: %s" % cgdir.strerror(rc))
    serial, batch = float(np.median(serials)), float(np.median(batches))
    return {"pairs": len(pairs), "voxel_iterations": vi, "repeats": repeats,
            "batched_value": vi / batch, "batched_ms": batch * 1e3,
            "one_at_a_time_value": vi / serial, "one_at_a_time_ms": serial * 1e3,
            "speedup": serial / batch, "unit": "voxel-iter/s",
            "batched_ms_each": [round(t * 1e3, 1) for t in batches],
            "one_at_a_time_ms_each": [round(t * 1e3, 1) for t in serials],
            "sizes": [list(p.dims) for p in pairs], "structures": [p.k for p in pairs]}


def stage(torch, pairs):
    dev = torch.device("cuda")
    items = [(torch.from_numpy(p.target).to(dev), torch.from_numpy(p.moving).to(dev),
              torch.from_numpy(p.target_masks).to(dev), torch.from_numpy(p.moving_masks).to(dev))
             for p in pairs]
    outs = [torch.empty((3,) + p.target.shape, device=dev) for p in pairs]
    return items, outs


def served(cgdir, torch, staged, prms, times, slots, pool_bytes):
    """Open-loop arrivals at `times` (seconds); request i registers pair i % len(pairs) (inputs
    and outputs device-resident).  Latency = completion - submission (steady clock)."""
    items, outs = staged
    with cgdir.Context(pool_bytes, max_slots=slots) as ctx:
        for it, pr, o in zip(items, prms, outs):   # warm-up: tile shapes tuned
            ctx.register(*it, pr, o)
        torch.cuda.synchronize()
        start = time.time()
        tickets = []
        for i, t in enumerate(times):
            now = time.time() - start
            if t > now:
                time.sleep(t - now)
            j = i % len(items)
            # requests for the same pair share its output tensor: they carry the same inputs,
            # so whatever overlaps writes the same values
            tickets.append(ctx.submit(*items[j], prms[j], outs[j]))
        for t in tickets:
            rc = ctx.wait(t)
            if rc != cgdir.OK:
                raise RuntimeError("served request failed: %s" % cgdir.strerror(rc))
        sts = [ctx.poll(t) for t in tickets]
    lat = np.array([(s.t_done_ns - s.t_submit_ns) / 1e6 for s in sts])
    wait = np.array([(s.t_admit_ns - s.t_submit_ns) / 1e6 for s in sts])
    first = min(s.t_submit_ns for s in sts)
    last = max(s.t_done_ns for s in sts)
    # the most requests running at once (admitted, not yet done)
    ev = sorted([(s.t_admit_ns, 1) for s in sts] + [(s.t_done_ns, -1) for s in sts])
    run = peak = 0
    for _, d in ev:
        run += d
        peak = max(peak, run)
    return {"slots": slots, "p50_ms": round(float(np.percentile(lat, 50)), 2),
            "p99_ms": round(float(np.percentile(lat, 99)), 2),
            "mean_ms": round(float(lat.mean()), 2),
            "queue_wait_p99_ms": round(float(np.percentile(wait, 99)), 2),
            "registrations_per_s": round(len(sts) / ((last - first) / 1e9), 3),
            "max_co_resident": peak}


def service_times(cgdir, torch, staged, prms):
    """Each distinct pair registered alone (after a tuning pass): milliseconds."""
    items, outs = staged
    ms = []
    with cgdir.Context(24 << 30) as ctx:
        for it, pr, o in zip(items, prms, outs):
            ctx.register(*it, pr, o)
        for it, pr, o in zip(items, prms, outs):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ctx.register(*it, pr, o)
            torch.cuda.synchronize()
            ms.append((time.perf_counter() - t0) * 1e3)
    return ms


def serving(cgdir, P, torch, pairs, rate, duration, high_seconds):
    times, _ = P.serve_schedule(rate=rate, duration=duration)
    pool = 24 << 30
    staged = stage(torch, pairs)
    prms = [cgdir.params_for_pair(p) for p in pairs]
    log("served: %d requests at %.1f/s, continuous batching" % (len(times), rate))
    cont = served(cgdir, torch, staged, prms, times, 8, pool)
    log("served: serial FIFO")
    fifo = served(cgdir, torch, staged, prms, times, 1, pool)
    out = {"requests": len(times), "rate_per_s": rate, "duration_s": duration,
           "distinct_pairs": len(pairs), "continuous_batching": cont, "serial_fifo": fifo}
    if high_seconds > 0:
        # above the serial FIFO's capacity: the mean service time of the cycled pairs alone
        ms = service_times(cgdir, torch, staged, prms)
        cap_fifo = 1e3 / float(np.mean(ms))
        hi = 1.1 * cap_fifo
        t_hi, _ = P.serve_schedule(rate=hi, duration=high_seconds)
        log("served: %d requests at %.1f/s, continuous batching" % (len(t_hi), hi))
        c2 = served(cgdir, torch, staged, prms, t_hi, 8, pool)
        log("served: serial FIFO")
        f2 = served(cgdir, torch, staged, prms, t_hi, 1, pool)
        out["above_fifo_capacity"] = {"rate_per_s": round(hi, 2), "duration_s": high_seconds,
                                      "requests": len(t_hi), "mean_service_ms": round(float(np.mean(ms)), 2),
                                      "capacity_fifo_per_s": round(cap_fifo, 2),
                                      "continuous_batching": c2, "serial_fifo": f2}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="pelvis", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--batch", type=int, default=32, metavar="PAIRS",
                    help="pairs of the uneven batched workload (0: skip it)")
    ap.add_argument("--batch-repeats", type=int, default=3,
                    help="timed repeats of the batched and the one-at-a-time runs (medians reported)")
    ap.add_argument("--serve-seconds", type=float, default=120.0,
                    help="duration of the served workload's arrivals (0: skip serving)")
    ap.add_argument("--serve-rate", type=float, default=4.0, help="Poisson arrivals per second")
    ap.add_argument("--serve-distinct", type=int, default=32,
                    help="distinct pairs the served requests cycle through")
    ap.add_argument("--serve-high-seconds", type=float, default=30.0,
                    help="duration of the run above the serial FIFO's capacity (0: skip it)")
    ap.add_argument("--warm-start", action="store_true",
                    help="also time a finest-level re-registration started from the full result")
    ap.add_argument("--cold-start", action="store_true",
                    help="also time the first registration of a fresh context, untuned and with imported tile shapes")
    ap.add_argument("--evaluate", action="store_true",
                    help="also evaluate (section 2.3 metrics) CG-DIR, CG-DIR with contour terms at every level and plain demons on the workload")
    ap.add_argument("--gen-workers", type=int, default=16,
                    help="worker processes that draw the batched and served pairs (1: in this process, "
                         "e.g. under a profiler that would also load itself into every worker)")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run 5 plain device copies of MIB MiB (calibrates HBM byte counters)")
    args = ap.parse_args()

    if args.gpus != 1:
        print("bench.py measures one GPU only: registration pairs shard across GPUs with no "
              "exchange, so there is no multi-GPU path to time (asked for --gpus %d)" % args.gpus,
              file=sys.stderr)
        sys.exit(2)

    from paper_1301_0970_amd import phantom as P

    if args.copy_probe:
        import torch
        n = args.copy_probe << 18   # float32 elements
        src = torch.ones(n, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes_read": n * 4, "copy_probe_bytes_written": n * 4}))
        return

    # every input is drawn before this process touches the GPU (worker processes)
    desc, make = WORKLOADS[args.workload]
    log("generating %s" % args.workload)
    pair = make(P)
    workers = max(1, min(args.gen_workers, len(os.sched_getaffinity(0))))
    batch_pairs, serve_pairs = [], []
    if args.batch:
        log("generating the uneven batch (%d pairs)" % args.batch)
        batch_pairs = generate(P.batch_specs(args.batch), workers)
    if args.serve_seconds > 0:
        _, specs = P.serve_schedule(rate=args.serve_rate, duration=args.serve_seconds)
        log("generating %d distinct served pairs" % min(args.serve_distinct, len(specs)))
        serve_pairs = generate(specs[:args.serve_distinct], workers)

    import torch
    from paper_1301_0970_amd import cgdir

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
    log("copy probe")
    copy_gbs = copy_peak_gbs(torch)
    roof = roofline(stats, pair, prm.stop_mode != 0, args.workload, copy_gbs)
    per_kernel = {x["name"]: {"launches": x["launches"], "avg_ms": round(x["total_ms"] / x["launches"], 5)}
                  for x in stats}
    del t, m, tm, mm, out

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
        "roofline": roof,
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
    if batch_pairs:
        log("batched workload")
        result["batched"] = batched(cgdir, torch, batch_pairs, args.batch_repeats)
    if serve_pairs:
        log("served workload")
        result["served"] = serving(cgdir, P, torch, serve_pairs, args.serve_rate, args.serve_seconds,
                                   args.serve_high_seconds)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
