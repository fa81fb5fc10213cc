"""Insertion benchmark on one MI355X.

A step is one insertion pass of the whole hot path (expand, sample, allocate,
store) over one batch.  The headline workload is the aerial-LiDAR-shaped
cloud: 100M points on a 1 km x 1 km fBm heightfield, 1M-point batches cut
from Morton order and shuffled (seed 1), root cube [0, 1024)^3 m, T = 50,000,
128^3 grids, Dmax = 16, chunks of 1,000.  The whole cloud is resident in HBM
before timing starts; W warmup batches go into a scratch build that is then
reset, and the timed region inserts batches 0..K-1 into an empty octree.

Printed JSON line: points/s over the timed region, ms per step (= per 1M-point
update), p50/p99 per-update latency from HIP events, two rooflines against the
8 TB/s HBM peak -- the dominant kernel's (algorithmic bytes per launch / its
event-timed average duration) and the whole pass's (algorithmic bytes the
insertion must move / wall-clock time of the timed region) -- the CPU oracle
(sequential C inserter, one thread) timed on a bounded prefix of the same
workload with the host's CPU model and core count, and, unless --no-extras,
the same measurement on the 1B-point dense-scan workload (10M-point batches)
and on the aerial cloud in plain Morton order and in fully random order.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

# Every workload uses the paper's octree parameters (T = 50,000, 128^3 grids,
# chunks of 1,000) and Dmax = 16; the capacities are the launch configuration
# the benchmark (and the full-size parity tests) run.
WORKLOADS = {
    "aerial": dict(
        desc="aerial-LiDAR-shaped heightfield, 100M points, 1M-point batches, Morton-shuffled",
        points=100_000_000, batch=1_000_000, root_min=(0.0, 0.0, 0.0), root_size=1024.0,
        caps=dict(max_nodes=1 << 20, arena_bytes=24 << 30, spill_capacity=16 << 20,
                  backlog_capacity=10_000_000)),
    "dense": dict(
        desc="dense-scan-shaped building, 1B points on 2,000 primitives with Gaussian "
             "hotspots, 10M-point batches in scan order",
        points=1_000_000_000, batch=10_000_000, root_min=(0.0, 0.0, 0.0), root_size=64.0,
        caps=dict(max_nodes=1 << 21, arena_bytes=96 << 30, spill_capacity=64 << 20,
                  backlog_capacity=40_000_000, hist_capacity=1 << 15)),
    "planes": dict(
        desc="3 planes + 5% noise in the unit cube, 1M points, 100k-point batches",
        points=1_000_000, batch=100_000, root_min=(0.0, 0.0, 0.0), root_size=1.0,
        caps=dict(max_nodes=1 << 16, arena_bytes=2 << 30, spill_capacity=1 << 20,
                  backlog_capacity=1 << 20)),
}


def octree_config(name):
    """simlod config of a workload's launch configuration."""
    from paper_2310_03567_amd import simlod

    w = WORKLOADS[name]
    return simlod.make_config(root_min=w["root_min"], root_size=w["root_size"],
                              max_batch=w["batch"], **w["caps"])

# Algorithmic bytes of k_sample_store per work item: read the 16-byte record,
# write the 16-byte record and its 4-byte key into the leaf chunk; a spilled
# item also reads its 4-byte key.
SAMPLE_STORE_BYTES_PER_ITEM = 36
SAMPLE_STORE_BYTES_PER_SPILLED = 4


TRAFFIC_SUMMARY = os.path.join(ROOT, "profiles", "k_sample_store_{}_hbm_traffic.txt")
# the device code: the kernels and the headers they inline
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2310_03567_amd", "csrc", f)
                  for f in ("kernels.hip", "octree_device.hpp", "launch.hpp")]
BUILD_SCRIPT = os.path.join(ROOT, "paper_2310_03567_amd", "build.py")  # compiler flags


def kernels_sha256():
    """SHA-256 over the device sources (name and contents of each, in order)."""
    import hashlib

    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(os.path.basename(f).encode() + b"\0")
        h.update(open(f, "rb").read())
    return h.hexdigest()


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def measured_traffic(name):
    """HBM bytes per k_sample_store launch on workload ``name`` from the
    committed rocprofv3 summary (FETCH_SIZE + WRITE_SIZE scaled by a plain
    copy), or None when the summary was taken on a different kernel source
    or with other compiler flags."""
    import hashlib

    try:
        text = open(TRAFFIC_SUMMARY.format(name)).read()
    except OSError:
        return None
    fields = dict(l.split(":", 1) for l in text.splitlines() if ":" in l and not l.startswith(" "))
    want = kernels_sha256()
    flags = hashlib.sha256(open(BUILD_SCRIPT, "rb").read()).hexdigest()
    if (fields.get("kernels_sha256", "").strip() != want
            or fields.get("build_sha256", "").strip() != flags):
        return None
    try:
        return float(fields["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def generate(name, n=None, order=None):
    import pointgen

    w = WORKLOADS[name]
    n = w["points"] if n is None else n
    if name == "aerial":
        return pointgen.aerial(n, seed=1, order=order or "morton_shuffled", batch=w["batch"])
    if name == "dense":
        return pointgen.dense_scan(n, seed=2)
    return pointgen.tiny_planes(n, seed=0)


def cloud_config(cloud, batch):
    """Launch configuration of one cloud of the batched workload, sized to it."""
    from paper_2310_03567_amd import simlod

    n = len(cloud["points"])
    return simlod.make_config(
        root_min=cloud["root_min"], root_size=cloud["root_size"], max_batch=batch,
        max_nodes=int(min(1 << 21, n // 2000 + 8192)),
        arena_bytes=int(48 * n + (n // 20_000) * (256 << 10) + (128 << 20)),
        spill_capacity=int(max(1 << 20, 4 * batch)), backlog_capacity=int(max(1 << 20, 2 * batch)),
        hist_capacity=int(min(8192, max(256, n // 20_000))))


def run_batched(args):
    """64 independent clouds of uneven size (log-uniform 100k..50M points,
    aerial heightfields and dense building scans), each cut into 10 batches;
    step s inserts batch s of every cloud.  The group form inserts a step in
    one pass over all clouds (autotuned launch shape, replayed hipGraph);
    the plain form inserts each cloud's batch with its own call, in turn, on
    the same stream.  Both start from empty octrees and insert the same
    points; the octrees must come out identical."""
    import torch

    import pointgen
    from paper_2310_03567_amd import simlod

    t0 = time.perf_counter()
    clouds = pointgen.cloud_set(count=64, seed=3)
    total = sum(len(c["points"]) for c in clouds)
    log(f"generated {len(clouds)} clouds, {total} points in {time.perf_counter() - t0:.1f} s")
    steps = 10
    devs, cuts = [], []
    for c in clouds:
        p = c["points"]
        devs.append(torch.from_numpy(p.view(np.uint8).reshape(-1)).to("cuda:0"))
        cuts.append(np.linspace(0, len(p), steps + 1).astype(np.int64))
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()

    def batch_of(i, k):
        return devs[i][int(cuts[i][k]) * 16:int(cuts[i][k + 1]) * 16]

    trees = [simlod.Octree(cloud_config(c, int(cuts[i][1] - cuts[i][0]) + 1))
             for i, c in enumerate(clouds)]

    def timed_run(insert_step):
        for t in trees:
            t.reset(stream)
        torch.cuda.synchronize()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(steps)]
        t_start = time.perf_counter()
        for k in range(steps):
            ev[k][0].record(stream)
            insert_step(k)
            ev[k][1].record(stream)
        torch.cuda.synchronize()
        el = time.perf_counter() - t_start
        return el, np.array([a.elapsed_time(b) for a, b in ev])

    def plain_step(k):
        for i, t in enumerate(trees):
            t.insert(batch_of(i, k), stream)

    group = simlod.Group(trees, graph=True, autotune=True)

    def group_step(k):
        group.insert([batch_of(i, k) for i in range(len(trees))], stream)

    # warmup: the group's tuning passes and graph capture, then the plain form
    for _ in range(max(1, -(-simlod.TUNE_PASSES // steps))):
        timed_run(group_step)
    timed_run(plain_step)
    el_plain, lat_plain = timed_run(plain_step)
    plain_canon = [t.snapshot(nodes_only=True).nodes.tobytes() for t in trees[:8]]
    el_group, lat_group = timed_run(group_step)
    group.sync()
    shape = group.shape()
    same = all(t.snapshot(nodes_only=True).nodes.tobytes() == c
               for t, c in zip(trees[:8], plain_canon))
    st = [t.stats() for t in trees]
    group.close()
    for t in trees:
        t.close()
    value = total / el_group
    result = {
        "metric": "inserted points/sec, 64 clouds per step (batched group form)",
        "value": round(value, 1), "unit": "points/s", "n_gpus": 1, "steps": steps,
        "warmup": steps, "ms_per_step": round(el_group * 1e3 / steps, 4),
        "step_ms_p50": round(float(np.percentile(lat_group, 50)), 4),
        "step_ms_p99": round(float(np.percentile(lat_group, 99)), 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "64 clouds, log-uniform 100k..50M points, aerial or dense-scan "
                               "by seed, 10 batches each", "points": total, "clouds": 64},
        "plain_form": {"value": round(total / el_plain, 1), "unit": "points/s",
                       "ms_per_step": round(el_plain * 1e3 / steps, 4),
                       "step_ms_p50": round(float(np.percentile(lat_plain, 50)), 4),
                       "step_ms_p99": round(float(np.percentile(lat_plain, 99)), 4)},
        "speedup_vs_plain": round(el_plain / el_group, 3),
        "group_shape": shape,
        "node_tables_identical": bool(same),
        "status_ok": all(x["status_bits"] == 0 for x in st),
    }
    print(json.dumps(result), flush=True)


def busy_seconds(spans):
    """Length of the union of the (start, end) intervals: the time in which
    at least one request was outstanding."""
    busy, end = 0.0, float("-inf")
    for a, b in sorted(spans):
        if b > end:
            busy += b - max(a, end)
            end = b
    return busy


def run_served(args):
    """Continuous batching under load.  16 stream slots serve 20 clouds of
    10M..200M points (log-uniform; aerial or dense scan by seed), each cut
    into requests of 50k..5M points (log-uniform); requests of a slot arrive
    as a Poisson process.  A finished cloud's octree is closed (after its
    last request) and the slot admits the next cloud against a 200 GB
    device-memory budget.  The same arrival trace is served twice: batched
    (every pass takes the oldest request of each stream) and unbatched (one
    request per pass, arrival order).  Latency = submission to completion.

    Offered loads: unless --offered names them, 0.5, 0.8 and 0.95 of the
    capacity of the unbatched form, measured first with every request
    arriving at once.  Throughput is reported over the wall time of a run and
    over its busy time (the union of the intervals in which at least one
    request was outstanding), which the arrival trace does not stretch."""
    import torch

    import pointgen
    from paper_2310_03567_amd import simlod

    t0 = time.perf_counter()
    clouds = pointgen.cloud_set(count=20, seed=4, lo=1e7, hi=2e8)
    total = sum(len(c["points"]) for c in clouds)
    log(f"generated {len(clouds)} clouds, {total} points in {time.perf_counter() - t0:.1f} s")
    devs = [torch.from_numpy(c["points"].view(np.uint8).reshape(-1)).to("cuda:0") for c in clouds]
    torch.cuda.synchronize()
    reqs = []
    for i, c in enumerate(clouds):
        rng = np.random.default_rng(4000 + i)
        n, a, cuts = len(c["points"]), 0, [0]
        while a < n:
            a = min(n, a + int(np.exp(rng.uniform(np.log(5e4), np.log(5e6)))))
            cuts.append(a)
        reqs.append(cuts)
    nreq = sum(len(r) - 1 for r in reqs)
    mean_req = total / nreq
    slots = 16
    cfgs = [cloud_config(c, 5_000_000) for c in clouds]

    def serve(sv, offered_pps, seed):
        rate = offered_pps / slots / mean_req  # requests/s per slot
        rng = np.random.default_rng(seed)
        lat = []
        spans = []  # (submission, completion) of every request, seconds
        c0 = sv.counters()
        queue = list(range(len(clouds)))
        active = {}  # slot index -> [cloud, next request, stream id, next arrival, tickets]
        start = time.perf_counter()
        for k in range(slots):
            active[k] = None
        done_points = 0
        while True:
            now = time.perf_counter() - start
            for k in range(slots):
                st = active[k]
                if st is None and queue:
                    sid = sv.open(cfgs[queue[0]])
                    if sid is not None:
                        ci = queue.pop(0)
                        active[k] = [ci, 0, sid, now + rng.exponential(1.0 / rate), []]
                    continue
                if st is None:
                    continue
                ci, r, sid, t_next, tickets = st
                cuts = reqs[ci]
                while r < len(cuts) - 1 and t_next <= now:
                    b = devs[ci][cuts[r] * 16:cuts[r + 1] * 16]
                    tickets.append((sv.submit(sid, b), time.perf_counter() - start))
                    r += 1
                    t_next += rng.exponential(1.0 / rate)
                st[1], st[3] = r, t_next
                if r == len(cuts) - 1 and all(sv.poll(t)[0] for t, _ in tickets[-1:]):
                    for t, ts in tickets:
                        d, ms, rc = sv.poll(t)
                        if not d or rc != simlod.OK:
                            raise RuntimeError(f"request failed ({rc})")
                        lat.append(ms)
                        spans.append((ts, ts + ms / 1e3))
                    done_points += cuts[-1]
                    sv.close_stream(sid)
                    active[k] = None
            if not queue and all(v is None for v in active.values()):
                break
            time.sleep(0.0002)
        el = time.perf_counter() - start
        sv.wait_closed()
        c = sv.counters()
        lat = np.array(lat)
        passes = int(c["passes"] - c0["passes"])
        busy = busy_seconds(spans)
        return {"offered_points_per_s": round(offered_pps, 1),
                "achieved_points_per_s": round(done_points / el, 1),
                "busy_points_per_s": round(done_points / max(busy, 1e-9), 1),
                "busy_seconds": round(busy, 3),
                "requests": int(len(lat)), "passes": passes,
                "requests_per_pass": round(len(lat) / max(passes, 1), 2),
                "latency_ms_p50": round(float(np.percentile(lat, 50)), 3),
                "latency_ms_p99": round(float(np.percentile(lat, 99)), 3),
                "seconds": round(el, 3)}

    # one server per form, one form at a time (each pools its octrees in
    # device memory); a warm-up run allocates the octrees, which the measured
    # runs then reuse from the server's pool.  batched_budget: batched, with a
    # pass budget of 1M points (a request of up to 5M points is inserted over
    # several passes, so small requests of other streams do not wait behind
    # it).  The unbatched form goes first: its capacity sets the loads.
    forms = (("unbatched", 1, 0), ("batched", 0, 0), ("batched_budget", 0, 1_000_000))
    capacity = None
    loads = [float(x) * 1e9 for x in str(args.offered).split(",")] if args.offered else None
    runs = {}
    for form, per_pass, budget in forms:
        sv = simlod.Server(max_streams=slots, hbm_budget=200 << 30, max_per_pass=per_pass,
                           pass_points=budget)
        serve(sv, 1e13 if loads is None else loads[0], seed=40)  # warm-up
        if loads is None:
            cap_run = serve(sv, 1e13, seed=39)  # every request at once
            capacity = cap_run["achieved_points_per_s"]
            log(f"unbatched capacity {capacity / 1e9:.2f} G points/s")
            loads = [f * capacity for f in (0.5, 0.8, 0.95)]
        runs[form] = [serve(sv, offered, seed=41 + k) for k, offered in enumerate(loads)]
        sv.close()
    sweep = []
    for k, offered in enumerate(loads):
        b, u = runs["batched"][k], runs["unbatched"][k]
        sweep.append({form: runs[form][k] for form, _, _ in forms})
        log(f"offered {offered / 1e9:.2f} G/s: batched {b['achieved_points_per_s'] / 1e9:.2f} G/s "
            f"(busy {b['busy_points_per_s'] / 1e9:.2f}) p99 {b['latency_ms_p99']} ms; unbatched "
            f"{u['achieved_points_per_s'] / 1e9:.2f} G/s (busy {u['busy_points_per_s'] / 1e9:.2f}) "
            f"p99 {u['latency_ms_p99']} ms; batched with a 1M-point pass budget p50 "
            f"{runs['batched_budget'][k]['latency_ms_p50']} p99 "
            f"{runs['batched_budget'][k]['latency_ms_p99']} ms")
    top = sweep[-1]["batched"]
    result = {
        "metric": "served insertion: points/sec with p50/p99 update latency",
        "value": top["achieved_points_per_s"], "unit": "points/s", "n_gpus": 1,
        "steps": top["requests"], "warmup": 1,
        "ms_per_step": round(top["seconds"] * 1e3 / max(top["requests"], 1), 4),
        "update_ms_p50": top["latency_ms_p50"], "update_ms_p99": top["latency_ms_p99"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "16 stream slots, 20 clouds of 10M..200M points, requests of "
                               "50k..5M points, Poisson arrivals, 200 GB admission budget",
                   "points": total, "requests": nreq},
        "unbatched_capacity_points_per_s": capacity,
        "offered_fractions_of_capacity": None if capacity is None else [0.5, 0.8, 0.95],
        "sweep": sweep,
    }
    print(json.dumps(result), flush=True)


def run_chunk_sweep(args):
    """Chunk capacity against construction time and memory (the paper's
    chunk-size experiment, section "Chunks and the Chunk Pool", here on the
    synthetic aerial workload): the whole 100M-point cloud is inserted in
    1M-point batches into a fresh octree for each chunk capacity."""
    import torch

    from paper_2310_03567_amd import simlod

    w = WORKLOADS["aerial"]
    B = w["batch"]
    pts = generate("aerial")
    dev = torch.from_numpy(pts.view(np.uint8).reshape(-1)).to("cuda:0")
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    rows = []
    for C in (500, 1000, 2000, 5000, 10000):
        cfg = octree_config("aerial")
        cfg.chunk_capacity = C
        tree = simlod.Octree(cfg)
        for rep in range(2):  # the first build warms up, the second is timed
            tree.reset(stream)
            torch.cuda.synchronize()
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            for i in range(len(pts) // B):
                tree.insert(dev[i * B * 16:(i + 1) * B * 16], stream)
            b.record(stream)
            torch.cuda.synchronize()
        st = tree.stats()
        tree.close()
        rec_bytes = (st["num_points"] + st["num_voxels"]) * 20
        rows.append({"chunk_capacity": C, "construct_ms": round(a.elapsed_time(b), 2),
                     "chunks": st["chunks_in_use"],
                     "arena_bytes_used": st["arena_bytes_used"],
                     "record_bytes": rec_bytes,
                     "arena_overhead": round(st["arena_bytes_used"] / rec_bytes - 1.0, 4)})
        log(json.dumps(rows[-1]))
    best = min(rows, key=lambda r: r["construct_ms"])
    result = {
        "metric": "construction time and memory against chunk capacity",
        "value": best["construct_ms"], "unit": "ms", "n_gpus": 1, "steps": len(pts) // B,
        "warmup": 1, "ms_per_step": round(best["construct_ms"] / (len(pts) // B), 4),
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": w["desc"], "points": len(pts), "batch": B},
        "sweep": rows,
    }
    print(json.dumps(result), flush=True)


def host_facts():
    """CPU model and thread counts of the host this runs on."""
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        usable = os.cpu_count()
    return {"cpu_model": model, "nproc": os.cpu_count(), "usable_cpus": usable}


def cpu_baseline(points, batch, cfg_kw, budget_s=20.0):
    """Sequential C oracle (one thread) on a prefix of the same batches."""
    from oracle import LodConfig
    from oracle.incremental import IncrementalOracle

    cfg = LodConfig(root_min=cfg_kw["root_min"], root_size=cfg_kw["root_size"])
    o = IncrementalOracle(cfg)
    done = 0
    t0 = time.perf_counter()
    while done < len(points) and time.perf_counter() - t0 < budget_s:
        o.insert(points[done:done + batch])
        done += min(batch, len(points) - done)
    dt = time.perf_counter() - t0
    o.close()
    out = {"value": done / dt, "unit": "points/s", "cores": 1, "kind": "oracle",
           "sample": f"first {done // batch} batches ({done} points) inserted in order, "
                     f"{dt:.1f} s, sequential C inserter on one thread"}
    out.update(host_facts())
    return out


def algorithmic_pass_bytes(points, spilled, new_voxels, new_inner):
    """What the insertion must move, summed over the timed passes: read each
    batch record (16 B) and write it with its key into a leaf (20 B); read
    and rewrite each spilled record with its key (40 B); write each new
    voxel (16 B); clear each new inner node's 128^3 occupancy grid
    (256 KiB)."""
    return (16 + 20) * points + 40 * spilled + 16 * new_voxels + (GRID_BYTES * new_inner)


GRID_BYTES = 128 ** 3 // 8


def measure(name, steps, warmup, order=None, pts=None):
    """Times one workload: W warmup batches into a scratch build (then reset),
    an untimed build with every kernel timed (picks the dominant kernel), the
    timed region (batches 0..K-1 into an empty octree, the dominant kernel
    bracketed by the library's fence-free events on the insertion stream),
    and a build with an event pair around every pass for the per-update
    latency.  Returns the result fields and the generated points."""
    import torch

    from paper_2310_03567_amd import simlod

    w = WORKLOADS[name]
    B = w["batch"]
    nb_total = w["points"] // B
    steps = min(steps, nb_total)
    warm = min(warmup, nb_total)
    t0 = time.perf_counter()
    if pts is None:
        pts = generate(name, order=order)
    log(f"{name}{'/' + order if order else ''}: {len(pts)} points generated in "
        f"{time.perf_counter() - t0:.1f} s")
    need = max(steps, warm) * B
    dev = torch.from_numpy(pts[:need].view(np.uint8).reshape(-1)).to("cuda:0")
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    tree = simlod.Octree(octree_config(name))

    def batch(i):
        return dev[i * B * 16:(i + 1) * B * 16]

    for i in range(warm):
        tree.insert(batch(i), stream)
    tree.sync()
    tree.reset(stream)
    simlod.set_kernel_timing(tree.handle, "all")
    for i in range(steps):
        tree.insert(batch(i), stream)
    tree.sync()
    per_kernel = simlod.get_kernel_times(tree.handle)
    dominant = max(per_kernel, key=lambda k: per_kernel[k][1])
    log(f"{name} per-kernel (launches, total ms): " + json.dumps(per_kernel))
    tree.reset(stream)
    tree.sync()

    simlod.set_kernel_timing(tree.handle, [dominant])
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for i in range(steps):
        tree.insert(batch(i), stream)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    st = tree.stats()
    kt = simlod.get_kernel_times(tree.handle)[dominant]

    simlod.set_kernel_timing(tree.handle, [])
    tree.reset(stream)
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(steps)]
    torch.cuda.synchronize()
    for i in range(steps):
        ev[i][0].record(stream)
        tree.insert(batch(i), stream)
        ev[i][1].record(stream)
    torch.cuda.synchronize()
    per_update_ms = np.array([a.elapsed_time(b) for a, b in ev])
    tree.close()
    del dev
    torch.cuda.empty_cache()

    n_ins = steps * B
    ms_per_step = elapsed * 1e3 / steps
    if dominant == "sample_store" and kt[0] > 0:
        work_items = n_ins + st["sum_spilled"]
        alg_bytes = (SAMPLE_STORE_BYTES_PER_ITEM * work_items
                     + SAMPLE_STORE_BYTES_PER_SPILLED * st["sum_spilled"])
        avg_s = kt[1] / 1e3 / kt[0]
        achieved = alg_bytes / kt[0] / avg_s / 1e9
        traffic = measured_traffic(name)
        roofline = {"kernel": "k_sample_store", "bound": "hbm", "achieved": round(achieved, 1),
                    "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(achieved / HBM_PEAK_GBS, 4),
                    "traffic": None if traffic is None else int(traffic),
                    "launches": kt[0], "avg_launch_us": round(avg_s * 1e6, 2),
                    "bytes_per_launch": int(alg_bytes / kt[0])}
    else:
        roofline = {"kernel": dominant, "bound": "hbm", "achieved": None, "peak": HBM_PEAK_GBS,
                    "unit": "GB/s", "frac": None, "traffic": None, "launches": kt[0],
                    "avg_launch_us": round(kt[1] * 1e3 / max(kt[0], 1), 2)}
    pass_bytes = algorithmic_pass_bytes(n_ins, st["sum_spilled"], st["sum_new_voxels"],
                                        st["num_inner"])
    pass_gbs = pass_bytes / elapsed / 1e9
    pass_roofline = {"scope": "whole insertion pass (all kernels), wall clock of the timed "
                              "region",
                     "bound": "hbm", "achieved": round(pass_gbs, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(pass_gbs / HBM_PEAK_GBS, 4),
                     "bytes_per_update": int(pass_bytes / steps),
                     "bytes": "16+20 B per point, 40 B per spilled point, 16 B per new voxel, "
                              "256 KiB per new inner node"}
    kernel_us = {k: round(v[1] * 1e3 / v[0], 2) for k, v in per_kernel.items() if v[0]}
    res = {
        "value": round(n_ins / elapsed, 1),
        "unit": "points/s",
        "steps": steps,
        "warmup": warm,
        "ms_per_step": round(ms_per_step, 4),
        "ms_per_1M_update": round(ms_per_step * 1e6 / B, 4),
        "update_ms_p50": round(float(np.percentile(per_update_ms, 50)), 4),
        "update_ms_p99": round(float(np.percentile(per_update_ms, 99)), 4),
        "config": {"workload": w["desc"] + (f", order {order}" if order else ""),
                   "points": n_ins, "batch": B,
                   "timed_batches": f"batches 0..{steps - 1} of {nb_total} "
                                    f"({n_ins} of {w['points']} points)",
                   "leaf_capacity": 50_000, "grid": 128, "max_depth": 16, "chunk": 1000},
        "octree": {k: st[k] for k in ("num_nodes", "num_inner", "num_points", "num_voxels",
                                      "max_rounds", "sum_spilled", "sum_new_voxels")},
        "roofline": roofline,
        "pass_roofline": pass_roofline,
        "kernel_avg_us": kernel_us,
    }
    return res, pts


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="aerial",
                    choices=sorted(WORKLOADS) + ["batched", "served", "chunk-sweep"])
    ap.add_argument("--order", default=None, choices=["morton_shuffled", "morton", "random"],
                    help="aerial workload: point order of the cloud (default Morton-shuffled)")
    ap.add_argument("--offered", default=None,
                    help="served workload: offered loads in G points/s over all streams "
                         "(comma-separated); default: 0.5, 0.8 and 0.95 of the measured "
                         "capacity of the plain (unbatched) form")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="headline workload only: no dense-scan and order-variant records")
    ap.add_argument("--cpu-budget", type=float, default=20.0)
    ap.add_argument("--copy-calibration-mb", type=int, default=0,
                    help="run one plain device-to-device copy of this size first (an HBM "
                         "counter reference for rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              f"(nothing in this build uses a second GPU)", file=sys.stderr)
        sys.exit(2)

    if args.workload == "batched":
        run_batched(args)
        return
    if args.workload == "served":
        run_served(args)
        return
    if args.workload == "chunk-sweep":
        run_chunk_sweep(args)
        return

    import torch

    if args.copy_calibration_mb:
        a = torch.empty(args.copy_calibration_mb << 20, dtype=torch.uint8, device="cuda:0")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    name = args.workload
    head, pts = measure(name, args.steps, args.warmup, order=args.order)
    result = {
        "metric": "inserted points/sec (ms per 1M-point update)",
        "value": head["value"], "unit": "points/s", "n_gpus": 1,
        "steps": head["steps"], "warmup": head["warmup"], "ms_per_step": head["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
    }
    result.update({k: v for k, v in head.items() if k not in result})
    if not args.no_cpu_baseline:
        result["cpu_baseline"] = cpu_baseline(pts, WORKLOADS[name]["batch"], WORKLOADS[name],
                                              args.cpu_budget)
    del pts
    if not args.no_extras and name == "aerial":
        extra, _ = measure("dense", args.steps, min(args.warmup, 3))
        result["dense"] = extra
        if args.order is None:
            result["order_variants"] = {}
            for order in ("morton", "random"):
                v, _ = measure("aerial", args.steps, args.warmup, order=order)
                result["order_variants"][order] = {
                    k: v[k] for k in ("value", "ms_per_step", "update_ms_p50", "update_ms_p99",
                                      "roofline", "pass_roofline")}
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
