"""Benchmark of the gridless ring solve on one MI355X.

One step = one pass of the whole hot path over one batch: every instance of
the batched workload (512 independent instances, ring counts log-uniform in
[1000, 8000], geometric spacing from 1e-4 to r=8, driver + witness beams,
2000 slices each) is reset to slice 0 and marched through its whole window
by one persistent launch replayed from a HIP graph.  value = ring-slice
updates per second over the timed steps (inputs resident in HBM).

Before the timed steps the autotuner measures the marcher's layout per
ring-count bucket on these instances (and on the two large single solves)
and installs it; the batch is built with it.

Also reported: the plain single-instance path (the same kernels, one
instance per launch: the linear 1000-ring workload through its 1200 slices,
and instances of the batch one after the other), the batched/plain ratio,
the roofline of the march kernel from live HIP-event timings, the large
single solves on the cooperative path (with their roofline fraction and
per-slice latency floor), the served form, and the CPU oracle timed on
bounded samples (the batch on every host core, the other workloads on one).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "ring-slice updates/s batched+served vs plain (FP64, 1e-8 rel); p50/p99 latency"
PEAK_FP64_VECTOR = 78.6e12       # FP64 vector FLOP/s of MI355X (256 CU x 2.4 GHz x 128)
PEAK_HBM = 8.0e12                 # HBM3E bytes/s

# Algorithmic work per ring-slice of the method (one ring, one slice), the
# per-unit figures of the measurement plan: 150-200 FP64 flops, one log and
# about eight divides counted as one flop each, and about four double-double
# additions of about 20 flops each.
ALG_FLOPS_PER_RING_SLICE = 280
# Bytes the method must move per ring-slice: read rho, u_r, the two AB2
# history terms, w and w^ (48 B); write rho, u_r and the history (32 B); the
# ion-table interpolation (32 B, cache resident).
ALG_BYTES_PER_RING_SLICE = 48 + 32 + 32
# Two-species (mobile ion) batch: hydrogen ions (proton over electron mass);
# bytes the method must move per species-ring-slice: read rho, u_r and the
# AB2 history (32 B) and the ring's constants w, w^, r0, 1/r0, ln r0 (dd) and
# dr (56 B); write rho, u_r and the history (32 B).
ION_MASS_H = 1836.15267
ALG_BYTES_PER_SPECIES_RING_SLICE = 32 + 56 + 32
# Slices each autotuner candidate marches (from slice 0: through the head of
# the batch's drivers, whose centres lie at slices 200-667).
TUNE_SLICES = 600


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def build_batch(wake, insts, stream, grid=None):
    solvers = [wake.WakeSolver.from_instance(inst, stream=stream) for inst in insts]
    for s in solvers:
        if grid is not None:
            s.wake_set_grid(*grid)
        s.wake_prepare()
    batch = wake.WakeBatch(solvers, stream=stream)
    return solvers, batch


_WORKER = r"""
import json, sys, time
sys.path.insert(0, sys.argv[1])
try:
    from threadpoolctl import threadpool_limits
    threadpool_limits(1)
except Exception:
    pass
from oracle.wake_oracle import RingOracle
from paper_2603_16623_amd import workloads as W
job = json.loads(sys.argv[2])
t0 = time.time()
done, parts = 0, []
if job["kind"] == "batch":
    insts = W.config3(n_inst=job["n_inst"], n_xi=job["n_xi"])
    for i in job["which"]:
        inst = insts[i]
        o = RingOracle(inst.r0, inst.dr, inst.dxi, inst.n_xi, inst.sources)
        state = o.initial_state()
        n = 0
        while n < inst.n_xi - 1 and time.time() - t0 < job["budget"]:
            _, state = o.slice(n, state)
            n += 1
        done += inst.n_rings * n
        parts.append((inst.n_rings, n, inst.n_xi - 1))
        if time.time() - t0 >= job["budget"]:
            break
elif job["kind"] == "ions":
    from oracle.mobile_ions import TwoSpeciesOracle
    inst = W.config3(n_inst=job["n_inst"], n_xi=job["n_xi"])[job["which"]]
    o = TwoSpeciesOracle(inst.r0, inst.dr, inst.dxi, inst.n_xi, job["m_i"], inst.sources)
    state = o.initial_state()
    n = 0
    t0 = time.time()
    while n < inst.n_xi - 1 and time.time() - t0 < job["budget"]:
        _, state = o.slice(n, state)
        n += 1
    done = 2 * inst.n_rings * n
    parts.append((inst.n_rings, n, inst.n_xi - 1))
else:
    inst = getattr(W, job["kind"])()
    o = RingOracle(inst.r0, inst.dr, inst.dxi, inst.n_xi, inst.sources, inst.dens)
    state = o.initial_state()
    n = 0
    t0 = time.time()
    while n < inst.n_xi - 1 and time.time() - t0 < job["budget"]:
        _, state = o.slice(n, state)
        n += 1
    done = inst.n_rings * n
    parts.append((inst.n_rings, n, inst.n_xi - 1))
print(json.dumps(dict(done=done, parts=parts, t0=t0, t1=time.time())))
"""


def _run_workers(jobs, budget_s):
    """One plain host process per job (no process pool: every worker is a
    child of this process, waited for, and gone when this returns).  Returns
    the workers' results."""
    import subprocess
    env = dict(os.environ, OMP_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1", MKL_NUM_THREADS="1")
    procs = [subprocess.Popen([sys.executable, "-c", _WORKER, ROOT, json.dumps(j)], env=env,
                              stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True) for j in jobs]
    out = []
    for p in procs:
        so, se = p.communicate(timeout=budget_s * 4 + 300)
        if p.returncode != 0:
            raise RuntimeError(f"oracle worker failed: {se[-2000:]}")
        out.append(json.loads(so.strip().splitlines()[-1]))
    return out


def host_cores() -> int:
    """Host cores this benchmark may use: the OpenMP thread setting of the
    machine if there is one, else the CPU count, at most 16."""
    try:
        n = int(os.environ.get("OMP_NUM_THREADS", "0"))
    except ValueError:
        n = 0
    return max(1, min(16, n or (os.cpu_count() or 1)))


def cpu_baseline(n_inst, n_xi, budget_s: float = 15.0, cores: int = 0):
    """Time the oracle on a bounded sample of the batch: one host process per
    core (numpy on one thread each), process i marching instances i, i + k,
    ... from slice 0 for about budget_s seconds; rate = all ring-slices over
    the span from the first worker's start to the last worker's end."""
    cores = max(1, min(cores or host_cores(), n_inst))
    jobs = [dict(kind="batch", n_inst=n_inst, n_xi=n_xi, budget=budget_s,
                 which=list(range(i, n_inst, cores))) for i in range(cores)]
    res = _run_workers(jobs, budget_s)
    done = sum(r["done"] for r in res)
    span = max(r["t1"] for r in res) - min(r["t0"] for r in res)
    parts = [p for r in res for p in r["parts"]]
    whole = sum(1 for _, ns, nw in parts if ns == nw)
    rings = [p[0] for p in parts]
    return dict(value=done / span, unit="ring-slice updates/s", cores=cores, kind="oracle",
                sample=f"oracle (numpy, one thread per process) in {cores} host processes, each "
                       f"marching instances of the batch from slice 0 (process i takes instances "
                       f"i, i + {cores}, ...): {len(parts)} instances of {min(rings)}-{max(rings)} "
                       f"rings, {whole} of them through the whole window; {done} ring-slices in "
                       f"{span:.1f} s")


def cpu_single_core(budget_s: float):
    """The oracle on one core for the single-instance workloads, side by side
    (one process each, started together): the linear 1000-ring workload
    through its whole window, and the first slices of the 20000-ring blowout
    and of the 200000-ring laser case, about budget_s seconds each."""
    names = {"config1": "linear 1000 rings x 1200 slices",
             "config2": "blowout 20000 rings x 4000 slices",
             "config5": "laser 200000 rings x 8000 slices"}
    res = _run_workers([dict(kind=k, budget=budget_s) for k in names], budget_s)
    out = {}
    for k, r in zip(names, res):
        n_rings, n, nw = r["parts"][0]
        out[names[k]] = dict(value=r["done"] / (r["t1"] - r["t0"]), unit="ring-slice updates/s",
                             cores=1, kind="oracle",
                             sample=f"slices 0-{n} of {nw + 1} ({n_rings} rings), {r['t1'] - r['t0']:.1f} s")
    return out


C4_MEAN_WORK = (50_000 - 500) / math.log(100.0) * (500 + 8000) / 2.0   # E[N] E[N_xi]


def _pct(x, q):
    return float(np.percentile(np.asarray(x), q)) if len(x) else None


def served_run(wake, W, stream, rate, seconds, budget_bytes, step_us, seed=4, max_wall=150.0):
    """Real-time Poisson stream of served-form requests (ring counts log-uniform
    in [500, 50000], window lengths uniform in [500, 8000], beams as the batched
    workload).  Instances are built before the clock starts; each arrives at its
    scheduled time.  Latency = result ready - scheduled arrival."""
    specs, build = W.config4_stream(seed=seed, rate=rate, duration=seconds)
    reqs = [(t, build(k)) for t, k in specs]
    srv = wake.WakeServer(device_bytes=budget_bytes, slices_per_step=100_000, step_us=step_us,
                          stream=stream)
    arrival, work, lat = {}, {}, []
    done_work, i, steps, max_queue = 0, 0, 0, 0
    t0 = time.perf_counter()
    while True:
        now = time.perf_counter() - t0
        while i < len(reqs) and reqs[i][0] <= now:
            t = srv.submit_instance(reqs[i][1])
            arrival[t] = reqs[i][0]
            work[t] = reqs[i][1].ring_slices
            i += 1
        st = srv.stats()
        max_queue = max(max_queue, st["queued"])
        if st["active"] + st["queued"] == 0:
            if i >= len(reqs):
                break
            time.sleep(max(0.0, min(0.002, reqs[i][0] - now)))
            continue
        srv.step()
        steps += 1
        tnow = time.perf_counter() - t0
        for t in srv.ready():
            r = srv.result(t)
            lat.append(tnow - arrival.pop(t))
            done_work += work.pop(t)
            if r["status"] not in (0, wake.WAKE_EBREAKDOWN):
                raise RuntimeError(f"request {t} failed: {r['status']}")
        if tnow > max_wall:
            break
    wall = time.perf_counter() - t0
    marched = srv.stats()["ring_slices"]
    srv.close()
    return dict(rate=rate, arrival_seconds=seconds, requests=len(reqs), completed=len(lat),
                unfinished=len(arrival), wall_s=wall, steps=steps, max_queue=max_queue,
                ring_slices_marched=marched, throughput=marched / wall,
                p50_latency_s=_pct(lat, 50), p99_latency_s=_pct(lat, 99),
                mean_latency_s=float(np.mean(lat)) if lat else None)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n-inst", type=int, default=512)
    ap.add_argument("--n-xi", type=int, default=2000)
    ap.add_argument("--plain-sample", type=int, default=16)
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--tiling", type=str, default="")
    ap.add_argument("--grid-nodes", type=int, default=64,
                    help="field-grid nodes per instance for the grid measurement (0: skip it)")
    ap.add_argument("--grid-r", type=float, default=1.0, help="field-grid radius")
    ap.add_argument("--grid-steps", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--served-seconds", type=float, default=60.0,
                    help="arrival window of the served run (0: skip)")
    ap.add_argument("--served-rate", type=float, default=0.0,
                    help="request rate of the served run (0: 85%% of the measured capacity)")
    ap.add_argument("--served-budget-gib", type=float, default=64.0)
    ap.add_argument("--no-large", dest="large", action="store_false",
                    help="skip the large single instances (cooperative path)")
    ap.add_argument("--no-tune", dest="tune", action="store_false",
                    help="skip the autotuner (tiling settings instead)")
    ap.add_argument("--ions-inst", type=int, default=256,
                    help="two-species (mobile hydrogen ion) batch: instances (0: skip)")
    ap.add_argument("--ions-xi", type=int, default=1000, help="two-species batch: slices each")
    ap.add_argument("--ions-steps", type=int, default=2)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (--gpus {args.gpus} requested); the "
              "batched instances would shard across GPUs with no exchange, but that "
              "path is not built or measured here.", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2603_16623_amd import wake, workloads as W
    wake.load()
    torch.cuda.init()
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    # a stream of our own (default priority) made current, so that the
    # library's launches and torch's timing events share one stream
    tstream = torch.cuda.Stream(device=dev)
    torch.cuda.set_stream(tstream)
    stream = tstream.cuda_stream
    if args.tiling:
        nt, wpc = (int(x) for x in args.tiling.split(","))
        wake.wake_set_tiling(nt, wpc)
    nt, wpc = wake.wake_get_tiling()

    log(f"building {args.n_inst} instances x {args.n_xi} slices")
    insts = W.config3(n_inst=args.n_inst, n_xi=args.n_xi)
    work = sum(i.ring_slices for i in insts)
    tuning = None
    if args.tune:
        log("autotune")
        t_tune = time.perf_counter()
        large = [W.config2(), W.config5()] if args.large else []
        tuning = wake.wake_autotune(insts + large, TUNE_SLICES, stream=stream)
        tuning["seconds"] = time.perf_counter() - t_tune
        log(f"tuning {tuning}")
    solvers, batch = build_batch(wake, insts, stream)
    batch.wake_batch_capture()
    log("warmup")
    for _ in range(args.warmup):
        batch.wake_batch_replay()
    torch.cuda.synchronize()

    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for a, b in ev:
        a.record()
        batch.wake_batch_replay()
        b.record()
        log("step done")
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kernel_ms = [a.elapsed_time(b) for a, b in ev]
    breakdowns = sum(1 for s in solvers if s.wake_status()[0] >= 0)
    value = work * args.steps / wall
    avg_kernel_s = float(np.mean(kernel_ms)) / 1e3

    # plain single-instance path: the same instances one launch at a time
    log("plain path")
    sample = insts[: args.plain_sample]
    plain_solvers = [wake.WakeSolver.from_instance(i, stream=stream) for i in sample]
    for s in plain_solvers:
        s.wake_prepare()
    torch.cuda.synchronize()
    tp = time.perf_counter()
    for s in plain_solvers:
        s.wake_solve(0, s.n_xi)
    torch.cuda.synchronize()
    tplain = time.perf_counter() - tp
    plain_value = sum(i.ring_slices for i in sample) / tplain
    # the linear workload (1000 rings x 1200 slices, 10^4 particles) as the
    # plain single instance: one solve, one launch
    c1 = W.config1()
    s1 = wake.WakeSolver.from_instance(c1, stream=stream)
    s1.wake_prepare()
    torch.cuda.synchronize()
    tp = time.perf_counter()
    s1.wake_solve(0, c1.n_xi)
    s1.wake_sync()
    t1 = time.perf_counter() - tp
    linear = dict(value=c1.ring_slices / t1, unit="ring-slice updates/s", seconds=t1,
                  us_per_slice=t1 / c1.n_xi * 1e6, threads=s1.threads(), breakdown_slice=s1.wake_status()[0])
    s1.close()

    # measured HBM traffic of one march dispatch of this workload, if the
    # counters were taken on the current marcher sources
    from paper_2603_16623_amd.profile_summary import read_traffic
    workload = f"batched-{args.n_inst}x[1000,8000]rings-x{args.n_xi}slices"
    tr = read_traffic(os.path.join(ROOT, "profiles", "wake_march_kernel_traffic.txt"))
    traffic = None
    if tr is not None and tr.get("workload") == workload:
        traffic = float(tr["fetch_bytes_per_dispatch"]) + float(tr["write_bytes_per_dispatch"])
    # The march moves several times its algorithmic bytes (two passes over
    # the rings, the slice scratch and the ion records) and its measured HBM
    # traffic runs at the larger part of the HBM peak, so the HBM roof is the
    # one that bounds it; the FP64 figure is reported beside it.
    alg_bytes = ALG_BYTES_PER_RING_SLICE * work
    achieved = alg_bytes / avg_kernel_s
    flops = ALG_FLOPS_PER_RING_SLICE * work
    roof = dict(bound="hbm", achieved=achieved / 1e9, peak=PEAK_HBM / 1e9, unit="GB/s",
                frac=achieved / PEAK_HBM, traffic=traffic,
                traffic_source=None if traffic is None else
                "replayed: rocprofv3 FETCH_SIZE and WRITE_SIZE of one march dispatch of this "
                "workload on the current marcher sources (profiles/wake_march_kernel_traffic.txt, "
                "copy-calibrated)",
                kernel="wake_march_kernel", kernel_ms=float(np.mean(kernel_ms)),
                alg_bytes_per_ring_slice=ALG_BYTES_PER_RING_SLICE,
                traffic_B_per_ring_slice=None if traffic is None else traffic / work,
                hbm_measured_GBps=None if traffic is None else traffic / avg_kernel_s / 1e9,
                hbm_measured_frac=None if traffic is None else traffic / avg_kernel_s / PEAK_HBM,
                alg_flops_per_ring_slice=ALG_FLOPS_PER_RING_SLICE,
                fp64_TFLOPs=flops / avg_kernel_s / 1e12,
                fp64_frac=flops / avg_kernel_s / PEAK_FP64_VECTOR)
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "ring-slice updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": workload,
                   "instances": args.n_inst, "ring_slices_per_step": work,
                   "tiling": {"threads": nt, "wgs_per_cu": wpc} if tuning is None else None,
                   "autotuned_layout": tuning, "breakdowns": breakdowns},
        "plain_single_instance": {"value": plain_value, "unit": "ring-slice updates/s",
                                  "instances": len(sample),
                                  "what": "the first instances of the batch, one launch each"},
        "linear_single_instance": linear,
        "batched_vs_plain": value / plain_value,
        "roofline": roof,
    }
    if args.grid_nodes > 0:
        # the same batch with a radial field grid on every instance: the
        # fields at grid_nodes cell-centred nodes to r = grid_r, every slice
        log("field grid")
        gsolvers, gbatch = build_batch(wake, insts, stream, grid=(args.grid_nodes, args.grid_r))
        gbatch.wake_batch_capture()
        gbatch.wake_batch_replay()
        torch.cuda.synchronize()
        tg = time.perf_counter()
        for _ in range(args.grid_steps):
            gbatch.wake_batch_replay()
            torch.cuda.synchronize()
            log("grid step done")
        gstep = (time.perf_counter() - tg) / args.grid_steps
        out["field_grid"] = dict(
            nodes=args.grid_nodes, r_max=args.grid_r, steps=args.grid_steps,
            value=work / gstep, unit="ring-slice updates/s", ms_per_step=gstep * 1e3,
            vs_without_grid=(work / gstep) / value,
            node_updates_per_s=args.n_inst * args.n_xi * args.grid_nodes / gstep)
        gbatch.close()
        for s in gsolvers:
            s.close()
    if args.ions_inst > 0:
        # the batch's instances (fewer, shorter windows) with mobile hydrogen
        # ions: one workgroup per instance, replayed from a HIP graph
        log("mobile ions batch")
        iinsts = W.config3(n_inst=args.ions_inst, n_xi=args.ions_xi)
        isolvers = [wake.WakeSolver(i.r0, i.dr, i.dxi, i.n_xi, i.sources, i.dens, stream=stream,
                                    ion_mass=ION_MASS_H) for i in iinsts]
        for s in isolvers:
            s.wake_prepare()
        ibatch = wake.WakeBatch(isolvers, stream=stream)
        ibatch.wake_batch_capture()
        ibatch.wake_batch_replay()
        torch.cuda.synchronize()
        iev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
               for _ in range(args.ions_steps)]
        ti = time.perf_counter()
        for a, b in iev:
            a.record()
            ibatch.wake_batch_replay()
            b.record()
            log("ions step done")
        torch.cuda.synchronize()
        iwall = (time.perf_counter() - ti) / args.ions_steps
        ikern = float(np.mean([a.elapsed_time(b) for a, b in iev])) / 1e3
        iwork = sum(2 * i.ring_slices for i in iinsts)          # species-ring-slices
        ibrk = sum(1 for s in isolvers if s.wake_status()[0] >= 0)
        ibatch.close()
        for s in isolvers:
            s.close()
        iach = ALG_BYTES_PER_SPECIES_RING_SLICE * iwork / ikern
        iload = f"ions-batched-{args.ions_inst}x[1000,8000]rings-x{args.ions_xi}slices"
        itr = read_traffic(os.path.join(ROOT, "profiles", "ions_march_kernel_traffic.txt"),
                           "ions_march_kernel")
        itraffic = None
        if itr is not None and itr.get("workload") == iload:
            itraffic = float(itr["fetch_bytes_per_dispatch"]) + float(itr["write_bytes_per_dispatch"])
        out["mobile_ions"] = dict(
            workload=f"batched-{args.ions_inst}x[1000,8000]rings-x{args.ions_xi}slices, electrons "
                     f"and mobile hydrogen ions (m_i = {ION_MASS_H})",
            ion_mass=ION_MASS_H, steps=args.ions_steps, ms_per_step=iwall * 1e3,
            value=iwork / iwall, unit="species-ring-slice updates/s",
            ring_slice_updates_per_s=iwork / 2 / iwall, breakdowns=ibrk,
            roofline=dict(bound="hbm", achieved=iach / 1e9, peak=PEAK_HBM / 1e9, unit="GB/s",
                          frac=iach / PEAK_HBM, traffic=itraffic,
                          traffic_source=None if itraffic is None else
                          "replayed: rocprofv3 FETCH_SIZE and WRITE_SIZE of one dispatch of this "
                          "workload on the current two-species sources "
                          "(profiles/ions_march_kernel_traffic.txt, copy-calibrated)",
                          traffic_B_per_species_ring_slice=None if itraffic is None else itraffic / iwork,
                          kernel="ions_march_kernel", kernel_ms=ikern * 1e3,
                          alg_bytes_per_species_ring_slice=ALG_BYTES_PER_SPECIES_RING_SLICE))
        if not args.no_cpu:
            log("cpu baseline of the two-species oracle (one core)")
            r = _run_workers([dict(kind="ions", n_inst=args.ions_inst, n_xi=args.ions_xi, which=0,
                                   m_i=ION_MASS_H, budget=args.cpu_budget)], args.cpu_budget)[0]
            n_r, n_s, n_w = r["parts"][0]
            out["mobile_ions"]["cpu_baseline"] = dict(
                value=r["done"] / (r["t1"] - r["t0"]), unit="species-ring-slice updates/s", cores=1,
                kind="oracle", sample=f"two-species oracle, instance 0 of the batch ({n_r} rings), "
                                      f"slices 0-{n_s} of {n_w + 1}, {r['t1'] - r['t0']:.1f} s")
    if args.served_seconds > 0:
        # capacity: sustained ring-slice rate of the server on the request mix
        # while it is saturated: a backlog of about 1000 requests submitted at
        # once, measured while some still wait for admission (the drain at
        # the end, when the last large requests run alone, is not capacity)
        budget = int(args.served_budget_gib * (1 << 30))
        step_us = 20_000
        log("served: capacity")
        specs, build = W.config4_stream(seed=40, rate=1000.0, duration=1.0)
        srv = wake.WakeServer(device_bytes=budget, slices_per_step=100_000, step_us=step_us,
                              stream=stream)
        for t, k in specs:
            srv.submit_instance(build(k))
        t0 = time.perf_counter()
        srv.step()                                   # first admissions
        w0, c0 = srv.stats()["ring_slices"], time.perf_counter()
        while time.perf_counter() - c0 < 8.0 and srv.stats()["queued"] > 0:
            srv.step()
            for t in srv.ready():
                srv.result(t)
        capacity = (srv.stats()["ring_slices"] - w0) / (time.perf_counter() - c0)
        srv.close()
        rate = args.served_rate or 0.85 * capacity / C4_MEAN_WORK
        log(f"served: capacity {capacity:.3e} ring-slices/s -> run at {rate:.1f} requests/s")
        run = served_run(wake, W, stream, rate, args.served_seconds, budget, step_us)
        offered = 2000.0 * C4_MEAN_WORK
        out["served"] = dict(
            workload="served Poisson stream, ring counts logU[500,50000], slices U[500,8000]",
            step_ms=step_us / 1e3,
            capacity_ring_slices_per_s=capacity,
            offered_at_2000_per_s=offered, stable_at_2000_per_s=bool(offered < capacity),
            max_sustainable_rate_per_s=capacity / C4_MEAN_WORK, **run)
    if args.large:
        # the large single instances on the cooperative (multi-workgroup) path,
        # in the layout the autotuner chose for their ring counts (or the
        # default layout without it); the first eighth of each window, before
        # the drivers disturb the order, gives the per-slice latency floor
        log("large instances")
        big = {}
        for name, mk in (("blowout 20000 rings x 4000 slices", W.config2),
                         ("laser 200000 rings x 8000 slices", W.config5)):
            inst = mk()
            s = wake.WakeSolver.from_instance(inst, stream=stream)
            s.wake_prepare()
            g, c = s.layout()
            torch.cuda.synchronize()
            q = inst.n_xi // 8
            t1 = time.perf_counter()
            s.wake_solve(0, q)
            s.wake_sync()
            tq = time.perf_counter() - t1
            s.wake_solve(q, inst.n_xi - q)
            s.wake_sync()
            dt = time.perf_counter() - t1
            brk = s.wake_status()[0]
            cnt = s.wake_counters()
            s.close()
            rate = inst.ring_slices / dt
            big[name] = dict(workgroups=g, rings_per_thread=c, seconds=dt, breakdown_slice=brk,
                             ring_slice_updates_per_s=rate, us_per_slice=dt / inst.n_xi * 1e6,
                             floor_us_per_slice=tq / q * 1e6,
                             roofline_frac=ALG_BYTES_PER_RING_SLICE * rate / PEAK_HBM,
                             fixups_per_slice=cnt["fixups"] / inst.n_xi,
                             meetings_per_slice=cnt["meetings"] / inst.n_xi)
        out["large_instances"] = big
    if not args.no_cpu:
        log("cpu baseline")
        out["cpu_baseline"] = cpu_baseline(args.n_inst, args.n_xi, args.cpu_budget)
        log("cpu baselines of the single-instance workloads (one core each)")
        out["cpu_baseline_single_core"] = cpu_single_core(args.cpu_budget)
    batch.close()
    for s in solvers + plain_solvers:
        s.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
