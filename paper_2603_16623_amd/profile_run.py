"""Profiling driver: one replay of the batched march, or a plain device copy.

    python -m paper_2603_16623_amd.profile_run --n-inst 512 --n-xi 400
    python -m paper_2603_16623_amd.profile_run --n-inst 256 --n-xi 1000 --ion-mass 1836.15267
    python -m paper_2603_16623_amd.profile_run --copy-mib 1024

The first builds the batched workload (ring counts log-uniform in
[1000, 8000], geometric spacing, driver and witness beams), captures the
graph, replays it once untimed and once timed, and prints the rate.  The
same with --ion-mass marches electrons and mobile ions of that mass (two-species
contexts, the two-species marcher).  The last copies a device buffer of the given size once (torch copy kernel):
its FETCH_SIZE / WRITE_SIZE counters calibrate the march kernel's against a
known byte count.  Meant to run under rocprofv3.
"""
from __future__ import annotations

import argparse
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--n-inst", type=int, default=512)
    ap.add_argument("--n-xi", type=int, default=400)
    ap.add_argument("--tiling", type=str, default="")
    ap.add_argument("--copy-mib", type=int, default=0)
    ap.add_argument("--ion-mass", type=float, default=0.0,
                    help="mobile ions of this mass (electron masses); 0: immobile ions")
    args = ap.parse_args()

    import torch
    torch.cuda.set_device(0)
    ts = torch.cuda.Stream()
    torch.cuda.set_stream(ts)
    if args.copy_mib:
        n = args.copy_mib * (1 << 20) // 8
        a = torch.ones(n, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        print(f"copied {args.copy_mib} MiB", flush=True)
        return
    from paper_2603_16623_amd import wake, workloads as W
    wake.load()
    if args.tiling:
        nt, wpc = (int(x) for x in args.tiling.split(","))
        wake.wake_set_tiling(nt, wpc)
    insts = W.config3(n_inst=args.n_inst, n_xi=args.n_xi)
    species = 2 if args.ion_mass > 0 else 1
    work = species * sum(i.ring_slices for i in insts)
    st = ts.cuda_stream
    sol = [wake.WakeSolver(i.r0, i.dr, i.dxi, i.n_xi, i.sources, i.dens, stream=st,
                           ion_mass=args.ion_mass if args.ion_mass > 0 else None) for i in insts]
    for s in sol:
        s.wake_prepare()
    b = wake.WakeBatch(sol, stream=st)
    b.wake_batch_capture()
    b.wake_batch_replay()
    torch.cuda.synchronize()
    t = time.perf_counter()
    b.wake_batch_replay()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t
    unit = "species-ring-slice" if species == 2 else "ring-slice"
    print(f"batched {args.n_inst} x {args.n_xi} slices: {work} {unit}s, {dt * 1e3:.1f} ms, "
          f"{work / dt:.3e} {unit} updates/s", flush=True)
    b.close()
    for s in sol:
        s.close()


if __name__ == "__main__":
    main()
