#!/usr/bin/env python3
"""Z4c zone-cycles per second on one MI355X.

Workload (default): 64 MeshBlocks of 32^3 (128^3 zones, dx = 0.25 on
[-16,16]^3), FP64, 6th-order finite differences, Brill-Lindquist puncture
M = 1 at the origin, outflow boundaries, classic RK4 with CFL 0.25.  Inputs
are synthetic and resident in HBM before timing starts.

Prints one JSON line: the whole-job ZCPS (interior zones x RK4 steps / s),
the HBM roofline of the dominant kernel (the fused RHS + RK4 stage kernel)
timed live with HIP events on its own stream, and the CPU oracle timed on
the host as a baseline.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Z4c zone-cycles/s (RK4, 6th-order FD), FP64 vs batched/FP32; % HBM roofline"
HBM_PEAK_GBS = 8000.0
# algorithmic bytes per zone per stage-kernel launch (classic RK4 on four
# registers, fused stage): 16 register accesses per field per RK4 step,
# 22 fields, over 4 launches; FP32 storage with an FP64 accumulator moves
# 88 bytes per field per step.
BYTES_PER_ZONE_LAUNCH = {"fp64": 16 * 22 * 8 / 4, "fp32": 88 * 22 / 4}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="bl64x32")
    ap.add_argument("--precision", choices=["fp64", "fp32"], default="fp64")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--tile", default=None,
                    help="fixed stage-kernel launch instead of the autotuner's choice: variant "
                         "index 0-3 (8x8x4, 16x4x4, 8x4x8, 16x8x2), suffix p = persistent")
    ap.add_argument("--profile-steps", type=int, default=5)
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the FP32 and batched multi-level measurements")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 1 GiB device copy (HBM counter calibration)")
    ap.add_argument("--summarize-pmc", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="turn two rocprofv3 --pmc runs (FETCH_SIZE, WRITE_SIZE) into "
                         "profiles/traffic_<workload>_<precision>.json and exit")
    return ap.parse_args()


def cpu_baseline(workload):
    """The oracle (single-threaded C, FP64) on a bounded sample of the same
    workload: three RK4 steps of a 2x2x2-block (64^3-zone) sub-mesh with the
    same cell size, order and data type (about 10-15 s on one core); ZCPS
    scaled per zone."""
    import oracle
    import z4c_inputs as zi
    mesh0, p, _, dt, _ = zi.workload(workload)
    n = int(mesh0.n[0])
    h = mesh0.dx0
    half = n * h
    mesh = zi.uniform_mesh((2, 2, 2), n, mesh0.g, (-half,) * 3, (half,) * 3, zi.BC_OUTFLOW)
    data = zi.brill_lindquist(mesh, [(1.0, (0.0, 0.0, 0.0))])
    om = oracle.OracleMesh(mesh)
    regs = oracle.Registers(om, data)
    nsteps = 3
    t0 = time.perf_counter()
    oracle.rk4_steps(regs, p, dt, nsteps)
    sec = time.perf_counter() - t0
    out = {"value": mesh.zones() * nsteps / sec, "unit": "zone-cycles/s", "cores": 1, "kind": "oracle",
           "sample": f"{nsteps} RK4 steps of 8 blocks of {n}^3 (dx={h}, order {p['fd_order']}, "
                     f"Brill-Lindquist) on one host core, {sec:.1f} s"}
    # all usable host cores (at most 16, one GPU's share): the same sample,
    # one independent copy per thread (the oracle's C calls release the GIL)
    import concurrent.futures as cf
    ncores = max(1, min(len(os.sched_getaffinity(0)), 16))

    def one(_):
        r = oracle.Registers(om, data)
        oracle.rk4_steps(r, p, dt, 1)

    t0 = time.perf_counter()
    with cf.ThreadPoolExecutor(max_workers=ncores) as ex:
        list(ex.map(one, range(ncores)))
    sec_all = time.perf_counter() - t0
    out["all_cores"] = {"value": ncores * mesh.zones() / sec_all, "cores": ncores,
                        "sample": f"one RK4 step of the same 8 blocks per thread, {ncores} threads, "
                                  f"{sec_all:.1f} s"}
    return out


def _pmc_rows(d, counter):
    """(kernel name, counter value in KiB) per dispatch, in dispatch order,
    from a rocprofv3 csv run."""
    import csv
    import glob
    rows = []
    for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
        with open(f) as fh:
            for r in csv.DictReader(fh):
                if r.get("Counter_Name") == counter:
                    rows.append((int(r["Dispatch_Id"]), r.get("Kernel_Name", ""), float(r["Counter_Value"])))
    return [(k, v) for _, k, v in sorted(rows)]


def variant_key(chosen):
    """Launch label of a stage-kernel variant: tile shape, p = persistent."""
    from paper_2409_10383_amd import TILE_SHAPES
    return "x".join(str(v) for v in TILE_SHAPES[chosen // 2]) + ("p" if chosen % 2 else "")


def summarize_pmc(args):
    """HBM bytes per stage-kernel launch from FETCH_SIZE and WRITE_SIZE,
    each scaled by what the same counter reads for a 1 GiB device copy, for
    the launch variant the counter runs used (--tile, required).  Only the
    last 8 stage-kernel dispatches count: the four RK stages of the timed
    step and of the profiled step of a `--steps 1 --profile-steps 1` run.
    The figures of each variant are kept side by side in the file, which is
    started afresh when the kernel sources change."""
    if args.tile is None:
        raise SystemExit("--summarize-pmc needs the --tile the counter runs used")
    key = variant_key(2 * int(args.tile[0]) + (1 if args.tile.endswith("p") else 0))
    path = os.path.join(ROOT, "profiles", f"traffic_{args.workload}_{args.precision}.json")
    doc = {"workload": args.workload, "precision": args.precision, "kernel_source_hash": kernel_hash(),
           "variants": {}}
    if os.path.exists(path):
        with open(path) as f:
            old = json.load(f)
        if old.get("kernel_source_hash") == doc["kernel_source_hash"] and "variants" in old:
            doc["variants"] = old["variants"]
    out = {}
    total = 0.0
    for d, ctr in zip(args.summarize_pmc, ("FETCH_SIZE", "WRITE_SIZE")):
        rows = _pmc_rows(d, ctr)
        stage = [v for k, v in rows if "k_stage" in k][-8:]
        copy = [v for k, v in rows if ("copy" in k.lower() or "elementwise" in k.lower())
                and v > 0.5 * 1024 * 1024]
        if not stage or not copy:
            raise SystemExit(f"no k_stage or copy dispatches with {ctr} in {d}")
        factor = (1 << 30) / (max(copy) * 1024.0)
        kib = sum(stage) / len(stage)
        out[ctr] = {"stage_kib_per_dispatch": kib, "dispatches": len(stage), "copy_kib": max(copy),
                    "scale": factor, "bytes_per_launch": kib * 1024.0 * factor,
                    "kernel": [k for k, v in rows if "k_stage" in k][-1]}
        total += kib * 1024.0 * factor
    out["bytes_per_launch"] = total
    doc["variants"][key] = out
    doc["variants"] = dict(sorted(doc["variants"].items()))
    with open(path, "w") as f:
        json.dump(doc, f, indent=1)
    print(json.dumps({key: out}))


def copy_bandwidth():
    """Achievable HBM bandwidth: a timed 2 GiB device-to-device copy
    (2 GiB read + 2 GiB written), best of 5."""
    import torch
    a = torch.ones(1 << 28, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    best = None
    for _ in range(5):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        b.copy_(a)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        best = ms if best is None else min(best, ms)
    del a, b
    torch.cuda.empty_cache()
    return 2.0 * (1 << 31) / (best * 1e-3) / 1e9


def copy_calibration():
    import torch
    a = torch.ones(1 << 27, dtype=torch.float64, device="cuda")   # 1 GiB
    b = torch.empty_like(a)
    for _ in range(2):
        b.copy_(a)
    torch.cuda.synchronize()


def extra_runs(z4c, zi, torch):
    """Batched multi-level pack (512 blocks, 4 levels, 8th order, graph
    replay, autotuned tiles) and FP32 storage on the default workload."""
    out = {}
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        mesh, p, data, dt, _ = zi.workload("bbh512mixed")
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        for prec, name in ((z4c.FP64, "fp64"), (z4c.FP32_MIXED, "fp32")):
            pk = z4c.Pack(mesh, dict(p, graph=1), prec)
            pk.upload(z4c.REG_U, data)
            chosen, times = pk.autotune(reps=2, stream=s)
            pk.rk4_step(dt, 1, stream=s)
            s.synchronize()
            e0.record(s)
            pk.rk4_step(dt, 5, stream=s)
            e1.record(s)
            s.synchronize()
            ms = e0.elapsed_time(e1)
            out[f"batched_bbh512mixed_{name}"] = {
                "zcps": pk.zones * 5 / (ms * 1e-3), "zones": pk.zones, "blocks": int(mesh.nb),
                "levels": int(mesh.level.max()) + 1, "fd_order": 8, "graph": True,
                "tile_variant": chosen, "autotune_ms": [float(x) for x in times]}
            print(f"bench: batched {name} done", file=sys.stderr, flush=True)
            del pk
            torch.cuda.empty_cache()
        mesh, p, data, dt, _ = zi.workload("bl64x32")
        pk = z4c.Pack(mesh, p, z4c.FP32_MIXED)
        pk.upload(z4c.REG_U, data)
        chosen32, _ = pk.autotune(reps=3, stream=s)
        pk.rk4_step(dt, 2, stream=s)
        s.synchronize()
        e0.record(s)
        pk.rk4_step(dt, 10, stream=s)
        e1.record(s)
        s.synchronize()
        ms = e0.elapsed_time(e1)
        out["fp32_storage_bl64x32"] = {"zcps": pk.zones * 10 / (ms * 1e-3),
                                       "tile": "x".join(str(v) for v in z4c.TILE_SHAPES[chosen32 // 2]),
                                       "persistent": bool(chosen32 % 2)}
        del pk
        torch.cuda.empty_cache()
    return out


def main():
    args = parse()
    if args.summarize_pmc:
        summarize_pmc(args)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU "
              "halo exchange is not built.", file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_2409_10383_amd as z4c
    import z4c_inputs as zi

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    prec = z4c.FP64 if args.precision == "fp64" else z4c.FP32_MIXED
    mesh, p, data, dt, _ = zi.workload(args.workload)
    pack = z4c.Pack(mesh, p, prec)
    pack.upload(z4c.REG_U, data)
    stream = torch.cuda.current_stream()
    # tile shape and launch mode from the built-in autotuner (state unchanged)
    if args.tile is None:
        chosen, _ = pack.autotune(reps=3)
    else:
        chosen = 2 * int(args.tile[0]) + (1 if args.tile.endswith("p") else 0)
        pack.set_variant(chosen // 2, bool(chosen % 2))
    for _ in range(args.warmup):
        pack.rk4_step(dt, 1)
    torch.cuda.synchronize()

    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    pack.rk4_step(dt, args.steps)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    zcps = pack.zones * args.steps / (ms * 1e-3)

    # dominant kernel: per-launch duration from events around each launch
    pack.profile(True)
    pack.profile_read(reset=True)
    pack.rk4_step(dt, max(args.profile_steps, 1))
    st_ms, st_n, fill_ms, fill_n, _, _ = pack.profile_read(reset=True)
    pack.profile(False)
    avg_stage_s = st_ms / st_n * 1e-3
    bpl = BYTES_PER_ZONE_LAUNCH[args.precision] * pack.zones
    achieved = bpl / avg_stage_s / 1e9

    traffic = None
    tfile = os.path.join(ROOT, "profiles", f"traffic_{args.workload}_{args.precision}.json")
    if os.path.exists(tfile):
        with open(tfile) as f:
            t = json.load(f)
        if t.get("kernel_source_hash") == kernel_hash():
            traffic = t.get("variants", {}).get(variant_key(chosen), {}).get("bytes_per_launch")

    out = {
        "metric": METRIC,
        "value": zcps,
        "unit": "zone-cycles/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32+f64acc",
        "data": "synthetic",
        "config": {"workload": args.workload, "blocks": int(mesh.nb),
                   "block_cells": int(mesh.n[0]), "zones": pack.zones,
                   "fd_order": p["fd_order"], "ghosts": mesh.g, "dt": dt,
                   "tile": "x".join(str(v) for v in z4c.TILE_SHAPES[chosen // 2]),
                   "persistent": bool(chosen % 2),
                   "initial_data": "Brill-Lindquist M=1" if args.workload.startswith("bl") else args.workload},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": "k_stage (fused RHS + RK4 stage)",
                     "avg_launch_ms": st_ms / st_n, "launches": int(st_n),
                     "achievable_copy_GBs": None,
                     "ghost_fill_avg_ms": (fill_ms / fill_n) if fill_n else None},
    }
    if args.copy_calibration:
        # counter runs: the 1 GiB copy must be the largest copy of the run
        copy_calibration()
    else:
        out["roofline"]["achievable_copy_GBs"] = copy_bandwidth()
    if not args.no_extras:
        del pack
        torch.cuda.empty_cache()
        out["extras"] = extra_runs(z4c, zi, torch)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(args.workload)
    print(json.dumps(out), flush=True)


def kernel_hash():
    """Hash of the sources that decide the stage kernel's memory traffic:
    its own file, the host code that builds its work list and launches it,
    and every shared header."""
    import hashlib
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_2409_10383_amd", "csrc")
    for f in sorted(os.listdir(d)):
        if f in ("stage.hip", "capi.hip") or f.endswith(".hpp"):
            with open(os.path.join(d, f), "rb") as fh:
                h.update(fh.read())
    return h.hexdigest()[:16]


if __name__ == "__main__":
    main()
