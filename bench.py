"""Benchmark of the liquid-gas-solid LBM hot path on one MI355X.

Workload (the configuration the headline metric is quoted on): a 128^3
basin, tau 0.55, gravity 5e-6, liquid depth 64, with a 32x32x16 box of
density 0.5 released at 20 deg heel about x (roll only).  One "step" is one
pass of the whole hot path: body remap, fused stream/collide/boundary/mass-
exchange/momentum-exchange sweep, interface conversions, force reduction and
the host rigid-body update feeding the next remap.  Inputs are synthetic and
resident in HBM before the timed region.

Prints one JSON line.  `value` is MLUPS over all cells of the FP32-storage
run; `fp16` repeats the timed run with FP16 deviation storage.  `roofline`
prices the dominant kernel (the sweep) with its algorithmic bytes against
the 8 TB/s HBM peak, its duration measured with HIP events around every
sweep launch inside the timed region.  `cpu_baseline` times the FP64 oracle
on the host on a bounded sample of the same workload.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "MLUPS + % of HBM roofline (FP32 vs FP16-storage) at ≤1% righting-moment error"
HBM_PEAK_GBS = 8000.0


def algorithmic_bytes(types, storage_bytes, n_boundary):
    """Bytes one sweep must move: liquid cells read and write 19 populations
    plus their flag; interface cells also read/write mass (hi, lo) and write
    the fill level; gas and obstacle cells cost their flag byte.  Split by
    kernel: the bulk kernel streams the liquid cells it keeps and reads every
    other flag; the boundary kernel handles the n_boundary listed cells (all
    interface cells and the liquid cells next to gas or a body)."""
    n_liq = int((types == 1).sum())
    n_if = int((types == 2).sum())
    n_other = int(types.size - n_liq - n_if)
    per_liq = 38 * storage_bytes + 1
    liq_bnd = max(0, n_boundary - n_if)
    bulk = (n_liq - liq_bnd) * per_liq + (types.size - n_liq + liq_bnd) * 1
    boundary = liq_bnd * (per_liq - 1) + n_if * (per_liq - 1 + 20)
    total = n_liq * per_liq + n_if * (per_liq + 20) + n_other * 1
    return dict(total=total, bulk=bulk, boundary=boundary), dict(liq=n_liq, iface=n_if, other=n_other,
                                                                  boundary_list=n_boundary)


def run_gpu(storage, steps, warmup):
    import numpy as np
    import torch

    from paper_1201_0351_amd import lbm
    from paper_1201_0351_amd import workloads as W

    w = W.config2(20.0, released=True, storage=storage)
    cfg = w["lattice"]
    L = lbm.Lattice(dict(cfg, max_bodies=1))
    # free body: the library runs the host rigid-body update after every step
    L.set_body(0, dict(w["bodies"][0], fixed=0, dof=w["dof"]))
    L.step(max(1, warmup))
    types = L.types()
    alg_bytes, counts = algorithmic_bytes(types, 4 if storage == "fp32" else 2, L.boundary_cells())
    L.sync()
    torch.cuda.synchronize()
    L.enable_kernel_timing(True)
    t0 = time.perf_counter()
    L.step(steps)
    L.sync()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    F, T = L.body_forces(0)
    body = L.get_body(0)
    bulk_ms, launches = L.kernel_time(0)
    bnd_ms, _ = L.kernel_time(1)
    L.enable_kernel_timing(False)
    n = L.ncells()
    dt = t1 - t0
    res = dict(value=n * steps / dt / 1e6, ms_per_step=1e3 * dt / steps, cells=n, counts=counts,
               bulk_ms=bulk_ms / max(1, launches), boundary_ms=bnd_ms / max(1, launches), alg_bytes=alg_bytes)
    q = body["quat"]
    heel = math.degrees(2.0 * math.atan2(q[1], q[0]))
    res["body"] = dict(heel_deg=heel, torque_x=float(T[0]), force_z=float(F[2]))
    L.close()
    return res


def cpu_baseline(target_s=15.0):
    """The FP64 oracle on the host cores: the same workload (128^3, box held at
    20 deg), timed over as many steps as fit in about target_s seconds."""
    from oracle.oracle import Oracle
    from paper_1201_0351_amd import workloads as W

    threads = min(16, os.cpu_count() or 1)
    w = W.config2(20.0, released=False)
    cfg = w["lattice"]
    o = Oracle(cfg["nx"], cfg["ny"], cfg["nz"], cfg["tau"], accel=cfg["accel"], eps=cfg["eps"], threads=threads)
    o.init_basin(cfg["fill_height"])
    b = w["bodies"][0]
    o.set_body(0, b["half"], b["pos"], b["quat"], b["vel"], b["omega"], b["density"], 1)
    o.step(1)  # mapping + first step, untimed
    t0 = time.perf_counter()
    o.step(1)
    one = time.perf_counter() - t0
    k = max(1, min(50, int(target_s / max(one, 1e-3)) - 1))
    t0 = time.perf_counter()
    o.step(k)
    dt = time.perf_counter() - t0
    n = o.ncells
    steps = k + 1
    return dict(value=n * steps / (dt + one) / 1e6, unit="MLUPS", cores=threads, kind="oracle",
                sample="%d steps of the 128^3 heeled-box basin (box held), FP64, %d OpenMP threads" % (steps, threads))


def copy_probe(mib):
    """A fill (writes 4n bytes) then five copies (read 4n, write 4n bytes each)
    of n float32: the kernels whose counter readings convert the profiler's
    FETCH_SIZE / WRITE_SIZE into HBM bytes."""
    import torch

    n = mib * (1 << 20) // 4
    a = torch.empty(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1.0)
    for _ in range(5):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes_per_copy": 4 * n}))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--no-fp16", action="store_true", help="skip the FP16-storage run")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run a plain fill and device copy of MIB MiB (calibrates the HBM byte counters)")
    args = ap.parse_args()
    if args.copy_probe:
        copy_probe(args.copy_probe)
        return
    if args.gpus != 1:
        print("bench.py: this build runs on one GPU only (the workload is a single-GPU lattice); "
              "--gpus %d is not supported" % args.gpus, file=sys.stderr)
        sys.exit(2)

    from oracle import analytic as A

    r32 = run_gpu("fp32", args.steps, args.warmup)
    print("fp32: %.1f MLUPS, %.4f ms/step, bulk %.4f ms, boundary %.4f ms" % (
        r32["value"], r32["ms_per_step"], r32["bulk_ms"], r32["boundary_ms"]), file=sys.stderr, flush=True)
    achieved = r32["alg_bytes"]["bulk"] / (r32["bulk_ms"] * 1e-3) / 1e9
    sweep_gbs = r32["alg_bytes"]["total"] / ((r32["bulk_ms"] + r32["boundary_ms"]) * 1e-3) / 1e9
    out = {
        "metric": METRIC,
        "value": round(r32["value"], 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(r32["ms_per_step"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "basin 128^3, tau 0.55, g 5e-6, depth 64, box 32x32x16 rho_s 0.5 released at "
                               "20 deg heel (roll only), FP32 deviation storage",
                   "cells": r32["cells"], "cell_types": r32["counts"]},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                     "kernel": "k_sweep_bulk<float,64>", "alg_bytes_per_launch": r32["alg_bytes"]["bulk"],
                     "avg_launch_ms": round(r32["bulk_ms"], 5),
                     "sweep_both_kernels": {"alg_bytes": r32["alg_bytes"]["total"],
                                            "avg_ms": round(r32["bulk_ms"] + r32["boundary_ms"], 5),
                                            "achieved": round(sweep_gbs, 1),
                                            "frac": round(sweep_gbs / HBM_PEAK_GBS, 4)}},
    }
    heel = r32["body"]["heel_deg"]
    ana = A.righting_moment_polygon(32, 16, 32, math.radians(heel), 5e-6, zw=0.0)
    out["body"] = dict(r32["body"], analytic_righting_moment=ana,
                       note="dynamic roll; measured -T_x vs the static curve at the current heel")
    if not args.no_fp16:
        r16 = run_gpu("fp16", args.steps, args.warmup)
        a16 = r16["alg_bytes"]["bulk"] / (r16["bulk_ms"] * 1e-3) / 1e9
        out["fp16"] = {"value": round(r16["value"], 1), "ms_per_step": round(r16["ms_per_step"], 4),
                       "bulk_roofline_frac": round(a16 / HBM_PEAK_GBS, 4), "bulk_achieved_GBs": round(a16, 1),
                       "bulk_avg_launch_ms": round(r16["bulk_ms"], 5),
                       "boundary_avg_launch_ms": round(r16["boundary_ms"], 5), "body": r16["body"]}
        print("fp16: %.1f MLUPS" % r16["value"], file=sys.stderr, flush=True)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out))


if __name__ == "__main__":
    main()
