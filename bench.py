"""Benchmark of the liquid-gas-solid LBM hot path on one MI355X.

Workload (the configuration the headline metric is quoted on): a 128^3
basin, tau 0.55, gravity 5e-6, liquid depth 64, with a 32x32x16 box of
density 0.5 released at 20 deg heel about x (roll only).  One "step" is one
pass of the whole hot path: body remap, fused stream/collide/boundary/mass-
exchange/momentum-exchange sweep, interface conversions, force reduction and
the rigid-body update feeding the next remap.  Inputs are synthetic and
resident in HBM before the timed region.

Prints one JSON line.  `value` is MLUPS over all cells of the FP32-storage
run with the rigid-body update on the device; `fp16` repeats the timed run
with FP16 deviation storage, `host_body_update` with the update on the host.
`roofline` prices the dominant kernel (the bulk sweep) with its algorithmic
bytes against the 8 TB/s HBM peak, its duration measured with HIP events
around every launch inside the timed region; `traffic` is the HBM bytes per
launch the profiler counted (profiles/k_sweep_bulk_basin128_traffic.txt),
reported only while the kernel source is the one that was profiled.
`righting_moment` holds the box at the heel angles of the oracle's golden
run and compares the averaged -T_x with the FP64 oracle's values
(tests/golden/righting_moment_128.json).  `cpu_baseline` times the FP64
oracle on the host on a bounded sample of the same workload.

Side experiments, each printed as JSON instead of the benchmark line:
`--free-advection` (the sphere in the moving-wall channel, for every tau and
wall speed of the paper's sweep), `--laplace` (resting droplets with surface
tension against Laplace's law), `--copy-probe MIB` (a plain device copy that
calibrates the HBM byte counters).
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "MLUPS + % of HBM roofline (FP32 vs FP16-storage) at ≤1% righting-moment error"
HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_sweep_bulk_basin128_traffic.txt")
GOLDEN_RM = os.path.join(ROOT, "tests", "golden", "righting_moment_128.json")
SWEEP_SOURCES = ("paper_1201_0351_amd/csrc/k_sweep.hip", "paper_1201_0351_amd/csrc/lgs_internal.h")


def sweep_source_hash():
    h = hashlib.sha256()
    for p in SWEEP_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def profiled_traffic(storage):
    """HBM bytes per bulk-sweep launch from the committed counter summary,
    if it was taken on the current kernel source; else None."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    vals = {}
    with open(TRAFFIC_FILE) as f:
        for line in f:
            if ":" in line and not line.startswith(" "):
                k, v = line.split(":", 1)
                vals[k.strip()] = v.strip()
    if vals.get("source_sha256_16") != sweep_source_hash():
        return None
    v = vals.get("traffic_bytes_per_launch_%s" % storage)
    return int(float(v)) if v else None


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


def run_gpu(storage, steps, warmup, host_update=0, timing=True):
    import torch

    from paper_1201_0351_amd import lbm
    from paper_1201_0351_amd import workloads as W

    w = W.config2(20.0, released=True, storage=storage)
    cfg = dict(w["lattice"], max_bodies=1, host_body_update=host_update)
    L = lbm.Lattice(cfg)
    # free body: the rigid-body update runs after every step
    L.set_body(0, dict(w["bodies"][0], fixed=0, dof=w["dof"]))
    L.step(max(1, warmup))
    types = L.types()
    alg_bytes, counts = algorithmic_bytes(types, 4 if storage == "fp32" else 2, L.boundary_cells())
    L.sync()
    torch.cuda.synchronize()
    # plain timed run (no events), then the same number of steps with the
    # sweep kernels bracketed by HIP events
    t0 = time.perf_counter()
    L.step(steps)
    L.sync()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    n = L.ncells()
    res = dict(value=n * steps / dt / 1e6, ms_per_step=1e3 * dt / steps, cells=n, counts=counts, alg_bytes=alg_bytes)
    if timing:
        L.enable_kernel_timing(True)
        L.step(steps)
        bulk_ms, launches = L.kernel_time(0)
        bnd_ms, _ = L.kernel_time(1)
        L.enable_kernel_timing(False)
        res.update(bulk_ms=bulk_ms / max(1, launches), boundary_ms=bnd_ms / max(1, launches))
    F, T = L.body_forces(0)
    body = L.get_body(0)
    q = body["quat"]
    res["body"] = dict(heel_deg=math.degrees(2.0 * math.atan2(q[1], q[0])), torque_x=float(T[0]),
                       force_z=float(F[2]))
    L.close()
    return res


def righting_moment(storage):
    """Held box at the golden heel angles: -T_x averaged like the oracle's
    golden run (every `every` steps over the last `window` of `steps`)."""
    from paper_1201_0351_amd import lbm
    from paper_1201_0351_amd import workloads as W

    if not os.path.exists(GOLDEN_RM):
        return None
    with open(GOLDEN_RM) as f:
        gold = json.load(f)
    out = []
    for run in gold["runs"]:
        w = W.config2(run["heel_deg"], released=False, storage=storage)
        L = lbm.Lattice(dict(w["lattice"], max_bodies=1))
        L.set_body(0, w["bodies"][0])
        done, samples = 0, []
        while done < run["steps"]:
            k = min(run["every"], run["steps"] - done)
            L.step(k)
            done += k
            if done > run["steps"] - run["window"]:
                samples.append(-L.body_forces(0)[1][0])
        L.close()
        ms = sum(samples) / len(samples)
        out.append(dict(heel_deg=run["heel_deg"], m_s=ms, m_s_oracle=run["m_s"],
                        rel_err=abs(ms - run["m_s"]) / abs(run["m_s"]), analytic=run["analytic_polygon"]))
    return out


def _timed(L, steps, warmup):
    import torch

    L.step(max(1, warmup))
    L.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    L.step(steps)
    L.sync()
    torch.cuda.synchronize()
    return time.perf_counter() - t0


def run_batch(storage, steps, warmup, batched=True, graph=False):
    """48 heeled-box instances of uneven size (64^3 .. 160x128x128), held, in
    one context: one launch per kernel for all of them (or one per instance
    with batched=False)."""
    from paper_1201_0351_amd import lbm
    from paper_1201_0351_amd import workloads as W

    w = W.config4(storage=storage)
    insts = w["instances"]
    L = lbm.Lattice([dict(i["lattice"], max_bodies=1) for i in insts])
    for k, i in enumerate(insts):
        L.set_body(0, i["bodies"][0], inst=k)
    L.set_tuning(batched=int(batched), use_graph=int(graph))
    L.step(2)
    tile, tune_ms = L.autotune(4)
    dt = _timed(L, steps, warmup)
    cells = sum(L.ncells(k) for k in range(len(insts)))
    L.close()
    return dict(instances=len(insts), cells=cells, steps=steps, ms_per_step=round(1e3 * dt / steps, 4),
                aggregate_mlups=round(cells * steps / dt / 1e6, 1),
                instance_steps_per_s=round(len(insts) * steps / dt, 1),
                instances_per_s=round(len(insts) / (w["steps"] * dt / steps), 3),
                note="instances_per_s: the %d-step heel sweep of all instances per second" % w["steps"],
                batched=batched, graph=graph, autotuned_tile_x=tile)


def run_single(workload, steps, warmup, free=False):
    from paper_1201_0351_amd import lbm

    L = lbm.Lattice(dict(workload["lattice"], max_bodies=1))
    b = dict(workload["bodies"][0])
    if free:
        b.update(fixed=0, dof=workload["dof"])
    L.set_body(0, b)
    dt = _timed(L, steps, warmup)
    n = L.ncells()
    L.close()
    return dict(cells=n, steps=steps, ms_per_step=round(1e3 * dt / steps, 4), mlups=round(n * steps / dt / 1e6, 1))


def other_configs(steps, warmup):
    from paper_1201_0351_amd import workloads as W

    out = {}
    out["batch48_heel_sweep"] = {st: run_batch(st, steps, warmup) for st in ("fp32", "fp16")}
    out["batch48_heel_sweep"]["fp32_one_launch_per_instance"] = run_batch("fp32", steps, warmup, batched=False)
    out["batch48_heel_sweep"]["fp32_graph"] = run_batch("fp32", steps, warmup, graph=True)
    out["basin256x192x192_box64x64x32_heel20_held"] = {st: run_single(W.config3(20.0, st), steps, warmup)
                                                      for st in ("fp32", "fp16", "bf16")}
    out["channel512x256x256_box48x24x24_free"] = {st: run_single(W.config5(st), steps, warmup, free=True)
                                                  for st in ("fp32", "fp16")}
    return out


# The paper's sphere velocities in the free advection channel (Table
# tab:velocities, g = 1e-5; None: not evaluated there because the empty
# channel showed spurious currents).
PAPER_TABLE_VELOCITIES = {
    0.62: (1.1e-4, None, None, None),
    0.8: (1.05e-4, 5.5e-5, 3.0e-5, 2.0e-5),
    1.1: (1.01e-4, 5.15e-5, 2.8e-5, 1.3e-5),
    1.7: (1.0e-4, 5.05e-5, 2.55e-5, 1.1e-5),
}


def free_advection(steps, window, every=100):
    """Sec. 3.2 free advection test: for every (tau, u) of the paper's sweep,
    the liquid starts at rest, the moving walls drive it, and the sphere's
    x velocity is averaged over the last `window` steps.  The paper's values
    are printed beside for context (its scheme differs in the readings listed
    in the design notes)."""
    from paper_1201_0351_amd import lbm
    from paper_1201_0351_amd import workloads as W

    rows = []
    for tau in W.FREE_ADVECTION_TAUS:
        for j, u in enumerate(W.FREE_ADVECTION_SPEEDS):
            w = W.free_advection(tau, u)
            L = lbm.Lattice(dict(w["lattice"], max_bodies=1))
            b = dict(w["bodies"][0], dof=w["dof"])
            L.set_body(0, b)
            t0 = time.perf_counter()
            L.step(steps - window)
            vx = []
            for _ in range(window // every):
                L.step(every)
                vx.append(float(L.get_body(0)["vel"][0]))
            dt = time.perf_counter() - t0
            L.close()
            vm = sum(vx) / len(vx)
            rows.append(dict(tau=tau, u=u, sphere_vx=vm, ratio=vm / u, vx_min=min(vx), vx_max=max(vx),
                             paper=PAPER_TABLE_VELOCITIES[tau][j], seconds=round(dt, 2)))
            print("tau %.2f u %.1e: sphere vx %.4e (ratio %.3f), paper %s" % (
                tau, u, vm, vm / u, PAPER_TABLE_VELOCITIES[tau][j]), file=sys.stderr, flush=True)
    return dict(experiment="free advection, 60x40x30 channel, moving walls, free sphere d = 12, rho_s 0.5, "
                           "g 1e-5, surface z = 19.5, start at rest",
                steps=steps, window=window, rows=rows)


LAPLACE_RADII = (8.0, 16.0, 24.0, 32.0)
# D3Q19 rest weights in the link order of Sec. 2.1 (centre, six axis links,
# twelve diagonals): the populations of fluid at rest with rho = 1
LATTICE_WEIGHTS = (1.0 / 3.0,) + (1.0 / 18.0,) * 6 + (1.0 / 36.0,) * 12


def laplace(steps, sigma=1e-3, n=128, every=200):
    """Sec. 2.2 Laplace pressure on the GPU path: a resting liquid droplet of
    radius R in gas on a periodic n^3 lattice (tau 1, no gravity, fills from
    the sphere's volume fractions) relaxes to rho_L - rho_G = 6 sigma / R
    (p = rho / 3).  For each radius the liquid density jump is averaged over
    the last quarter of the run and set against 6 sigma / R_eq, R_eq the
    radius of the liquid volume; the largest speed (spurious currents) is
    reported beside."""
    from paper_1201_0351_amd import lbm
    from paper_1201_0351_amd import workloads as W

    rows = []
    for R in LAPLACE_RADII:
        shape = (n, n, n)
        t, phi = W.droplet(shape, R, (n / 2 + 0.3, n / 2 - 0.2, n / 2 + 0.1))
        f = np.zeros((19,) + t.shape)
        fl = (t == W.LIQ) | (t == W.IF)
        for i, wi in enumerate(LATTICE_WEIGHTS):
            f[i][fl] = wi
        L = lbm.Lattice(dict(nx=n, ny=n, nz=n, tau=1.0, accel=(0.0, 0.0, 0.0), fill_height=0.0, periodic=7,
                             surface_tension=sigma, max_bodies=1))
        L.write(lbm.FIELD_FLAGS, t)
        L.write(lbm.FIELD_POP, f)
        L.write(lbm.FIELD_PHI, phi)
        L.write(lbm.FIELD_MASS, np.where(t == W.IF, phi, 0.0))
        t0 = time.perf_counter()
        L.step(steps - steps // 4)
        acc = []
        for _ in range(max(1, (steps // 4) // every)):
            L.step(every)
            tt = L.types()
            acc.append(float(L.read(lbm.FIELD_RHO)[tt == W.LIQ].mean() - 1.0))
        L.sync()
        dt = time.perf_counter() - t0
        tt = L.types()
        ph = L.phi()
        vol = float((tt == W.LIQ).sum() + ph[tt == W.IF].sum())
        req = (3.0 * vol / (4.0 * math.pi)) ** (1.0 / 3.0)
        vel = L.read(lbm.FIELD_VEL)
        fluid = (tt == W.LIQ) | (tt == W.IF)
        umax = float(np.sqrt((vel ** 2).sum(axis=0))[fluid].max())
        L.close()
        jump = sum(acc) / len(acc)
        rows.append(dict(radius=R, r_eq=round(req, 4), drho=jump, laplace=6.0 * sigma / req,
                         ratio=jump / (6.0 * sigma / req), u_max=umax, seconds=round(dt, 2)))
        print("R %.0f: rho_L - rho_G %.4e, 6 sigma / R_eq %.4e, ratio %.4f, u_max %.2e" % (
            R, jump, 6.0 * sigma / req, jump / (6.0 * sigma / req), umax), file=sys.stderr, flush=True)
    return dict(experiment="Laplace pressure of resting droplets, %d^3 periodic, tau 1, sigma %g" % (n, sigma),
                steps=steps, rows=rows)


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


def roofline(r, storage):
    achieved = r["alg_bytes"]["bulk"] / (r["bulk_ms"] * 1e-3) / 1e9
    sweep_gbs = r["alg_bytes"]["total"] / ((r["bulk_ms"] + r["boundary_ms"]) * 1e-3) / 1e9
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": profiled_traffic(storage),
            "kernel": "k_sweep_bulk<%s,64>" % ("float" if storage == "fp32" else "__half"),
            "alg_bytes_per_launch": r["alg_bytes"]["bulk"], "avg_launch_ms": round(r["bulk_ms"], 5),
            "sweep_both_kernels": {"alg_bytes": r["alg_bytes"]["total"],
                                   "avg_ms": round(r["bulk_ms"] + r["boundary_ms"], 5),
                                   "achieved": round(sweep_gbs, 1), "frac": round(sweep_gbs / HBM_PEAK_GBS, 4)}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--no-fp16", action="store_true", help="skip the FP16-storage run")
    ap.add_argument("--no-extra", action="store_true",
                    help="only the timed runs (no host-update run, no righting moment)")
    ap.add_argument("--free-advection", action="store_true",
                    help="only run the paper's free advection sweep (Table tab:velocities) and print it as JSON")
    ap.add_argument("--laplace", action="store_true",
                    help="only run resting droplets with surface tension (Laplace's law) and print them as JSON")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run a plain fill and device copy of MIB MiB (calibrates the HBM byte counters)")
    args = ap.parse_args()
    if args.copy_probe:
        copy_probe(args.copy_probe)
        return
    if args.laplace:
        print(json.dumps(laplace(steps=args.steps)))
        return
    if args.free_advection:
        print(json.dumps(free_advection(steps=args.steps, window=max(100, args.steps // 4))))
        return
    if args.gpus != 1:
        print("bench.py: this build runs on one GPU only (the workload is a single-GPU lattice); "
              "--gpus %d is not supported" % args.gpus, file=sys.stderr)
        sys.exit(2)

    r32 = run_gpu("fp32", args.steps, args.warmup)
    print("fp32: %.1f MLUPS, %.4f ms/step, bulk %.4f ms, boundary %.4f ms" % (
        r32["value"], r32["ms_per_step"], r32["bulk_ms"], r32["boundary_ms"]), file=sys.stderr, flush=True)
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
                               "20 deg heel (roll only), FP32 deviation storage, rigid-body update on the device",
                   "cells": r32["cells"], "cell_types": r32["counts"]},
        "roofline": roofline(r32, "fp32"),
    }
    from oracle import analytic as A

    heel = r32["body"]["heel_deg"]
    out["body"] = dict(r32["body"], analytic_righting_moment=A.righting_moment_polygon(
        32, 16, 32, math.radians(heel), 5e-6, zw=0.0), note="dynamic roll; measured -T_x vs the static curve")
    if not args.no_fp16:
        r16 = run_gpu("fp16", args.steps, args.warmup)
        out["fp16"] = {"value": round(r16["value"], 1), "ms_per_step": round(r16["ms_per_step"], 4),
                       "roofline": roofline(r16, "fp16"), "body": r16["body"]}
        print("fp16: %.1f MLUPS" % r16["value"], file=sys.stderr, flush=True)
    if not args.no_extra:
        steps_h = max(1, args.steps // 4)
        rh = run_gpu("fp32", steps_h, args.warmup, host_update=1, timing=False)
        out["host_body_update"] = {"value": round(rh["value"], 1), "ms_per_step": round(rh["ms_per_step"], 4),
                                   "steps": steps_h, "body": rh["body"]}
        print("fp32 host update: %.1f MLUPS" % rh["value"], file=sys.stderr, flush=True)
        rm = {}
        for st in ("fp32", "fp16"):
            v = righting_moment(st)
            if v is not None:
                rm[st] = v
        if rm:
            out["righting_moment"] = dict(rm, reference="FP64 oracle, held box, tests/golden/righting_moment_128.json",
                                          max_rel_err={k: round(max(x["rel_err"] for x in v), 5)
                                                       for k, v in rm.items()})
        out["other_configs"] = other_configs(max(50, args.steps // 10), 20)
        print("other configs done", file=sys.stderr, flush=True)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out))


if __name__ == "__main__":
    main()
