"""Benchmark of the liquid-gas-solid LBM hot path on one MI355X.

Workload of the headline (the largest single-GPU configuration): a
512x256x256 open channel, periodic along x and y, walls at the bottom and
the top, liquid depth 128, tau 0.8, gravity 1e-5, a body-force drive for a
surface speed of 0.05 (the liquid starts on the half-Poiseuille profile),
and one free 48x24x24 box of density 0.6 advected along x in 6 DOF.  One
"step" is one pass of the whole hot path: body remap, fused stream / collide
/ boundary / mass-exchange / momentum-exchange sweep, interface conversions,
force reduction and the rigid-body update feeding the next remap.  Inputs
are synthetic and resident in HBM before the timed region.

The box sticks through the free surface and moves with it at 0.05 cells
per step.  After some 1500 steps the refilling of the cells it uncovers has
piled liquid up behind it (7 cells above the far level), the hydrostatic
head drives it faster than the flow and the run goes unstable near step
1800, on the FP64 oracle's rules as on the GPU (the paper reports this
refilling error for bodies sticking through the interface).  So every
timed window runs on a channel built afresh: 200 preparation steps (the
start-up transient), the warm-up steps, then K/5 timed steps; no lattice
runs longer than `steps_per_lattice`.

Prints one JSON line.  `value` is MLUPS over all cells of the FP32-storage
run with the rigid-body update on the device; `ms_per_step` is the median
over 5 windows of K/5 steps (each window bracketed by stream
synchronisation; `ms_windows` lists them).  `roofline` prices the dominant
kernel (the bulk sweep) with its algorithmic bytes against the 8 TB/s HBM
peak, its duration measured with HIP events attached to every one of its
dispatches over up to 500 steps of a further fresh channel (`kernels` gives
the boundary sweep too); `traffic` is the HBM
bytes per launch the profiler counted for the same kernel and workload
(profiles/k_sweep_bulk_channel512_traffic.txt), reported only while the
kernel source is the one that was profiled.  `channel` repeats the timed run
with FP16 and BF16 deviation storage and with the rigid-body update on the
host; `accuracy` compares the channel's body force and torque after four
steps with the FP64 oracle's, and `accuracy_basin256` those of the
256x192x192 held box after three (with the count of cells whose type
differs); `righting_moment` holds the 128^3 box at the heel angles of the
oracle's golden run and compares the averaged -T_x and the final cell types
(tests/golden/righting_moment_128.json); `other_configs` times the 128^3
basin (cache resident), the 256x192x192 held box and the 48-instance heel
sweep, whose righting moment of four instances is compared with the oracle's
(tests/golden/batch48_righting.json).  `cpu_baseline` times the FP64 oracle
on the host on a bounded sample of the headline workload, on all cores and
on one thread, and on two steps of the 256x192x192 basin.

Side experiments, each printed as JSON instead of the benchmark line:
`--free-advection` (the sphere in the moving-wall channel, for every tau and
wall speed of the paper's sweep), `--laplace` (resting droplets with surface
tension against Laplace's law), `--copy-probe MIB` (a plain device copy that
calibrates the HBM byte counters).  `--profile CASE` runs only one timed case
(for the profiler).
"""
import argparse
import hashlib
import json
import math
import os
import statistics
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "MLUPS + % of HBM roofline (FP32 vs FP16-storage) at ≤1% righting-moment error"
HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_sweep_bulk_channel512_traffic.txt")
GOLDEN_RM = os.path.join(ROOT, "tests", "golden", "righting_moment_128.json")
GOLDEN_BATCH = os.path.join(ROOT, "tests", "golden", "batch48_righting.json")
SWEEP_SOURCES = ("paper_1201_0351_amd/csrc/k_sweep.hip", "paper_1201_0351_amd/csrc/lgs_internal.h")
PREP_STEPS = 200
WINDOWS = 5
EVENT_STEPS = 500
TUNE_REPS = 16  # autotuner launches per candidate (candidates lie within a few percent)
STORAGE_BYTES = {"fp32": 4, "fp16": 2, "bf16": 2}
KERNEL_NAMES = {"fp32": "float", "fp16": "__half", "bf16": "__hip_bfloat16"}


def sweep_source_hash():
    h = hashlib.sha256()
    for p in SWEEP_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def profiled_traffic(storage):
    """HBM bytes per bulk-sweep launch on the channel from the committed
    counter summary, if it was taken on the current kernel source; else None."""
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


def _sync(L):
    import torch

    L.sync()
    torch.cuda.synchronize()


def _lattice(workload, storage, free, host_update):
    from paper_1201_0351_amd import lbm

    lat = dict(workload["lattice"], storage=storage)
    L = lbm.Lattice(dict(lat, max_bodies=1, host_body_update=host_update))
    b = dict(workload["bodies"][0])
    if free:
        b.update(fixed=0, dof=workload["dof"])
    L.set_body(0, b)
    return L


def run_case(workload, storage, steps, warmup, free=True, host_update=0, prep=0, timing=True, tune=True):
    """Time K = `steps` full steps of one instance in WINDOWS windows (each
    bracketed by synchronisation); then, with HIP events on the two sweep
    kernels, up to EVENT_STEPS more steps for the per-kernel times.  Every
    window (and the event-timed pass) runs on a lattice built afresh,
    prepared by `prep` steps, tuned as the autotuner chose on the first one
    and warmed up by `warmup` steps, so no lattice runs longer than
    prep + warmup + K / WINDOWS steps: the channel's surface-piercing box
    is only followed over its physically meaningful start (see the module
    docstring)."""
    tuned = None
    if tune:
        L = _lattice(workload, storage, free, host_update)
        if prep:
            L.step(prep)
        t = L.autotune(TUNE_REPS)
        tuned = dict(tile_x=t["tile_x"], stream_store=t["stream_store"], boundary_layout=t["boundary_layout"])
        L.close()

    def prepared():
        L = _lattice(workload, storage, free, host_update)
        if prep:
            L.step(prep)
        if tuned:
            L.set_tuning(**tuned)
        L.step(max(1, warmup))
        _sync(L)
        return L

    # exactly `steps` timed steps in WINDOWS windows of nearly equal length
    nwin = max(1, min(WINDOWS, steps))
    sizes = [steps // nwin + (1 if k < steps % nwin else 0) for k in range(nwin)]
    win = []
    for k, per in enumerate(sizes):
        L = prepared()
        t0 = time.perf_counter()
        L.step(per)
        _sync(L)
        win.append(1e3 * (time.perf_counter() - t0) / per)
        if k < nwin - 1:
            L.close()
    ms = statistics.median(win)
    n = L.ncells()
    types = L.types()
    alg, counts = algorithmic_bytes(types, STORAGE_BYTES[storage], L.boundary_cells())
    res = dict(value=n / ms / 1e3, ms_per_step=ms, ms_windows=[round(v, 5) for v in win], steps=sum(sizes),
               cells=n, counts=counts, alg_bytes=alg, tuning=tuned, steps_per_lattice=prep + max(1, warmup) + max(sizes))
    F, T = L.body_forces(0)
    bd = L.get_body(0)
    q = bd["quat"]
    res["body"] = dict(heel_deg=math.degrees(2.0 * math.atan2(q[1], q[0])), torque_x=float(T[0]),
                       force_z=float(F[2]), pos=[round(float(v), 4) for v in bd["pos"]],
                       vel=[round(float(v), 6) for v in bd["vel"]])
    L.close()
    if timing:
        L = prepared()
        L.enable_kernel_timing(True)
        L.step(max(1, min(steps, EVENT_STEPS)))
        _sync(L)
        bulk_ms, launches = L.kernel_time(0)
        bnd_ms, _ = L.kernel_time(1)
        L.enable_kernel_timing(False)
        L.close()
        res.update(bulk_ms=bulk_ms / max(1, launches), boundary_ms=bnd_ms / max(1, launches), event_launches=launches)
    return res


def kernel_rooflines(r, storage):
    """Per-kernel achieved bandwidth (algorithmic bytes / event-timed
    duration) of the two sweep kernels."""
    out = {}
    for k, key in (("bulk", "bulk_ms"), ("boundary", "boundary_ms")):
        gbs = r["alg_bytes"][k] / (r[key] * 1e-3) / 1e9
        out[k] = dict(avg_us=round(1e3 * r[key], 2), alg_bytes=r["alg_bytes"][k], achieved_gbs=round(gbs, 1),
                      frac=round(gbs / HBM_PEAK_GBS, 4))
    return out


def roofline(r, storage):
    achieved = r["alg_bytes"]["bulk"] / (r["bulk_ms"] * 1e-3) / 1e9
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": profiled_traffic(storage),
            "kernel": "k_sweep_bulk<%s>" % KERNEL_NAMES[storage],
            "alg_bytes_per_launch": r["alg_bytes"]["bulk"], "avg_launch_ms": round(r["bulk_ms"], 5)}


def summary(r, storage):
    return {"value": round(r["value"], 1), "ms_per_step": round(r["ms_per_step"], 4), "ms_windows": r["ms_windows"],
            "roofline": roofline(r, storage), "kernels": kernel_rooflines(r, storage), "tuning": r["tuning"],
            "steps_per_lattice": r["steps_per_lattice"], "body": r["body"]}


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
        mism = None
        if "final_types" in run:
            mism = int((L.types() != unpack_types(run["final_types"], L.shape())).sum())
        L.close()
        ms = sum(samples) / len(samples)
        out.append(dict(heel_deg=run["heel_deg"], m_s=ms, m_s_oracle=run["m_s"],
                        rel_err=abs(ms - run["m_s"]) / abs(run["m_s"]), analytic=run["analytic_polygon"],
                        type_mismatches=mism))
    return out


def unpack_types(s, shape):
    """Cell types stored by the golden scripts: four 2-bit codes per byte, zlib, base64."""
    import base64
    import zlib

    packed = np.frombuffer(zlib.decompress(base64.b64decode(s)), np.uint8)
    t = np.stack([(packed >> k) & 3 for k in (0, 2, 4, 6)], axis=1).ravel()
    return t[: int(np.prod(shape))].reshape(shape)


def batch_righting(storage):
    """The batched 48-instance context from its initial state for the
    golden's steps: the righting moment of the four instances the oracle ran
    alone (tests/golden/batch48_righting.json), averaged the same way."""
    from paper_1201_0351_amd import lbm
    from paper_1201_0351_amd import workloads as W

    if not os.path.exists(GOLDEN_BATCH):
        return None
    with open(GOLDEN_BATCH) as f:
        gold = json.load(f)
    insts = W.config4(storage=storage)["instances"]
    L = lbm.Lattice([dict(i["lattice"], max_bodies=1) for i in insts])
    for k, i in enumerate(insts):
        L.set_body(0, i["bodies"][0], inst=k)
    L.set_tuning(batched=1)
    samples = {r["instance"]: [] for r in gold["runs"]}
    done = 0
    while done < gold["steps"]:
        L.step(gold["every"])
        done += gold["every"]
        if done > gold["steps"] - gold["window"]:
            for k in samples:
                samples[k].append(-L.body_forces(0, inst=k)[1][0])
    L.close()
    out = []
    for r in gold["runs"]:
        ms = sum(samples[r["instance"]]) / len(samples[r["instance"]])
        row = dict(instance=r["instance"], shape=r["shape"], heel_deg=round(r["heel_deg"], 2), density=r["density"],
                   m_s=ms, m_s_oracle=r["m_s"], rel_err=abs(ms - r["m_s"]) / abs(r["m_s"]))
        if "m_s_noise_1e-7" in r:
            # the low deck edge just under the water: the oracle's own m_s
            # spreads over round-off-level noise (its runs from noisy starts)
            ens = [r["m_s"]] + r["m_s_noise_1e-7"]
            row.update(thin_film=True, oracle_range=[min(ens), max(ens)])
        out.append(row)
    return out


def _timed(L, steps, warmup):
    L.step(max(1, warmup))
    _sync(L)
    t0 = time.perf_counter()
    L.step(steps)
    _sync(L)
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
    tuned = L.autotune(TUNE_REPS)
    dt = _timed(L, steps, warmup)
    cells = sum(L.ncells(k) for k in range(len(insts)))
    res = dict(instances=len(insts), cells=cells, steps=steps, ms_per_step=round(1e3 * dt / steps, 4),
               aggregate_mlups=round(cells * steps / dt / 1e6, 1),
               instance_steps_per_s=round(len(insts) * steps / dt, 1),
               instances_per_s=round(len(insts) / (w["steps"] * dt / steps), 3),
               note="instances_per_s: the %d-step heel sweep of all instances per second" % w["steps"],
               batched=batched, graph=graph, autotuned={k: tuned[k] for k in ("tile_x", "stream_store",
                                                                               "boundary_layout")})
    if batched and not graph:
        # the two sweeps' event-timed launches against the bytes of all instances
        L.enable_kernel_timing(True)
        n = max(10, min(steps, 100))
        L.step(n)
        _sync(L)
        bulk_ms, launches = L.kernel_time(0)
        bnd_ms, _ = L.kernel_time(1)
        L.enable_kernel_timing(False)
        alg = dict(bulk=0, boundary=0)
        for k in range(len(insts)):
            a, _ = algorithmic_bytes(L.types(k), STORAGE_BYTES[storage], L.boundary_cells(k))
            alg["bulk"] += a["bulk"]
            alg["boundary"] += a["boundary"]
        res["kernels"] = kernel_rooflines(dict(alg_bytes=alg, bulk_ms=bulk_ms / launches,
                                               boundary_ms=bnd_ms / launches), storage)
    L.close()
    return res


def other_configs(steps, warmup):
    """The 128^3 basin (the released box, roll only; cache resident: its
    160 MB per step fit the 256 MB cache in front of HBM), the 256x192x192
    held box (FP32 / FP16 / BF16) and the 48-instance heel sweep."""
    from paper_1201_0351_amd import workloads as W

    out = {}
    b128 = {}
    for st in ("fp32", "fp16"):
        r = run_case(W.config2(20.0, released=True), st, steps, warmup)
        b128[st] = summary(r, st)
    r = run_case(W.config2(20.0, released=True), "fp32", max(5, steps // 4), warmup, host_update=1, timing=False,
                 tune=False)
    b128["fp32_host_update"] = {"value": round(r["value"], 1), "ms_per_step": round(r["ms_per_step"], 4)}
    b128["note"] = "cache resident (160 MB per FP32 step < 256 MB cache): not an HBM figure"
    out["basin128_box32x32x16_released"] = b128
    b3 = {}
    for st in ("fp32", "fp16", "bf16"):
        r = run_case(W.config3(20.0), st, steps, warmup, free=False)
        b3[st] = summary(r, st)
    b3["accuracy"] = "righting moment vs the FP64 oracle on the 128^3 geometry held at the same angles: " \
                     "see righting_moment"
    out["basin256x192x192_box64x64x32_heel20_held"] = b3
    out["batch48_heel_sweep"] = {st: run_batch(st, steps, warmup) for st in ("fp32", "fp16")}
    for st in ("fp32", "fp16"):
        rt = batch_righting(st)
        if rt is not None:
            out["batch48_heel_sweep"][st]["righting_moment"] = dict(
                runs=rt, max_rel_err=round(max(r["rel_err"] for r in rt if not r.get("thin_film")), 5),
                reference="FP64 oracle runs of four instances alone, tests/golden/batch48_righting.json",
                note="max_rel_err over the instances without a thin film over the deck edge; a thin-film "
                     "instance lists the range of the oracle's runs from starts with 1e-7 noise")
    out["batch48_heel_sweep"]["fp32_one_launch_per_instance"] = run_batch("fp32", steps, warmup, batched=False)
    out["batch48_heel_sweep"]["fp32_graph"] = run_batch("fp32", steps, warmup, graph=True)
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


def channel_oracle(steps_all=2, steps_one=1):
    """The FP64 oracle on the headline workload (the channel with its free
    box, coupled host update after every step): one untimed step (it maps
    the box), `steps_all` steps timed on all host cores, `steps_one` steps
    timed on one thread.  Returns the timings and the body force, torque and
    pose after the 1 + steps_all + steps_one steps."""
    from oracle.oracle import Oracle, lib
    from paper_1201_0351_amd import workloads as W

    threads = min(16, os.cpu_count() or 1)
    w = W.config5()
    c = w["lattice"]
    o = Oracle(c["nx"], c["ny"], c["nz"], c["tau"], accel=c["accel"], eps=c["eps"], periodic=c["periodic"],
               threads=threads)
    o.init_basin(c["fill_height"], c["init_ux_surface"])
    b = w["bodies"][0]
    o.set_body(0, b["half"], b["pos"], b["quat"], b["vel"], b["omega"], b["density"], 0)
    o.step_coupled(1, [w["dof"]])
    t0 = time.perf_counter()
    o.step_coupled(steps_all, [w["dof"]])
    t_all = time.perf_counter() - t0
    lib().ob_set_threads(o._h, 1)
    t0 = time.perf_counter()
    o.step_coupled(steps_one, [w["dof"]])
    t_one = time.perf_counter() - t0
    F, T = o.body_forces(0)
    bd = o.get_body(0)
    flags = o.get_flags()
    n = o.ncells
    o.close()
    return dict(threads=threads, n=n, steps_all=steps_all, t_all=t_all, steps_one=steps_one, t_one=t_one,
                steps=1 + steps_all + steps_one, F=F, T=T, pos=bd["pos"], flags=flags)


def channel_accuracy(ref, storages=("fp32", "fp16", "bf16")):
    """The channel on the GPU for the oracle's number of steps from the same
    initial state: error of the body force and torque of the last sweep,
    relative to the oracle's vector and (since the box floats near balance,
    so that the net force is a small difference of large link sums) to the
    box's weight M g and M g h/2; the body position after the rigid-body
    updates; and the cells whose type differs."""
    from paper_1201_0351_amd import lbm
    from paper_1201_0351_amd import workloads as W

    b = W.config5()["bodies"][0]
    g = abs(W.config5()["lattice"]["accel"][2])
    weight = b["density"] * 8.0 * b["half"][0] * b["half"][1] * b["half"][2] * g
    out = {"steps": ref["steps"], "reference": "FP64 oracle, same initial state, coupled host update every step",
           "oracle_force": [float(v) for v in ref["F"]], "oracle_torque": [float(v) for v in ref["T"]],
           "weight": weight}
    for st in storages:
        w = W.config5(st)
        L = lbm.Lattice(dict(w["lattice"], max_bodies=1))
        L.set_body(0, dict(w["bodies"][0], fixed=0, dof=w["dof"]))
        L.step(ref["steps"])
        F, T = L.body_forces(0)
        pos = L.get_body(0)["pos"]
        mism = int((L.flags() != ref["flags"]).sum())
        L.close()
        dF, dT = np.linalg.norm(F - ref["F"]), np.linalg.norm(T - ref["T"])
        out[st] = dict(force_rel_err=float(dF / np.linalg.norm(ref["F"])),
                       torque_rel_err=float(dT / np.linalg.norm(ref["T"])),
                       force_err_of_weight=float(dF / weight), torque_err_of_weight_arm=float(dT / (weight * b["half"][2])),
                       pos_err=float(np.abs(np.asarray(pos) - ref["pos"]).max()), flag_mismatches=mism,
                       force=[float(v) for v in F], torque=[float(v) for v in T])
    return out


def basin256_oracle(steps=2):
    """The FP64 oracle on the 256x192x192 held-box basin (truncated run): one
    untimed step (it maps the box), then `steps` steps on all host cores."""
    from oracle.oracle import Oracle
    from paper_1201_0351_amd import workloads as W

    threads = min(16, os.cpu_count() or 1)
    w = W.config3(20.0)
    c, b = w["lattice"], w["bodies"][0]
    o = Oracle(c["nx"], c["ny"], c["nz"], c["tau"], accel=c["accel"], eps=c["eps"], threads=threads)
    o.init_basin(c["fill_height"])
    o.set_body(0, b["half"], b["pos"], b["quat"], density=b["density"], fixed=1)
    o.step(1)
    t0 = time.perf_counter()
    o.step(steps)
    dt = time.perf_counter() - t0
    n = o.ncells
    F, T = o.body_forces(0)
    flags = o.get_flags()
    o.close()
    return dict(value=n * steps / dt / 1e6, unit="MLUPS", cores=threads,
                sample="%d steps of the 256x192x192 basin with its held box (after one untimed mapping step), FP64"
                       % steps, state=dict(steps=1 + steps, F=F, T=T, flags=flags))


def basin256_accuracy(ref, storages=("fp32", "fp16", "bf16")):
    """The 256x192x192 held box on the GPU for the oracle's number of steps
    from the same initial state: error of the force and torque of the last
    sweep (relative to the oracle's vector and to the box's buoyancy scale)
    and the cells whose type differs."""
    from paper_1201_0351_amd import lbm
    from paper_1201_0351_amd import workloads as W

    w = W.config3(20.0)
    b = w["bodies"][0]
    g = abs(w["lattice"]["accel"][2])
    scale = 8.0 * b["half"][0] * b["half"][1] * b["half"][2] * g * 0.5
    out = {"steps": ref["steps"], "reference": "FP64 oracle, same initial state",
           "oracle_force": [float(v) for v in ref["F"]], "oracle_torque": [float(v) for v in ref["T"]]}
    for st in storages:
        w = W.config3(20.0, st)
        L = lbm.Lattice(dict(w["lattice"], max_bodies=1))
        L.set_body(0, w["bodies"][0])
        L.step(ref["steps"])
        F, T = L.body_forces(0)
        mism = int((L.flags() != ref["flags"]).sum())
        L.close()
        dF, dT = np.linalg.norm(F - ref["F"]), np.linalg.norm(T - ref["T"])
        out[st] = dict(force_rel_err=float(dF / np.linalg.norm(ref["F"])),
                       torque_rel_err=float(dT / np.linalg.norm(ref["T"])),
                       force_err_of_half_weight=float(dF / scale), flag_mismatches=mism)
    return out


def cpu_baseline(ref, ref3):
    n = ref["n"]
    return dict(value=n * ref["steps_all"] / ref["t_all"] / 1e6, unit="MLUPS", cores=ref["threads"], kind="oracle",
                sample="%d steps of the 512x256x256 channel with its free box (after one untimed mapping step), "
                       "FP64, %d OpenMP threads; one_thread: %d more step(s) on 1 thread" % (
                           ref["steps_all"], ref["threads"], ref["steps_one"]),
                one_thread=dict(value=n * ref["steps_one"] / ref["t_one"] / 1e6, cores=1),
                basin256={k: v for k, v in ref3.items() if k != "state"})


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
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline and the accuracy check")
    ap.add_argument("--no-extra", action="store_true",
                    help="only the headline and its FP16 / BF16 / host-update runs")
    ap.add_argument("--profile", choices=["channel-fp32", "channel-fp16", "channel-bf16", "basin128-fp32",
                                          "basin256-fp32", "basin256-fp16", "batch48-fp32", "batch48-fp16"],
                    help="only run this timed case (for the profiler) and print its summary")
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
        print("bench.py: the benchmark runs on one GPU (its workload is one lattice on one device); "
              "--gpus %d is not supported" % args.gpus, file=sys.stderr)
        sys.exit(2)
    from paper_1201_0351_amd import workloads as W

    if args.profile and args.profile.startswith("batch48"):
        st = args.profile.split("-")[1]
        print(json.dumps(dict(case=args.profile, **run_batch(st, args.steps, args.warmup))))
        return
    if args.profile:
        name, st = args.profile.split("-")
        wl = {"channel": (W.config5(), True, PREP_STEPS), "basin128": (W.config2(20.0, released=True), True, 0),
              "basin256": (W.config3(20.0), False, 0)}[name]
        r = run_case(wl[0], st, args.steps, args.warmup, free=wl[1], prep=wl[2])
        print(json.dumps(dict(case=args.profile, **summary(r, st))))
        return

    chan = W.config5()
    r32 = run_case(chan, "fp32", args.steps, args.warmup, prep=PREP_STEPS)
    print("channel fp32: %.1f MLUPS, %.4f ms/step (windows %s), bulk %.4f ms, boundary %.4f ms" % (
        r32["value"], r32["ms_per_step"], r32["ms_windows"], r32["bulk_ms"], r32["boundary_ms"]),
        file=sys.stderr, flush=True)
    out = {
        "metric": METRIC,
        "value": round(r32["value"], 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": r32["steps"],
        "warmup": args.warmup,
        "ms_per_step": round(r32["ms_per_step"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "channel 512x256x256, periodic x and y, walls at z = 0 and 256, liquid depth 128, "
                               "tau 0.8, g 1e-5, body-force drive for surface speed 0.05 (half-Poiseuille start), "
                               "free 48x24x24 box of density 0.6 in 6 DOF, remap and conversions every step, FP32 "
                               "deviation storage, rigid-body update on the device; each timed window on a channel "
                               "prepared afresh by %d steps from its start and the warm-up" % PREP_STEPS,
                   "cells": r32["cells"], "cell_types": r32["counts"], "steps_per_lattice": r32["steps_per_lattice"]},
        "roofline": roofline(r32, "fp32"),
        "kernels": kernel_rooflines(r32, "fp32"),
        "ms_windows": r32["ms_windows"],
        "tuning": r32["tuning"],
        "body": r32["body"],
    }
    chan_out = {}
    for st in ("fp16", "bf16"):
        r = run_case(W.config5(st), st, args.steps, args.warmup, prep=PREP_STEPS)
        chan_out[st] = summary(r, st)
        print("channel %s: %.1f MLUPS" % (st, r["value"]), file=sys.stderr, flush=True)
    rh = run_case(chan, "fp32", max(5, args.steps // 4), args.warmup, prep=PREP_STEPS, host_update=1, timing=False,
                  tune=False)
    chan_out["fp32_host_update"] = {"value": round(rh["value"], 1), "ms_per_step": round(rh["ms_per_step"], 4),
                                    "steps": rh["steps"]}
    print("channel fp32 host update: %.1f MLUPS" % rh["value"], file=sys.stderr, flush=True)
    out["channel"] = chan_out
    if not args.no_extra:
        rm = {}
        for st in ("fp32", "fp16", "bf16"):
            v = righting_moment(st)
            if v is not None:
                rm[st] = v
        if rm:
            out["righting_moment"] = dict(rm, reference="FP64 oracle, held box, tests/golden/righting_moment_128.json",
                                          max_rel_err={k: round(max(x["rel_err"] for x in v), 5)
                                                       for k, v in rm.items()})
        out["other_configs"] = other_configs(max(50, args.steps // 4), 20)
        print("other configs done", file=sys.stderr, flush=True)
    if not args.no_cpu:
        ref = channel_oracle()
        out["accuracy"] = channel_accuracy(ref)
        ref3 = basin256_oracle()
        out["accuracy_basin256"] = basin256_accuracy(ref3["state"])
        out["cpu_baseline"] = cpu_baseline(ref, ref3)
        print("oracle done", file=sys.stderr, flush=True)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
