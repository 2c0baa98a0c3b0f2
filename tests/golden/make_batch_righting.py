"""Write tests/golden/batch48_righting.json with the FP64 oracle.

Workload: the 48-instance heel sweep (paper_1201_0351_amd/workloads.py,
config4: uneven basins 64^3 .. 160x128x128, tau 0.55, g 5e-6, depth nz/2,
one held box of side b = ny/4, length b, height b/2 per instance, heel
uniform in [0, 60] deg, density 0.3 / 0.5 / 0.7).  Four instances stand for
the batch: the smallest, the largest, the one heeled furthest, and the
furthest-heeled of density 0.7.  Each is run alone for the workload's 3000
steps; the righting moment m_s = -T_x is averaged over the last 1000 steps
(sampled every 10).  Only the oracle and the seeded workload generator are
called.

An instance whose low deck edge lies under the water plane by less than 1.5
cells carries a thin film of liquid over the deck edge.  Conversions there
turn on round-off, and m_s with them.  For such an instance --realisations N
adds N more oracle runs from initial populations with noise of amplitude
1e-7 (seeds 1..N) to an existing file, as the spread the oracle itself shows.

Usage: python tests/golden/make_batch_righting.py [--threads 8]
       python tests/golden/make_batch_righting.py --realisations 4 [--jobs 4]
"""
import argparse
import json
import math
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle.oracle import Oracle  # noqa: E402
from paper_1201_0351_amd import workloads as W  # noqa: E402

STEPS, WINDOW, EVERY = 3000, 1000, 10


def heel_of(inst):
    q = inst["bodies"][0]["quat"]
    return math.degrees(2.0 * math.atan2(q[1], q[0]))


def chosen(insts):
    """Indices of the smallest, the largest, the furthest-heeled instance and
    the furthest-heeled one of density 0.7 (each distinct)."""
    cells = [i["lattice"]["nx"] * i["lattice"]["ny"] * i["lattice"]["nz"] for i in insts]
    picks = [min(range(len(insts)), key=lambda k: (cells[k], k)), max(range(len(insts)), key=lambda k: (cells[k], -k))]
    by_heel = sorted(range(len(insts)), key=lambda k: (-heel_of(insts[k]), k))
    picks.append(next(k for k in by_heel if k not in picks))
    picks.append(next(k for k in by_heel if k not in picks and insts[k]["bodies"][0]["density"] == 0.7))
    return picks


def deck_edge_depth(inst):
    """Depth (cells) of the low deck edge under the water plane (negative:
    above it) for the held box heeled about +x."""
    c, b = inst["lattice"], inst["bodies"][0]
    hy, hz = b["half"][1], b["half"][2]
    th = math.radians(heel_of(inst))
    edge = -hy * math.sin(th) + hz * math.cos(th)  # height over G
    water = c["fill_height"] - b["pos"][2]  # water plane over G
    return water - edge


def thin_film(inst):
    return 0.0 < deck_edge_depth(inst) < 1.5


def run(inst, threads, seed=0, noise_amp=0.0):
    c, b = inst["lattice"], inst["bodies"][0]
    o = Oracle(c["nx"], c["ny"], c["nz"], c["tau"], accel=c["accel"], eps=c["eps"], threads=threads)
    o.init_basin(c["fill_height"], seed=seed, noise_amp=noise_amp)
    o.set_body(0, b["half"], b["pos"], b["quat"], density=b["density"], fixed=1)
    samples, done, t0 = [], 0, time.time()
    while done < STEPS:
        o.step(EVERY)
        done += EVERY
        if done > STEPS - WINDOW:
            samples.append(-o.body_forces(0)[1][0])
    print("  %dx%dx%d heel %.2f rho_s %.1f: m_s %.6e (%.0f s)" % (c["nx"], c["ny"], c["nz"], heel_of(inst),
                                                                   b["density"], sum(samples) / len(samples),
                                                                   time.time() - t0), flush=True)
    o.close()
    return sum(samples) / len(samples)


def _realisation(a):
    k, seed, threads = a
    return k, seed, run(W.config4()["instances"][k], threads, seed=seed, noise_amp=1e-7)


def add_realisations(path, n, jobs, threads):
    from concurrent.futures import ProcessPoolExecutor

    with open(path) as f:
        res = json.load(f)
    insts = W.config4()["instances"]
    work = [(r["instance"], seed, threads) for r in res["runs"] if thin_film(insts[r["instance"]])
            for seed in range(1, n + 1)]
    with ProcessPoolExecutor(jobs) as ex:
        got = list(ex.map(_realisation, work))
    for r in res["runs"]:
        r["deck_edge_depth"] = deck_edge_depth(insts[r["instance"]])
        mine = [m for k, _, m in sorted(got) if k == r["instance"]]
        if mine:
            r["m_s_noise_1e-7"] = mine
    with open(path, "w") as f:
        json.dump(res, f, indent=1)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--threads", type=int, default=min(8, os.cpu_count() or 1))
    ap.add_argument("--out", type=str, default=os.path.join(HERE, "batch48_righting.json"))
    ap.add_argument("--realisations", type=int, default=0)
    ap.add_argument("--jobs", type=int, default=4)
    args = ap.parse_args()
    if args.realisations:
        add_realisations(args.out, args.realisations, args.jobs, args.threads)
        print("wrote", args.out)
        return
    insts = W.config4()["instances"]
    rows = []
    for k in chosen(insts):
        c, b = insts[k]["lattice"], insts[k]["bodies"][0]
        rows.append(dict(instance=k, shape=[c["nx"], c["ny"], c["nz"]], heel_deg=heel_of(insts[k]),
                         density=b["density"], m_s=run(insts[k], args.threads)))
    res = dict(_source="FP64 oracle (oracle/lgs_oracle.c), written by tests/golden/make_batch_righting.py",
               workload="config4 heel sweep, seed 4", steps=STEPS, window=WINDOW, every=EVERY, runs=rows)
    with open(args.out, "w") as f:
        json.dump(res, f, indent=1)
    print("wrote", args.out)


if __name__ == "__main__":
    main()
