"""Write tests/golden/floating_cubes_130x40x40.json with the FP64 oracle.

Workload (equilibrium of floating cubes, Sec. "Equilibrium Position of
Floating Cubes"): a 130x40x40 basin filled to z = 20, tau 1/1.9, gravity
7.5e-4, three 32x16x16 boxes (the cube of side 16 extruded along x) of
density 0.75, 0.5 and 0.25 at x = 21, 65, 109, centred at the upright
equilibrium draft (z = 28 - 16 rho_s) and heeled 2.86 deg about x, free in
heave and roll (DOF mask 0x0C); z and heel sampled every 250 steps.

(At 2.86 deg every cell centre lies on the same side of every face as in the
upright pose, so the mapped boxes are upright and the y-symmetric basin
exerts no roll torque beyond round-off: a roll-only run stays at 2.86 deg
until round-off breaks the symmetry, which in FP64 takes far longer than in
FP32.  With heave the bottom faces sink onto a row of cell centres within a
few hundred steps, the mapping turns asymmetric and the trajectory is
deterministic enough to compare.)

The paper starts its cubes far from equilibrium.  Three more runs do that:
  settle    heave and roll from 10 deg at the upright draft, `--settle`
            steps; the heels averaged over the last quarter are the settled
            heels to set against the paper's 26.565 / 45 / 26.565 deg
  settle_perturbed  the same from 10.001 deg: the box of density 3/4 comes
            to rest at another heel (its resting heel is not unique at 16
            cells a side), the other two where they did
  roll_only roll only (centre held at the upright draft) from 15 deg,
            `--steps` steps (the closed form for a held centre is
            20.7 / 45 / 20.7 deg)

Only the oracle is called.  `--sections a,b` recomputes only those sections
and keeps the others of the existing file (the runs are independent).

Usage: python tests/golden/make_floating_cubes.py [--steps 3000] [--settle 15000] [--threads 8]
       [--sections heave_roll,roll_only,settle,settle_perturbed]
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

NX, NY, NZ, H, S = 130, 40, 40, 20.0, 16
TAU, G, EPS = 1.0 / 1.9, 7.5e-4, 1e-2
DENSITIES = (0.75, 0.5, 0.25)
HEEL0 = 2.86


def heel_deg(q):
    return math.degrees(2.0 * math.atan2(q[1], q[0]))


def run(dof, steps, every, threads, heel0=HEEL0):
    o = Oracle(NX, NY, NZ, TAU, accel=(0.0, 0.0, -G), eps=EPS, threads=threads)
    o.init_basin(H)
    a = math.radians(heel0)
    for k, rs in enumerate(DENSITIES):
        o.set_body(k, (S, S / 2, S / 2), (21.0 + 44.0 * k, 20.0, H + S / 2 - rs * S),
                   (math.cos(a / 2), math.sin(a / 2), 0.0, 0.0), density=rs, fixed=0)
    M0, L0 = o.mass_total()
    trace = []
    t0 = time.time()
    done = 0
    while done < steps:
        o.step_coupled(every, [dof] * 3)
        done += every
        row = [done]
        for k in range(3):
            b = o.get_body(k)
            row += [heel_deg(b["quat"]), float(b["pos"][2])]
        trace.append(row)
        if done % 1000 == 0:
            print("dof 0x%02x step %d heel/z %s (%.0f s)" % (dof, done, [round(v, 3) for v in row[1:]],
                                                          time.time() - t0), flush=True)
    M1, L1 = o.mass_total()
    late = [row for row in trace if row[0] > 0.75 * steps]
    settled = [sum(abs(row[1 + 2 * k]) for row in late) / len(late) for k in range(3)]
    return dict(dof=dof, heel0_deg=heel0, steps=steps, every=every, columns="step, then heel_deg and z per body",
                trace=trace, mass_minus_ledger=[M0 - L0, M1 - L1], settled_heel_deg=settled)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--steps", type=int, default=3000)
    ap.add_argument("--settle", type=int, default=15000)
    ap.add_argument("--every", type=int, default=250)
    ap.add_argument("--threads", type=int, default=min(8, os.cpu_count() or 1))
    ap.add_argument("--out", type=str, default=os.path.join(HERE, "floating_cubes_130x40x40.json"))
    ap.add_argument("--sections", type=str, default="heave_roll,roll_only,settle,settle_perturbed")
    args = ap.parse_args()
    runs = dict(heave_roll=lambda: run(0x0C, args.steps, args.every, args.threads),
                roll_only=lambda: run(0x08, args.steps, args.every, args.threads, heel0=15.0),
                settle=lambda: run(0x0C, args.settle, args.every, args.threads, heel0=10.0),
                settle_perturbed=lambda: run(0x0C, args.settle, args.every, args.threads, heel0=10.001))
    want = [k for k in args.sections.split(",") if k]
    for k in want:
        if k not in runs:
            raise SystemExit("unknown section %s" % k)
    res = {}
    if set(want) != set(runs) and os.path.exists(args.out):
        with open(args.out) as fh:
            res = json.load(fh)
    res.update(_source="FP64 oracle (oracle/lgs_oracle.c), written by tests/golden/make_floating_cubes.py",
               nx=NX, ny=NY, nz=NZ, fill_height=H, side=S, tau=TAU, g=G, eps=EPS, densities=list(DENSITIES),
               heel0_deg=HEEL0)
    for k in want:
        res[k] = runs[k]()
    with open(args.out, "w") as fh:
        json.dump(res, fh, indent=1)
    print("wrote", args.out)


if __name__ == "__main__":
    main()
