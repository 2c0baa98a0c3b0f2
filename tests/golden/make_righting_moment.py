"""Write tests/golden/righting_moment_128.json with the FP64 oracle.

Workload: 128^3 basin, tau 0.55, gravity 5e-6, liquid depth 64, a 32x32x16
box (density 0.5) held with its centre on the water plane at a heel of 10,
20 and 30 deg about x (the held form of the 128^3 heeled-box workload).  The
righting moment m_s = -T_x is averaged over the last `window` of `steps`
steps (sampled every `every` steps).  The cell types after the last step
are stored too (2 bits per cell, z-major, packed four to a byte, zlib,
base64) so that a run of the same workload can count the cells whose type
differs.  Only the oracle is called.

Usage: python tests/golden/make_righting_moment.py [--steps 5000] [--threads 8]
       [--heels 10,20,30] [--out FILE]
       python tests/golden/make_righting_moment.py --merge PART1 PART2 ... [--out FILE]
(the heels are independent runs: --merge joins files this script wrote for
some of them into one, in the order given)
"""
import argparse
import base64
import json
import math
import os
import sys
import time
import zlib

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import analytic as A  # noqa: E402
from oracle.oracle import Oracle  # noqa: E402


def pack_types(t):
    """Cell types (0..3, [nz, ny, nx]) as base64 of zlib of four 2-bit codes per byte."""
    flat = np.ascontiguousarray(t, dtype=np.uint8).ravel()
    flat = np.concatenate([flat, np.zeros((-len(flat)) % 4, np.uint8)]).reshape(-1, 4)
    packed = (flat[:, 0] | (flat[:, 1] << 2) | (flat[:, 2] << 4) | (flat[:, 3] << 6)).astype(np.uint8)
    return base64.b64encode(zlib.compress(packed.tobytes(), 9)).decode("ascii")


def unpack_types(s, shape):
    packed = np.frombuffer(zlib.decompress(base64.b64decode(s)), np.uint8)
    t = np.stack([(packed >> k) & 3 for k in (0, 2, 4, 6)], axis=1).ravel()
    return t[: int(np.prod(shape))].reshape(shape)


def run(heel, steps, window, every, threads):
    g, H = 5e-6, 64.0
    o = Oracle(128, 128, 128, 0.55, accel=(0, 0, -g), eps=1e-2, threads=threads)
    o.init_basin(H)
    a = math.radians(heel)
    o.set_body(0, (16, 16, 8), (64, 64, 64), (math.cos(a / 2), math.sin(a / 2), 0, 0), density=0.5)
    samples, trace = [], []
    t0 = time.time()
    done = 0
    while done < steps:
        n = min(every, steps - done)
        o.step(n)
        done += n
        F, T = o.body_forces(0)
        trace.append((done, -T[0], F[2]))
        if done > steps - window:
            samples.append(-T[0])
        if done % 500 == 0:
            print("heel %g step %d m_s %.6e (%.0f s)" % (heel, done, -T[0], time.time() - t0), flush=True)
    ms = sum(samples) / len(samples)
    return dict(heel_deg=heel, steps=steps, window=window, every=every, m_s=ms,
                final_types=pack_types(o.types()),
                analytic_polygon=A.righting_moment_polygon(32, 16, 32, a, g, zw=0.0),
                trace=trace[:: max(1, len(trace) // 100)])


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--steps", type=int, default=5000)
    ap.add_argument("--window", type=int, default=1000)
    ap.add_argument("--every", type=int, default=10)
    ap.add_argument("--threads", type=int, default=min(8, os.cpu_count() or 1))
    ap.add_argument("--heels", type=str, default="10,20,30")
    ap.add_argument("--out", type=str, default=os.path.join(HERE, "righting_moment_128.json"))
    ap.add_argument("--merge", nargs="+", default=None)
    args = ap.parse_args()
    res = dict(_source="FP64 oracle (oracle/lgs_oracle.c), written by tests/golden/make_righting_moment.py",
               workload="128^3 basin tau 0.55 g 5e-6 depth 64, box 32x32x16 rho_s 0.5 held, G on the water plane")
    if args.merge:
        runs = []
        for part in args.merge:
            with open(part) as f:
                runs += json.load(f)["runs"]
        res["runs"] = runs
    else:
        res["runs"] = [run(float(h), args.steps, args.window, args.every, args.threads) for h in args.heels.split(",")]
    with open(args.out, "w") as f:
        json.dump(res, f, indent=1)
    print("wrote", args.out)


if __name__ == "__main__":
    main()
