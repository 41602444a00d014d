"""Write tests/golden/c2_window.txt: the oracle's Dormand-Prince trajectory of
the 1024 x 1024 x 1 vortex film (2 nm cells, Msat 8e5 A/m, Aex 1.3e-11 J/m,
alpha 0.01, B_ext 10 mT along x; MaxErr 1e-5, headroom 0.8, first step
1e-14 s) through the output times k * 5 ps, k = 1..10, then every 10 ps up to
--t-end (sections "Dynamics" and "Adaptive time step"; the run is clipped to
land on every output time).

Recorded per output time: the accepted steps so far and the average
magnetisation; m at a fixed seeded sample of cells at the last output time.
The file is rewritten after every output time, so an interrupted run leaves a
complete, shorter window.  Only the oracle and the seeded input generator are
used:

    python tests/golden/make_c2_window.py [--workers N] [--t-end SECONDS] [--out PATH]

(hours of CPU: about 10 s per accepted step of 6 FP64 field evaluations of a
2048 x 2048 padded convolution on 8 cores; 1029 steps by 140 ps, the default end).
"""
import argparse
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import fields, integrate  # noqa: E402
from paper_1406_7635_amd import synth  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c2_window.txt")
T_FIRST = [k * 5e-12 for k in range(1, 11)]  # the first 50 ps every 5 ps, then every 10 ps
NSAMPLE = 2048
SAMPLE_SEED = 21


def sample_cells(n=1024):
    rng = np.random.Generator(np.random.PCG64(SAMPLE_SEED))
    return rng.integers(0, n, NSAMPLE), rng.integers(0, n, NSAMPLE)  # (y, x)


def write(rows, it, out):
    ys, xs = sample_cells()
    tmp = out + ".tmp"
    with open(tmp, "w") as f:
        f.write("# Oracle (FP64) Dormand-Prince trajectory of the 1024x1024x1 vortex film, seed 2\n")
        f.write("# (2 nm cells, Msat 8e5, Aex 1.3e-11, alpha 0.01, B_ext 10 mT x; MaxErr 1e-5,\n")
        f.write("# headroom 0.8, first dt 1e-14 s), clipped onto each output time.\n")
        f.write("# written by tests/golden/make_c2_window.py (oracle/ and the seeded inputs only)\n")
        f.write("# section mean: t_out steps rejects <mx> <my> <mz>\n")
        for t_out, ns, nr, mean in rows:
            f.write("mean %.6e %d %d %.12e %.12e %.12e\n" % (t_out, ns, nr, mean[0], mean[1], mean[2]))
        f.write("# section cell: y x mx my mz at the last output time (cells from PCG64 seed %d)\n"
                % SAMPLE_SEED)
        for y, x in zip(ys, xs):
            m = it.m[:, 0, y, x]
            f.write("cell %d %d %.9e %.9e %.9e\n" % (y, x, m[0], m[1], m[2]))
    os.replace(tmp, out)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workers", type=int, default=-1)
    ap.add_argument("--t-end", type=float, default=140e-12)
    ap.add_argument("--out", default=OUT)
    args = ap.parse_args()
    t_out_all = T_FIRST + [k * 1e-11 for k in range(6, 10000) if k * 1e-11 <= args.t_end * (1 + 1e-9)]
    case = synth.vortex_film(seed=2, n=1024)
    prob = fields.Problem(case["grid"], case["cell"], case["region"], case["params"])
    prob.workers = args.workers
    it = integrate.Integrator(prob.torque, case["m0"], "rk45", dt=1e-14, max_err=1e-5)
    rows = []
    t0 = time.time()
    for t_out in t_out_all:
        it.run(t_out)
        mean = it.m.reshape(3, -1).mean(axis=1)
        rows.append((t_out, it.nsteps, it.nrejects, mean))
        print("t %.3e steps %d rejects %d <m> %s (%.0f s)" % (t_out, it.nsteps, it.nrejects, mean,
                                                               time.time() - t0), flush=True)
        write(rows, it, args.out)
    print("wrote", args.out)


if __name__ == "__main__":
    main()
