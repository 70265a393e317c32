"""Writes flame_speed_4096.txt: the oracle's laminar flame speed of the quasi-1D premixed
flame of 4096 cells (the synthetic 9-species / 19-reaction mechanism, unburnt 300 K at
equivalence ratio 1, 64-cell hot slab at 2000 K) over 20 000 steps.

The front x_f is the first crossing of T = 3 T_u from the unburnt side, linearly
interpolated, every 100 steps; S_L is minus the slope of the least-squares line through
x_f over steps 10 000..20 000 (the flame-speed measurement of Sec. 5.1).  Only the FP64
CPU oracle runs here.

    python tests/golden/make_flame_speed.py [threads]
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import oracle as orc                       # noqa: E402
from paper_2101_01702_amd import workloads as W       # noqa: E402

NX, STEPS, EVERY, FIT_FROM, T_U = 4096, 20000, 100, 10000, 300.0
OUT = os.path.join(HERE, "flame_speed_4096.txt")


def front(T, T_u):
    hot = np.nonzero(T >= 3.0 * T_u)[0]
    k = int(hot[0])
    return k - 1 + (3.0 * T_u - T[k - 1]) / (T[k] - T[k - 1])


def main():
    threads = int(sys.argv[1]) if len(sys.argv) > 1 else (os.cpu_count() or 1)
    prob = W.flame1d(nx=NX)
    sim = orc.OracleSim(prob).init()
    t0 = time.time()
    ts, xs = [], []
    for n in range(EVERY, STEPS + 1, EVERY):
        anom = sim.step(EVERY, threads)
        if anom:
            raise RuntimeError(f"oracle anomaly bits {anom} at step {n}")
        if n >= FIT_FROM:
            ts.append(n)
            xs.append(front(sim.macros()["T"], T_U))
        if n % 1000 == 0:
            print(f"step {n}, {time.time() - t0:.0f} s", flush=True)
    speed = -np.polyfit(np.array(ts, float), np.array(xs), 1)[0]
    with open(OUT, "w") as f:
        f.write("# oracle laminar flame speed, quasi-1D flame of 4096 cells, 20000 steps (FP64 CPU oracle)\n")
        f.write("# command: python tests/golden/make_flame_speed.py\n")
        f.write("# front: first crossing of T = 3 T_u (T_u = 300 K) from the unburnt side, every 100 steps;\n")
        f.write("# S_L: minus the least-squares slope of the front over steps 10000..20000 (cells/step)\n")
        f.write(f"S_L {speed:.15e}\n")
        for t, x in zip(ts, xs):
            f.write(f"{t} {x:.15e}\n")
    print(f"S_L = {speed:.9e} cells/step ({time.time() - t0:.0f} s)")


if __name__ == "__main__":
    main()
