"""Laminar flame speed of the quasi-1D premixed flame (Sec. 5.1): HIP path against
the FP64 oracle, within 0.5%.

Parity unpinned: a flame speed has no closed form, and the paper's values are for real
hydrogen/air through Cantera; the comparison is GPU against oracle only.

Front x_f: first crossing of T = 3 T_u from the unburnt side, linearly interpolated
(the isoline the paper takes for the front of its expanding flame, Sec. 5.2).  S_L is
minus the slope of a least-squares line through x_f over steps 2000..6000, after the
ignition transient; the flame moves about 20 cells in that window.
"""
import numpy as np
import pytest

from oracle import oracle as orc
from paper_2101_01702_amd import workloads as W

pytestmark = pytest.mark.gpu

NX, STEPS, EVERY, FIT_FROM = 1024, 6000, 250, 2000


@pytest.fixture(scope="module")
def lbm_mod():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2101_01702_amd import lbm
    lbm.load()
    return lbm


def front(T, T_u):
    hot = np.nonzero(T >= 3.0 * T_u)[0]
    k = int(hot[0])
    assert k > 0
    return k - 1 + (3.0 * T_u - T[k - 1]) / (T[k] - T[k - 1])


def flame_speed(step, temperature, T_u):
    xs, ts = [], []
    for n in range(EVERY, STEPS + 1, EVERY):
        step(EVERY)
        if n >= FIT_FROM:
            xs.append(front(temperature(), T_u))
            ts.append(n)
    slope = np.polyfit(np.array(ts, float), np.array(xs), 1)[0]
    return -slope, np.array(xs)


@pytest.fixture(scope="module")
def oracle_speed():
    prob = W.flame1d(nx=NX, hot_cells=64)
    sim = orc.OracleSim(prob).init()
    speed, xs = flame_speed(lambda n: sim.step(n, 8), lambda: sim.macros()["T"], 300.0)
    assert speed > 0.003, speed            # the flame propagates into the premixture
    return speed, xs


@pytest.mark.parametrize("storage", [W.STORE_F64, W.STORE_F32])
def test_flame_speed_matches_oracle(lbm_mod, oracle_speed, storage):
    prob = W.flame1d(nx=NX, hot_cells=64)
    s = lbm_mod.Solver(prob, storage=storage).init()
    speed, xs = flame_speed(s.step, lambda: s.macros()["T"], 300.0)
    assert s.status() == 0
    ref, ref_xs = oracle_speed
    rel = abs(speed - ref) / ref
    print(f"[storage={storage}] S_L gpu {speed:.6e} oracle {ref:.6e} cells/step, rel diff {rel:.2e}, "
          f"max front shift {np.abs(xs - ref_xs).max():.2e} cells", flush=True)
    assert rel <= 5e-3


def _golden_4096():
    """The oracle's S_L and front positions of the 4096-cell flame over 20 000 steps,
    written by tests/golden/make_flame_speed.py (oracle only)."""
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "flame_speed_4096.txt")
    speed, ts, xs = None, [], []
    with open(path) as f:
        for line in f:
            if line.startswith("#"):
                continue
            key, val = line.split()
            if key == "S_L":
                speed = float(val)
            else:
                ts.append(int(key))
                xs.append(float(val))
    return speed, np.array(ts), np.array(xs)


@pytest.mark.parametrize("storage", [W.STORE_F64, W.STORE_F32])
def test_full_size_flame_speed_against_oracle_golden(lbm_mod, storage):
    """The 4096-cell flame over 20 000 steps (steps replayed from a graph, 100 at a time):
    S_L from a least-squares line through the front every 100 steps over steps
    10 000..20 000, against the oracle's value stored in tests/golden, within 0.5%.  The
    FP64 path's fronts also match the oracle's to 1e-6 cells."""
    ref, ref_ts, ref_xs = _golden_4096()
    prob = W.flame1d(nx=4096)
    s = lbm_mod.Solver(prob, storage=storage).init()
    xs, ts = [], []
    for n in range(100, 20001, 100):
        s.step_graph(100)
        if n >= 10000:
            xs.append(front(s.macros()["T"], 300.0))
            ts.append(n)
    assert s.status() == 0
    s.close()
    assert np.array_equal(np.array(ts), ref_ts)
    got = -np.polyfit(np.array(ts, float), np.array(xs), 1)[0]
    rel = abs(got - ref) / ref
    shift = float(np.abs(np.array(xs) - ref_xs).max())
    print(f"[flame1d 4096, 20k steps, storage={storage}] S_L gpu {got:.9e} oracle {ref:.9e} cells/step, "
          f"rel diff {rel:.2e}, max front shift {shift:.2e} cells", flush=True)
    assert ref > 0.003
    assert rel <= 5e-3
    if storage == W.STORE_F64:
        assert shift <= 1e-6
