"""Flame-front speeds (lbm_flame_speeds: S_d and S_a of eq. sd, isosurface weights and
their sums) of the HIP path against the oracle's, on the same run.

Bar for FP64 storage: the two states agree to ~1e-13 after the run, and S_d holds a
second difference of T (the divergence of lambda grad T over a one-cell stencil) divided
by |grad T|: near the front a temperature rounding of 1e-13 T becomes ~1e-13 T / (cell
change of T), at most ~1e-11 for these fronts.  The bar is 1e-9 relative to the largest
|S_d| among the nodes of the isosurface (w > 0), 1e-9 absolute on the weights (which lie
in [0, 1]) and 1e-9 relative on the sums."""
import dataclasses

import numpy as np
import pytest

from paper_2101_01702_amd import workloads as W
from gpu_cases import oracle_run

pytestmark = pytest.mark.gpu

TOL = 1e-9


@pytest.fixture(scope="module")
def lbm_mod():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2101_01702_amd import lbm
    lbm.load()
    return lbm


def _compare(gpu, ref, label, idx=None, totals=True):
    g = {k: (v if idx is None else v[idx]) for k, v in gpu.items() if k != "totals"}
    sel = ref["w"] > 0
    assert sel.sum() > 0
    scale = max(np.abs(ref["Sd"][sel]).max(), np.abs(ref["Sa"][sel]).max())
    e_d = np.abs(g["Sd"] - ref["Sd"])[sel].max() / scale
    e_a = np.abs(g["Sa"] - ref["Sa"])[sel].max() / scale
    e_w = np.abs(g["w"] - ref["w"]).max()
    msg = f"[{label}] isosurface nodes {sel.sum()}: S_d {e_d:.2e} S_a {e_a:.2e} w {e_w:.2e}"
    if totals:
        e_t = np.abs(gpu["totals"] - ref["totals"]) / np.maximum(np.abs(ref["totals"]), 1e-300)
        e_t = float(np.where(np.abs(ref["totals"]) > 0, e_t, np.abs(gpu["totals"])).max())
        msg += f" totals {e_t:.2e}"
    print(msg, flush=True)
    assert e_d <= TOL and e_a <= TOL and e_w <= TOL
    if totals:
        assert e_t <= TOL


def test_front_speeds_quasi_1d_flame_fp64(lbm_mod):
    prob = W.flame1d(nx=512, hot_cells=64)
    s = lbm_mod.Solver(prob, storage=W.STORE_F64).init()
    s.step(300)
    sim, anom = oracle_run(prob, 300)
    assert anom == 0 and s.status() == 0
    for T_iso in (900.0, 1500.0):
        _compare(s.flame_speeds(T_iso, centre=(511.0, 0.0, 0.0)),
                 sim.flame_speeds(T_iso, centre=(511.0, 0.0, 0.0)), f"flame1d T_iso {T_iso}")
    s.close()


def test_front_speeds_3d_with_symmetry_faces_fp64(lbm_mod):
    prob = W.perturb_velocity(W.sphere3d(shape=(13, 10, 9), radius=3.5, storage=W.STORE_F64), 1e-3, 12)
    prob = dataclasses.replace(prob, bc=(W.BC_SYMMETRY, W.BC_OPEN, W.BC_SYMMETRY, W.BC_OPEN, 0, 0))
    s = lbm_mod.Solver(prob, storage=W.STORE_F64).init()
    s.step(60)
    sim, anom = oracle_run(prob, 60)
    assert anom == 0 and s.status() == 0
    c = (6.0, 4.5, 4.0)
    _compare(s.flame_speeds(700.0, centre=c), sim.flame_speeds(700.0, centre=c), "sphere 13x10x9 symmetry")
    s.close()


def test_front_speeds_of_a_flame_batch_fp64(lbm_mod):
    prob = W.flame_batch(lengths=[96, 150, 64], phis=[1.0, 2.0, 0.6], hot_cells=24, storage=W.STORE_F64)
    s = lbm_mod.Solver(prob, storage=W.STORE_F64).init()
    s.step(150)
    g = s.flame_speeds(900.0)
    assert s.status() == 0
    for k, part in enumerate(W.split_batch(prob)):
        sim, anom = oracle_run(part, 150)
        assert anom == 0
        _compare(g, sim.flame_speeds(900.0), f"batch flame {k}", idx=W.batch_nodes(prob, k), totals=False)
    s.close()


def test_front_speeds_fp32_storage(lbm_mod):
    """FP32 storage: the state carries the storage rounding (~1e-6 relative after 300
    steps), which the second difference in S_d amplifies by about the ratio of T to its
    change per cell at the front; the bar is 1e-3 relative."""
    prob = W.flame1d(nx=512, hot_cells=64)
    s = lbm_mod.Solver(prob, storage=W.STORE_F32).init()
    s.step(300)
    g = s.flame_speeds(900.0)
    sim, _ = oracle_run(prob, 300)
    ref = sim.flame_speeds(900.0)
    sel = ref["w"] > 0
    scale = np.abs(ref["Sd"][sel]).max()
    e = np.abs(g["Sd"] - ref["Sd"])[sel].max() / scale
    print(f"[flame1d fp32] S_d {e:.2e}, sum w {g['totals'][0]:.6f} vs {ref['totals'][0]:.6f}", flush=True)
    assert e <= 1e-3
    s.close()


def test_front_speeds_away_from_the_isosurface(lbm_mod):
    """A uniform state (config 1 at its mean composition, at rest): grad T is rounding
    noise, no node lies within one cell of T_iso = 1500 K, so every weight and every sum
    is exactly 0, and the speeds are finite."""
    prob = W.config1()
    prob.Y = np.repeat(prob.Y.mean(axis=1)[:, None], prob.N, axis=1)
    prob.rho = np.full(prob.N, prob.rho.mean())
    s = lbm_mod.Solver(prob, storage=W.STORE_F64).init()
    g = s.flame_speeds(1500.0)
    assert not np.any(g["w"]) and not np.any(g["totals"])
    assert np.all(np.isfinite(g["Sd"])) and np.all(np.isfinite(g["Sa"]))
    s.close()


def test_mean_radius_of_a_spherical_isotherm(lbm_mod):
    """Solver.mean_radius (eq. rmean from the isosurface sums) on a spherical isotherm of
    radius 10: the oracle's value to 1e-9, and 10 cells to 0.1 (the oracle's pin)."""
    R0, n, edge = 10.0, 44, 8.0
    prob = W.sphere3d(shape=(n, n, n), radius=R0, edge=edge, T_ig=1500.0, storage=W.STORE_F64)
    c = np.array([(n - 1) / 2] * 3) + np.array([0.13, -0.21, 0.34])
    z, y, x = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    r = np.sqrt((x - c[0]) ** 2 + (y - c[1]) ** 2 + (z - c[2]) ** 2).reshape(-1)
    prob.T = 300.0 + 1200.0 * W.tanh_profile(R0 - r, edge)
    prob.rho = W.lattice_density(np.full(prob.N, W.P_ATM), prob.T,
                                 np.full(prob.N, W.mean_molar_mass(W.premixed_h2air_X(prob.mech, 0.8),
                                                                    prob.mech.molar_mass)), prob.rho_ref)
    s = lbm_mod.Solver(prob, storage=W.STORE_F64).init()
    rg = s.mean_radius(900.0, centre=c)
    from oracle import oracle as orc
    tot = orc.OracleSim(prob).init().flame_speeds(900.0, centre=c)["totals"]
    print(f"[mean radius] gpu {rg:.6f} oracle {tot[4] / tot[0]:.6f}", flush=True)
    assert abs(rg - tot[4] / tot[0]) <= 1e-9 * R0
    assert abs(rg - R0) < 0.1
    s.close()
