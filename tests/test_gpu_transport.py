"""Temperature-dependent diffusivities, D_ab(T) = D_ab (T / T_ref)^n (lbm_desc.diff_T_ref,
diff_T_exp; a power law standing in for the temperature-dependent transport data of
Sec. 3): the HIP path against the oracle.  With T_ref = 600 K and n = 1.7 the flame's
diffusivities span a factor of 22 between its unburnt and burnt sides, and its
temperature after 1000 steps differs from the constant-diffusivity flame by up to 39 K."""
import dataclasses

import numpy as np
import pytest

from paper_2101_01702_amd import workloads as W
from gpu_cases import check_fp32, check_fp64, field_errors, oracle_run, pop_errors, zeta_of

pytestmark = pytest.mark.gpu

TOL64 = 1e-12


@pytest.fixture(scope="module")
def lbm_mod():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2101_01702_amd import lbm
    lbm.load()
    return lbm


def _flame():
    prob = W.flame1d(nx=512, hot_cells=64)
    prob.diff_T_ref, prob.diff_T_exp = 600.0, 1.7
    return prob


def test_flame_with_temperature_dependent_diffusivity_fp64(lbm_mod):
    prob = _flame()
    s = lbm_mod.Solver(prob, storage=W.STORE_F64).init()
    s.step(200)
    mac = s.macros()
    sim, anom = oracle_run(prob, 200)
    assert s.status() == 0 and anom == 0
    check_fp64(field_errors(mac, sim.macros(), zeta_of(prob)), "flame D(T) fp64")
    pop, _ = s.populations(np.arange(prob.N))
    assert max(pop_errors(pop, sim.state()[0])) <= TOL64
    # the front speeds use the same diffusion velocities
    g, r = s.flame_speeds(900.0), sim.flame_speeds(900.0)
    sel = r["w"] > 0
    assert np.abs(g["Sd"] - r["Sd"])[sel].max() <= 1e-9 * np.abs(r["Sd"][sel]).max()
    s.close()


def test_flame_with_temperature_dependent_diffusivity_fp32(lbm_mod):
    prob = _flame()
    s = lbm_mod.Solver(prob, storage=W.STORE_F32).init()
    s.step(1000)
    mac = s.macros()
    sim, anom = oracle_run(prob, 1000)
    assert s.status() == 0 and anom == 0
    check_fp32(field_errors(mac, sim.macros(), zeta_of(prob)), "flame D(T) fp32")
    s.close()


def test_3d_with_temperature_dependent_diffusivity_fp64(lbm_mod):
    prob = W.perturb_velocity(W.sphere3d(shape=(13, 10, 9), radius=3.0, storage=W.STORE_F64), 2e-3, 9)
    prob = dataclasses.replace(prob, diff_T_ref=400.0, diff_T_exp=-0.8)
    s = lbm_mod.Solver(prob, storage=W.STORE_F64).init()
    s.step(60)
    mac = s.macros()
    sim, anom = oracle_run(prob, 60)
    assert s.status() == 0 and anom == 0
    check_fp64(field_errors(mac, sim.macros(), zeta_of(prob)), "sphere D(T) fp64")


# Temperature-dependent viscosity and conductivity: 1/omega - 1/2 and 1/omega1 - 1/2
# scale with (T / 600 K)^0.5, together with the diffusivity law above; the burnt side
# relaxes at omega = 0.67 against 1.0 in the unburnt gas.
def _flame_all():
    prob = _flame()
    prob.visc_T_ref, prob.visc_T_exp = 600.0, 0.5
    return prob


def test_flame_with_temperature_dependent_transport_fp64(lbm_mod):
    prob = _flame_all()
    s = lbm_mod.Solver(prob, storage=W.STORE_F64).init()
    s.step(200)
    mac = s.macros()
    sim, anom = oracle_run(prob, 200)
    assert s.status() == 0 and anom == 0
    check_fp64(field_errors(mac, sim.macros(), zeta_of(prob)), "flame mu(T), D(T) fp64")
    pop, _ = s.populations(np.arange(prob.N))
    assert max(pop_errors(pop, sim.state()[0])) <= TOL64
    g, r = s.flame_speeds(900.0), sim.flame_speeds(900.0)
    sel = r["w"] > 0
    assert np.abs(g["Sd"] - r["Sd"])[sel].max() <= 1e-9 * np.abs(r["Sd"][sel]).max()
    s.close()


def test_flame_with_temperature_dependent_transport_fp32(lbm_mod):
    prob = _flame_all()
    s = lbm_mod.Solver(prob, storage=W.STORE_F32).init()
    s.step(1000)
    mac = s.macros()
    sim, anom = oracle_run(prob, 1000)
    assert s.status() == 0 and anom == 0
    check_fp32(field_errors(mac, sim.macros(), zeta_of(prob)), "flame mu(T), D(T) fp32")
    s.close()


def test_3d_with_temperature_dependent_viscosity_fp64(lbm_mod):
    prob = W.perturb_velocity(W.sphere3d(shape=(13, 10, 9), radius=3.0, storage=W.STORE_F64), 2e-3, 9)
    prob = dataclasses.replace(prob, visc_T_ref=800.0, visc_T_exp=-0.6,
                               bc=(W.BC_SYMMETRY, W.BC_OPEN, W.BC_OPEN, W.BC_OPEN, W.BC_SYMMETRY, W.BC_OPEN))
    s = lbm_mod.Solver(prob, storage=W.STORE_F64).init()
    s.step(60)
    mac = s.macros()
    sim, anom = oracle_run(prob, 60)
    assert s.status() == 0 and anom == 0
    check_fp64(field_errors(mac, sim.macros(), zeta_of(prob)), "sphere mu(T) fp64")
