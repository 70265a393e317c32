"""Every species count the library builds (M = 2..10): mechanisms extended with inert
species (the last one slaved), on a ragged 3D lattice with open, zero-velocity and
symmetry faces, FP64 storage against the oracle to 1e-12 after 30 steps."""
import dataclasses

import numpy as np
import pytest

from paper_2101_01702_amd import workloads as W
from gpu_cases import check_fp64, field_errors, oracle_run, pop_errors, zeta_of

pytestmark = pytest.mark.gpu


def with_inert(mech, n_extra):
    """mech plus n_extra inert species (molar masses 20, 24, ..., c_p/R 3.5 + k/4)."""
    if n_extra == 0:
        return mech
    M = mech.M
    mm = np.concatenate([mech.molar_mass, 20.0 + 4.0 * np.arange(n_extra)])
    nasa = np.concatenate([mech.nasa7, np.stack([W.nasa7_coeffs((3.5 + 0.25 * k, 0, 0, 0, 0), 0.0, 190.0 + 5 * k)
                                                 for k in range(n_extra)])])
    pad = np.zeros((mech.R, n_extra), np.int32)
    el = np.concatenate([mech.elements, np.zeros((n_extra, mech.elements.shape[1]), mech.elements.dtype)])
    return dataclasses.replace(mech, names=list(mech.names) + [f"I{k}" for k in range(n_extra)], molar_mass=mm,
                               elements=el, nasa7=nasa, nu_reac=np.concatenate([mech.nu_reac, pad], axis=1),
                               nu_prod=np.concatenate([mech.nu_prod, pad], axis=1))


def problem(M):
    if M == 2:
        base = W.config1(nx=7, ny=5, nz=4, reacting=False)
        mech = dataclasses.replace(base.mech, names=base.mech.names[:2], molar_mass=base.mech.molar_mass[:2],
                                   elements=base.mech.elements[:2], nasa7=base.mech.nasa7[:2],
                                   nu_reac=np.zeros((0, 2), np.int32), nu_prod=np.zeros((0, 2), np.int32))
    elif M < 9:
        base = W.config1(nx=7, ny=5, nz=4)
        mech = with_inert(base.mech, M - 3)
    else:
        base = W.sphere3d(shape=(7, 5, 4), radius=2.0, storage=W.STORE_F64)
        mech = with_inert(base.mech, M - 9)
    rng = np.random.default_rng(M)
    N = 7 * 5 * 4
    z, y, x = np.meshgrid(np.arange(4), np.arange(5), np.arange(7), indexing="ij")
    wave = (np.cos(2 * np.pi * x / 7 + 0.3) * np.cos(np.pi * y / 5) + np.sin(np.pi * z / 4)).reshape(-1)
    X = rng.uniform(0.5, 1.5, size=M)
    X = np.repeat((X / X.sum())[:, None], N, axis=1)
    X[0] *= 1.0 + 0.05 * wave
    X /= X.sum(axis=0)
    T = (1000.0 if M < 9 else 900.0) + 15.0 * wave
    m = W.mean_molar_mass(X, mech.molar_mass)
    kappa, rho_ref = W.lattice_scales(0.05 if M < 9 else 0.01, 1000.0, float(m.mean()), W.P_ATM)
    rho = W.lattice_density(np.full(N, W.P_ATM), T, m, rho_ref)
    D = W.symmetric_uniform(rng, M, 0.02, 0.06)
    u = np.stack([5e-4 * wave, 4e-4 * wave, -3e-4 * wave])
    return W.Problem(f"M{M}", 7, 5, 4, (W.BC_OPEN, W.BC_SYMMETRY, W.BC_OPEN_U0, W.BC_OPEN, W.BC_SYMMETRY,
                                         W.BC_OPEN), mech, D, 1.3, W.omega1_from_prandtl(1.3, 0.7), kappa,
                     base.dt_phys, rho_ref, W.P_ATM, rho, u, T, W.mole_to_mass(X, mech.molar_mass))


@pytest.fixture(scope="module")
def lbm_mod():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2101_01702_amd import lbm
    lbm.load()
    return lbm


@pytest.mark.parametrize("M", range(2, 11))
def test_species_count_fp64(lbm_mod, M):
    prob = problem(M)
    assert prob.M == M
    s = lbm_mod.Solver(prob, storage=W.STORE_F64).init()
    s.step(30)
    mac = s.macros()
    pop, _ = s.populations(np.arange(prob.N))
    assert s.status() == 0
    sim, anom = oracle_run(prob, 30)
    assert anom == 0
    err = field_errors(mac, sim.macros(), zeta_of(prob))
    print(f"[M={M}] worst {max(err, key=err.get)} {max(err.values()):.2e}", flush=True)
    check_fp64(err, prob.name)
    assert max(pop_errors(pop, sim.state()[0])) <= 1e-12
    s.close()


def test_max_reaction_count_fp64(lbm_mod):
    """LBM_MAX_REACTIONS = 64 reactions: the 19 of the synthetic mechanism repeated with
    their pre-exponential factors divided by 4 (the repeats add up like one faster
    reaction), on the M = 9 lattice."""
    prob = problem(9)
    mech = prob.mech
    reps = -(-64 // mech.R)
    idx = np.arange(64) % mech.R
    arr = mech.arrhenius[idx].copy()
    arr[:, 0] = arr[:, 0] / 4.0
    mech64 = dataclasses.replace(mech, nu_reac=mech.nu_reac[idx], nu_prod=mech.nu_prod[idx], arrhenius=arr,
                                 reversible=mech.reversible[idx])
    prob = dataclasses.replace(prob, mech=mech64, name="M9_R64")
    assert prob.mech.R == 64 and reps >= 3
    s = lbm_mod.Solver(prob, storage=W.STORE_F64).init()
    s.step(30)
    mac = s.macros()
    assert s.status() == 0
    sim, anom = oracle_run(prob, 30)
    assert anom == 0
    err = field_errors(mac, sim.macros(), zeta_of(prob))
    print(f"[M=9 R=64] worst {max(err, key=err.get)} {max(err.values()):.2e}", flush=True)
    check_fp64(err, prob.name)
    s.close()


def test_sixth_order_reaction_fp64(lbm_mod):
    """A reaction with 6 molecules on each side (3A + 3B -> 3C, A = 1e28 CGS, next to
    configuration 1's A + B -> C): the concentration products of the rate kernel at
    high order.  Over 30 steps it moves the mean Y_C by 0.04 (the oracle's run)."""
    base = W.config1(nx=8, ny=3, nz=2)
    mech = dataclasses.replace(base.mech, nu_reac=np.array([[1, 1, 0], [3, 3, 0]], np.int32),
                               nu_prod=np.array([[0, 0, 1], [0, 0, 3]], np.int32),
                               arrhenius=np.array([base.mech.arrhenius[0], [1e28, 0.0, 8000.0]]),
                               reversible=np.array([0, 0], np.uint8))
    prob = dataclasses.replace(base, mech=mech, name="abc_order6")
    s = lbm_mod.Solver(prob, storage=W.STORE_F64).init()
    s.step(30)
    mac = s.macros()
    assert s.status() == 0
    sim, anom = oracle_run(prob, 30)
    assert anom == 0
    err = field_errors(mac, sim.macros(), zeta_of(prob))
    print(f"[order 6] worst {max(err, key=err.get)} {max(err.values()):.2e}", flush=True)
    check_fp64(err, prob.name)
    s.close()
