"""16-bit deviation storage of the populations against the FP64 oracle.

One step from the GPU's own decoded state: the oracle advances the same state, and
every population may differ from the oracle's by the rounding of its stored deviation,
u |f - f_ref| with u = 2^-11 (FP16) or 2^-8 (BF16) and f_ref the equilibrium of its
set at the reference state at rest, or by half the format's smallest step at the set's
scale sc_s (FP16 subnormals end at 2^-24 sc_s: a species near the 1e-12 floor of the
premixture is below it and reads as its reference value), plus rounding at FP32 level
(side fields, corrections, the inter-species term).  These rounding errors accumulate over steps: a
200-step run of configuration 1 ends at about 8e-4 field error in FP16, the flame far
higher, so the formats do not reach 1e-4 (measured by bench.py --storage f16dev).
"""
import numpy as np
import pytest

from oracle import oracle as orc
from paper_2101_01702_amd import workloads as W

pytestmark = pytest.mark.gpu

U16 = {W.STORE_F16_DEV: 2.0 ** -11, W.STORE_BF16_DEV: 2.0 ** -8}
TINY = {W.STORE_F16_DEV: 2.0 ** -24, W.STORE_BF16_DEV: 2.0 ** -133}


def set_scales(prob, ref_state, fref):
    """sc_s of the deviation formats: 1e-3 of the reference mixture density for f and
    every species, 1e-3 of sum_i |g_ref,i| for g."""
    sc = np.full(prob.M + 1, 1e-3 * ref_state[0])
    sc[prob.M] = 1e-3 * np.abs(fref[prob.M]).sum()
    return sc[:, None, None]


def format_bound(storage, want, fref, sc, scale, fp32_rel):
    return (1.05 * U16[storage] * np.abs(want - fref[:, :, None]) + 0.5 * TINY[storage] * sc
            + fp32_rel * scale)


@pytest.fixture(scope="module")
def lbm_mod():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2101_01702_amd import lbm
    lbm.load()
    return lbm


def reference_populations(prob, ref_state):
    """f_ref[s][i]: equilibria of the species a < M-1, f and g at the reference state
    at rest, from the oracle's product and Grad forms (eqs. feq, gieq)."""
    sim = orc.OracleSim(prob)
    M = prob.M
    rho, T, Y = ref_state[0], ref_state[1], np.asarray(ref_state[2:])
    Ra = prob.kappa * W.R_U / (prob.mech.molar_mass * 1e-3)
    za = Ra * T
    zeta = float((Y * za).sum())
    U = sum(Y[a] * sim.thermo(a, T)["U"] for a in range(M))
    H = sum(Y[a] * sim.thermo(a, T)["H"] for a in range(M))
    out = np.zeros((M + 1, 27))
    for a in range(M - 1):
        out[a] = orc.product_form(rho * Y[a], np.zeros(3), za[a])
    out[M - 1] = orc.product_form(rho, np.zeros(3), zeta)
    out[M] = orc.grad_form(rho * U, np.zeros(3), H * rho * zeta * np.eye(3))
    return out


def _problem(case):
    if case == "config1":
        return W.config1()
    if case == "flame1d":
        return W.flame1d(nx=128, hot_cells=32)
    if case == "flame_batch":      # x ghost cells per segment
        return W.flame_batch(lengths=[60, 17, 40], phis=[1.0, 2.5, 0.7], hot_cells=12)
    prob = W.perturb_velocity(W.sphere3d(shape=(13, 10, 9), radius=3.0), 2e-3, 9)
    if case == "sphere3d_symmetry":   # mirror copies of the stored deviations
        prob.bc = (W.BC_SYMMETRY, W.BC_OPEN, W.BC_SYMMETRY, W.BC_OPEN, W.BC_OPEN_U0, W.BC_SYMMETRY)
    return prob


def _oracle_one_step(prob, pop, T):
    """The oracle's step from the given state; a batch is stepped lattice by lattice."""
    want, want_T = np.zeros_like(pop), np.zeros_like(T)
    parts = W.split_batch(prob)
    for k, part in enumerate(parts):
        idx = W.batch_nodes(prob, k) if prob.segments else np.arange(prob.N)
        sim = orc.OracleSim(part)
        sim.set_state(np.ascontiguousarray(pop[..., idx]), np.ascontiguousarray(T[idx]))
        assert sim.step(1) == 0
        w, wT = sim.state()
        want[..., idx] = w
        want_T[idx] = wT
    return want, want_T


@pytest.mark.parametrize("storage", [W.STORE_F16_DEV, W.STORE_BF16_DEV])
@pytest.mark.parametrize("case", ["config1", "flame1d", "sphere3d", "sphere3d_symmetry", "flame_batch"])
def test_one_step_within_format_rounding(lbm_mod, storage, case):
    prob = _problem(case)
    s = lbm_mod.Solver(prob, storage=storage).init()
    s.step(3)                                   # non-equilibrium parts, pending corrections
    nodes = np.arange(prob.N)
    pop, T = s.populations(nodes)
    want, want_T = _oracle_one_step(prob, pop, T)
    s.step(1)
    got, got_T = s.populations(nodes)
    assert s.status() == 0
    fref = reference_populations(prob, s.ref_state)
    scale = np.abs(want).max(axis=(1, 2), keepdims=True)
    bound = format_bound(storage, want, fref, set_scales(prob, s.ref_state, fref), scale, 4e-6)
    excess = (np.abs(got - want) / bound).max()
    rel = (np.abs(got - want) / scale).max()
    print(f"[{case} storage={storage}] max |err|/bound {excess:.3f}, max rel {rel:.2e}", flush=True)
    assert excess <= 1.0
    np.testing.assert_allclose(got_T, want_T, rtol=1e-12)


@pytest.mark.parametrize("storage", [W.STORE_F16_DEV, W.STORE_BF16_DEV])
def test_initial_state_encodes_equilibria(lbm_mod, storage):
    """The initial populations are the equilibria of the fields, stored to the format's
    rounding of their deviation."""
    prob = W.sphere3d(shape=(9, 8, 7), radius=2.5)
    s = lbm_mod.Solver(prob, storage=storage).init()
    got, _ = s.populations(np.arange(prob.N))
    sim = orc.OracleSim(prob).init()
    want, _ = sim.state()
    fref = reference_populations(prob, s.ref_state)
    scale = np.abs(want).max(axis=(1, 2), keepdims=True)
    bound = format_bound(storage, want, fref, set_scales(prob, s.ref_state, fref), scale, 1e-6)
    assert (np.abs(got - want) <= bound).all()
