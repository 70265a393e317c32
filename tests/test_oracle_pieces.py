"""Pins of the oracle's building blocks against what the mathematics fixes.

Each test checks an identity, closed form or invariant stated or implied by the
paper; none re-types the oracle's formula.
"""
import math
import os

import numpy as np
import pytest

from oracle import oracle as orc
from paper_2101_01702_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
C = np.array([[i % 3 - 1, (i // 3) % 3 - 1, i // 9 - 1] for i in range(27)], dtype=np.float64)


def _moments(f):
    return f.sum(), C.T @ f, np.einsum("i,ia,ib->ab", f, C, C)


# --- product-form equilibria (Sec. 2, eqs. phis/feq/fstar) ---------------------------
@pytest.mark.parametrize("seed", range(5))
def test_product_form_moments(oracle_lib, seed):
    """sum Psi = 1, Psi_1 - Psi_-1 = xi, Psi_1 + Psi_-1 = xi^2 + zeta per axis imply
    moments rho, rho u and rho (u u + zeta I) of the product form."""
    rng = np.random.default_rng(seed)
    rho, u, zeta = rng.uniform(0.3, 3), rng.uniform(-0.2, 0.2, 3), rng.uniform(0.02, 0.9)
    f = orc.product_form(rho, u, zeta)
    m0, m1, m2 = _moments(f)
    assert m0 == pytest.approx(rho, rel=1e-15, abs=0)
    np.testing.assert_allclose(m1, rho * u, rtol=0, atol=1e-15 * rho)
    np.testing.assert_allclose(m2, rho * (np.outer(u, u) + zeta * np.eye(3)), rtol=0, atol=2e-15 * rho)


def test_product_form_axis_factors(oracle_lib):
    """One-dimensional factors read off a population with the other two axes at rest."""
    xi, zeta = 0.13, 0.41
    f = orc.product_form(1.0, [xi, 0.0, 0.0], zeta)
    rest = (1 - zeta) ** 2  # Psi_0(0, zeta)^2 of the y and z axes
    psi = {c: f[(c + 1) + 3 * 1 + 9 * 1] / rest for c in (-1, 0, 1)}
    assert psi[0] == pytest.approx(1 - (xi * xi + zeta), rel=1e-15)
    assert psi[1] - psi[-1] == pytest.approx(xi, rel=1e-14)
    assert psi[1] + psi[-1] == pytest.approx(xi * xi + zeta, rel=1e-14)


# --- Grad form for g (eqs. gieq/giqeq) --------------------------------------------------
@pytest.mark.parametrize("seed", range(5))
def test_grad_form_moments(oracle_lib, seed):
    """On D3Q27 with theta = 1/3 the Grad form reproduces its 0th, 1st and 2nd moment."""
    rng = np.random.default_rng(100 + seed)
    rhoE = rng.uniform(-3, 3)
    q = rng.uniform(-1, 1, 3)
    A = rng.uniform(-1, 1, (3, 3))
    Rt = 0.5 * (A + A.T)
    g = orc.grad_form(rhoE, q, Rt)
    m0, m1, m2 = _moments(g)
    scale = max(1.0, abs(rhoE))
    assert abs(m0 - rhoE) <= 1e-14 * scale
    np.testing.assert_allclose(m1, q, rtol=0, atol=1e-14 * scale)
    np.testing.assert_allclose(m2, Rt, rtol=0, atol=1e-14 * scale)


def _golden(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return [ln.split() for ln in f if ln.strip() and not ln.startswith("#")]


def test_grad_weights_are_d3q27(oracle_lib):
    """The weights are the products of the paper's one-dimensional weights
    (tests/golden/d3q27_weights.txt: 8/27, 2/27, 1/54, 1/216 by |c|^2)."""
    g = orc.grad_form(1.0, np.zeros(3), np.eye(3) / 3.0)   # R = rhoE theta I: only the weight remains
    rows = _golden("d3q27_weights.txt")
    assert len(rows) == 27
    for i, cx, cy, cz, num, den in rows:
        i = int(i)
        assert (int(cx), int(cy), int(cz)) == tuple(C[i].astype(int))
        assert g[i] == pytest.approx(int(num) / int(den), rel=1e-15)


# --- thermodynamics (eq. specHa, Umix) ---------------------------------------------------
def _sim_h2air():
    return orc.OracleSim(W.flame1d(nx=8, steps=0))


@pytest.mark.parametrize("a", range(9))
def test_nasa7_enthalpy_is_integral_of_cp(oracle_lib, a):
    """dH/dT = C_p, dU/dT = C_v, d(s)/dT = c_p/T, H - U = R_a T, and H(T0) = h_f."""
    sim = _sim_h2air()
    mech = sim.prob.mech
    kappa = sim.prob.kappa
    Ra = kappa * W.R_U / (mech.molar_mass[a] * 1e-3)
    for T in (300.0, 900.0, 1800.0, 2900.0):
        h = 1e-4 * T
        tp, tm = sim.thermo(a, T + h), sim.thermo(a, T - h)
        t0 = sim.thermo(a, T)
        dH = (tp["H"] - tm["H"]) / (2 * h)
        dU = (tp["U"] - tm["U"]) / (2 * h)
        ds = (tp["s_R"] - tm["s_R"]) / (2 * h)
        assert dH == pytest.approx(Ra * t0["cp_R"], rel=1e-7)
        assert dU == pytest.approx(t0["Cv"], rel=1e-7)
        assert ds == pytest.approx(t0["cp_R"] / T, rel=1e-7)
        assert t0["H"] - t0["U"] == pytest.approx(Ra * T, rel=1e-12)


def test_formation_enthalpy_and_entropy_at_reference(oracle_lib):
    """The thermo data reproduce the formation enthalpy and entropy they were built
    from at T0 = 298.15 K (Sec. 4 reference state)."""
    ref = {k: float(v) for k, v in _golden("standard_state.txt")}
    T0 = ref["T0_K"]
    assert W.T_REF == T0 and W.P_ATM == ref["P0_Pa"]
    mech = W.abc_mechanism(h_f=(0.0, 1.0e4, -5.0e4), s0=(150.0, 200.0, 250.0), cp=(2.5, 3.5, 4.5))
    prob = W.config1()
    prob.mech = mech
    sim = orc.OracleSim(prob)
    for a, (hf, s0) in enumerate([(0.0, 150.0), (1.0e4, 200.0), (-5.0e4, 250.0)]):
        t = sim.thermo(a, T0)
        assert t["h_RT"] * W.R_U * T0 == pytest.approx(hf, abs=1e-6)
        assert t["s_R"] * W.R_U == pytest.approx(s0, rel=1e-13)


# --- temperature inversion (eq. temperature) -------------------------------------------
@pytest.mark.parametrize("seed", range(4))
def test_newton_round_trip(oracle_lib, seed):
    """T(E(T)) = T for random compositions and temperatures across the flame range."""
    rng = np.random.default_rng(seed)
    sim = _sim_h2air()
    M = sim.M
    for _ in range(10):
        Y = rng.dirichlet(np.ones(M))
        T = rng.uniform(280, 3200)
        e = sum(Y[a] * sim.thermo(a, T)["U"] for a in range(M))
        T_back, it = sim.temperature(Y, e, T * rng.uniform(0.6, 1.5))
        assert it > 0
        assert T_back == pytest.approx(T, rel=1e-13)


def test_newton_constant_cp_closed_form(oracle_lib):
    """With constant c_p, U_a is affine in T and the inversion has a closed form."""
    prob = W.config1()
    sim = orc.OracleSim(prob)
    mech = prob.mech
    Y = np.array([0.1, 0.3, 0.6])
    Ra = prob.kappa * W.R_U / (mech.molar_mass * 1e-3)
    a1, a6 = mech.nasa7[:, 0], mech.nasa7[:, 5]
    e = float((Y * Ra * (a1 - 1) * 1234.5).sum() + (Y * Ra * a6).sum())
    T_exact = (e - (Y * Ra * a6).sum()) / (Y * Ra * (a1 - 1)).sum()
    T, it = sim.temperature(Y, e, 700.0)
    assert T == pytest.approx(T_exact, rel=1e-14)
    assert 1 <= it <= 3


# --- production rates (Sec. 2 eq. sumRhoDot; Sec. 4 item 3) -------------------------------
@pytest.mark.parametrize("seed", range(6))
def test_rates_conserve_mass_and_elements(oracle_lib, seed):
    """sum_a rho_dot_a = 0 and every element is conserved by every reaction set."""
    rng = np.random.default_rng(seed)
    sim = _sim_h2air()
    mech = sim.prob.mech
    for _ in range(5):
        rho_a = rng.dirichlet(np.ones(sim.M)) * rng.uniform(0.2, 2.0)
        T = rng.uniform(600, 3000)
        rd = sim.rates(rho_a, T)
        scale = np.abs(rd).max()
        assert scale > 0
        assert abs(rd.sum()) <= 1e-13 * scale
        moles = rd / mech.molar_mass
        elem = mech.elements.T @ moles
        assert np.all(np.abs(elem) <= 1e-13 * np.abs(moles).max())


def test_rates_vanish_at_chemical_equilibrium(oracle_lib):
    """A reversible A+B<=>C at the composition where [C]/([A][B]) equals K_c from the
    Gibbs function has zero net rate.  With constant c_p the Gibbs function has the
    closed form G/(R T) = a1 (1 - ln T) + a6/T - a7."""
    mech = W.abc_mechanism(reversible=True, h_f=(0.0, 0.0, -50e3), cp=(2.5, 3.5, 4.5), A=3e8, Ta=4000)
    prob = W.config1()
    prob.mech = mech
    sim = orc.OracleSim(prob)
    T = 1400.0
    g = mech.nasa7[:, 0] * (1 - math.log(T)) + mech.nasa7[:, 5] / T - mech.nasa7[:, 6]
    nu = np.array([-1, -1, 1])
    c0 = W.P_ATM / (W.R_U * T) * 1e-6
    Kc = math.exp(-(nu * g).sum()) * c0 ** nu.sum()
    cA, cB = 2e-6, 3e-6
    cC = Kc * cA * cB
    conc = np.array([cA, cB, cC])
    rho_a = conc * mech.molar_mass / prob.rho_ref
    rd = sim.rates(rho_a, T)
    # compare against the forward rate alone: equilibrium means cancellation
    kf = 3e8 * math.exp(-4000 / T)
    fwd_scale = mech.molar_mass[0] * kf * cA * cB * prob.dt_phys / prob.rho_ref
    assert np.abs(rd).max() <= 1e-12 * fwd_scale
    # off equilibrium the reaction runs toward it
    rd2 = sim.rates(rho_a * np.array([1.1, 1.0, 1.0]), T)
    assert rd2[2] > 0 and rd2[0] < 0


def test_rate_arrhenius_temperature_dependence(oracle_lib):
    """At fixed concentrations ln|rate| is linear in 1/T with slope -Ta, and scales as
    T^b (A+B->C irreversible)."""
    for b in (0.0, 0.7):
        mech = W.abc_mechanism(A=1e6, b=b, Ta=8000.0)
        prob = W.config1()
        prob.mech = mech
        sim = orc.OracleSim(prob)
        rho_a = np.array([0.05, 0.4, 0.55])
        Ts = np.array([800.0, 1000.0, 1300.0, 1700.0])
        r = np.array([-sim.rates(rho_a, T)[0] for T in Ts])
        y = np.log(r) - b * np.log(Ts)
        slope = np.polyfit(1 / Ts, y, 1)[0]
        assert slope == pytest.approx(-8000.0, rel=1e-10)


# --- Stefan-Maxwell diffusion velocities (eqs. tauab, transform1) -------------------------
@pytest.mark.parametrize("seed", range(5))
def test_diffusion_velocities_carry_no_mass(oracle_lib, seed):
    """sum_a rho_a du_a = 0 whenever sum_a rho_a (u_a - u) = 0 (symmetric tau_ab)."""
    rng = np.random.default_rng(seed)
    sim = _sim_h2air()
    M = sim.M
    Y = rng.dirichlet(np.ones(M))
    rhs = rng.uniform(-0.05, 0.05, (M, 3))
    rhs[-1] = -(Y[:-1, None] * rhs[:-1]).sum(0) / Y[-1]
    du, beta = sim.diffusion(Y, rng.uniform(300, 2500), rhs)
    np.testing.assert_allclose((Y[:, None] * du).sum(0), 0.0, atol=1e-14 * np.abs(Y[:, None] * du).sum())
    assert np.all((beta > 0) & (beta < 1))


def test_diffusion_velocities_binary_closed_form(oracle_lib):
    """Two species: du_a = (u_a - u) / (1 + 1/(2 tau_12)) and beta_a = Y_b/tau_12 /
    (2 + Y_b/tau_12), with 1/tau_12 = m R_U T / (m_1 m_2 D_12) (eq. tauab)."""
    prob = W.config1()
    mech = W.abc_mechanism(R_count=0)
    mech.names, mech.molar_mass = mech.names[:2], mech.molar_mass[:2]
    mech.nasa7, mech.elements = mech.nasa7[:2], mech.elements[:2]
    mech.nu_reac = np.zeros((0, 2), np.int32)
    mech.nu_prod = np.zeros((0, 2), np.int32)
    prob.mech = mech
    prob.diff = np.array([[0.0, 0.045], [0.045, 0.0]])
    prob.Y = prob.Y[:2] / prob.Y[:2].sum(0)
    sim = orc.OracleSim(prob)
    Y = np.array([0.2, 0.8])
    T = 1234.0
    r1 = np.array([0.01, -0.02, 0.005])
    rhs = np.stack([r1, -Y[0] / Y[1] * r1])
    du, beta = sim.diffusion(Y, T, rhs)
    m = 1.0 / (Y / mech.molar_mass).sum()
    # tau_12 in physical form, then to lattice units with kappa (zeta = kappa R T)
    inv_tau = prob.kappa * (m * 1e-3) * W.R_U * T / ((mech.molar_mass[0] * 1e-3) * (mech.molar_mass[1] * 1e-3) * 0.045)
    np.testing.assert_allclose(du, rhs / (1 + 0.5 * inv_tau), rtol=1e-13)
    assert beta[0] == pytest.approx(Y[1] * inv_tau / (2 + Y[1] * inv_tau), rel=1e-13)
    assert beta[1] == pytest.approx(Y[0] * inv_tau / (2 + Y[0] * inv_tau), rel=1e-13)


# --- isotropic lattice gradient (Sec. 3, Thampi et al.) -----------------------------------
def _grid_sim(nx, ny, nz, bc):
    prob = W.config1(nx=nx, ny=ny, nz=nz)
    prob.bc = bc
    return orc.OracleSim(prob)


def test_iso_grad_exact_on_quadratics(oracle_lib):
    """Second-order stencil: exact on polynomials of degree <= 2 (interior nodes)."""
    nx, ny, nz = 9, 8, 7
    sim = _grid_sim(nx, ny, nz, (1,) * 6)
    n = np.arange(nx * ny * nz)
    x, y, z = n % nx, (n // nx) % ny, n // (nx * ny)
    f = 0.3 * x * x - 1.1 * x * y + 0.7 * z * z + 2.0 * y - 0.25 * x * z + 5.0
    g = sim.iso_grad(f)
    inner = (x > 0) & (x < nx - 1) & (y > 0) & (y < ny - 1) & (z > 0) & (z < nz - 1)
    np.testing.assert_allclose(g[0][inner], (0.6 * x - 1.1 * y - 0.25 * z)[inner], atol=1e-12)
    np.testing.assert_allclose(g[1][inner], (-1.1 * x + 2.0)[inner], atol=1e-12)
    np.testing.assert_allclose(g[2][inner], (1.4 * z - 0.25 * x)[inner], atol=1e-12)


def test_iso_grad_fourier_symbol(oracle_lib):
    """On a periodic lattice the stencil maps sin(kx) to sin(k) cos(kx)."""
    nx = 16
    sim = _grid_sim(nx, 3, 2, (0,) * 6)
    n = np.arange(nx * 3 * 2)
    x = n % nx
    k = 2 * math.pi * 3 / nx
    g = sim.iso_grad(np.sin(k * x))
    np.testing.assert_allclose(g[0], math.sin(k) * np.cos(k * x), atol=1e-14)
    np.testing.assert_allclose(g[1:], 0.0, atol=1e-14)


def test_iso_grad_zero_gradient_at_open_faces(oracle_lib):
    """Open faces clamp the neighbour to the boundary node: a field constant across the
    face has a one-sided (halved) difference at the boundary node."""
    nx = 6
    sim = _grid_sim(nx, 1, 1, (1, 1, 0, 0, 0, 0))
    x = np.arange(nx, dtype=float)
    g = sim.iso_grad(x)
    np.testing.assert_allclose(g[0][1:-1], 1.0, atol=1e-14)
    assert g[0][0] == pytest.approx(0.5, abs=1e-14)
    assert g[0][-1] == pytest.approx(0.5, abs=1e-14)
