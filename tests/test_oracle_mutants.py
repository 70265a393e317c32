"""The pins must catch plausible mistakes.

Each case plants one mistake in a temporary copy of the oracle source (a dropped
term, a wrong sign, a wrong factor, a transposed operand), builds it, and checks that
at least one pin of the battery below fails on it, while all of them hold on the
unmodified oracle.  The planted mistakes live only in the temporary copy.
"""
import math
import os
import shutil

import numpy as np
import pytest

from oracle import build as obuild
from oracle import oracle as orc
from paper_2101_01702_amd import workloads as W

from oracle_cases import CI, fourier_amp, lattice_problem, moments, two_species

MUTANTS = {
    "drop_qdiff": ("qstar[a] = d->q[a] - uPdiff + qdiff + qcorr;", "qstar[a] = d->q[a] - uPdiff + qcorr;"),
    "drop_qcorr": ("qstar[a] = d->q[a] - uPdiff + qdiff + qcorr;", "qstar[a] = d->q[a] - uPdiff + qdiff;"),
    "drop_viscous_heating": ("qstar[a] = d->q[a] - uPdiff + qdiff + qcorr;", "qstar[a] = d->q[a] + qdiff + qcorr;"),
    "x_sign": ("of[(int64_t)i * N + n] = f + om * (feq - f) + AX;", "of[(int64_t)i * N + n] = f + om * (feq - f) - AX;"),
    "fstar_raw_velocity": ("ub[a] = d->u[a] + d->du[b][a];", "ub[a] = d->u_a[b][a];"),
    "source_weight": ("(d->beta[sp] - 1.0) * F + src;", "(d->beta[sp] - 1.0) * F + (1.0 - d->beta[sp]) * src;"),
    "beta_factor": ("f + 2.0 * d->beta[sp] * (feq - f)", "f + d->beta[sp] * (feq - f)"),
    "interspecies_sign": ("(d->beta[sp] - 1.0) * F + src;", "(1.0 - d->beta[sp]) * F + src;"),
    "grad_divisor": ("contr / (2.0 * THETA * THETA)", "contr / (THETA * THETA)"),
    "psi_mirror_sign": ("iso_grad_v(s, fld, n, a, a);", "iso_grad_v(s, fld, n, a, -1);"),
    "mirror_direction": ("const int im = mirror_dir(i, mirror);", "const int im = i;"),
    "diff_T_inverted": ("pow(T / s->p.diff_T_ref, s->p.diff_T_exp)", "pow(s->p.diff_T_ref / T, s->p.diff_T_exp)"),
    "visc_T_inverted": ("*om = 1.0 / (0.5 + (1.0 / s->p.omega - 0.5) * sc);",
                        "*om = 1.0 / (0.5 + (1.0 / s->p.omega - 0.5) / sc);"),
    "sd_drop_enthalpy_flux": ("Sd = (hrr + div - d[n].rho * flux)", "Sd = (hrr + div)"),
    "sd_lambda_factor": ("lam[n] = (1.0 / om1 - 0.5) * d[n].P * cp[n];", "lam[n] = (1.0 / om1) * d[n].P * cp[n];"),
    "sa_sign": ("for (int a = 0; a < 3; ++a) un -= d[n].u[a] * gT[a * N + n] / mag;",
                "for (int a = 0; a < 3; ++a) un += d[n].u[a] * gT[a * N + n] / mag;"),
    "psi_sign": ("if (c == 1) return 0.5 * (xi + s);", "if (c == 1) return 0.5 * (-xi + s);"),
    "kc_sign": ("const real Kc = exp(-dG) * pow(c0, dnu);", "const real Kc = exp(dG) * pow(c0, dnu);"),
    "kinetic_energy_half": ("E - usq / 2.0, T_start", "E - usq, T_start"),
    "transform_sign": ("-0.5 * K[a][b] * Y[b];", "0.5 * K[a][b] * Y[b];"),
    "stream_direction": ("int v = xyz[a] - CI(i, a);", "int v = xyz[a] + CI(i, a);"),
    "iso_grad_scale": ("return acc / THETA;", "return acc;"),
    "tau_ab_mixture_mass": ("zeta_a[a] * zeta_a[b] / (zeta * diffusivity(s, a, b, T))",
                            "zeta_a[a] * zeta_a[b] / (diffusivity(s, a, b, T))"),
    "ghost_velocity": ("for (int a = 0; a < 3; ++a) ug[a] = zero_u ? (real)0.0 : d->u[a];",
                       "for (int a = 0; a < 3; ++a) ug[a] = 0.0;"),
    "slaved_momentum": ("d->j_a[M - 1][a] = d->j[a] - j_sum[a];", "d->j_a[M - 1][a] = d->j[a] + j_sum[a];"),
    "phi_cubic_sign": ("- d->rho * d->u[a] * d->u[a] * d->u[a];", "+ d->rho * d->u[a] * d->u[a] * d->u[a];"),
}


# ---- pin battery (each returns True when the pin holds) --------------------------------
def pin_moments(lib):
    rng = np.random.default_rng(0)
    u = rng.uniform(-0.2, 0.2, 3)
    f = orc.product_form(1.3, u, 0.3, lib=lib)
    ok = abs(f.sum() - 1.3) < 1e-13 and np.allclose(CI.T @ f, 1.3 * u, atol=1e-13)
    A = rng.uniform(-1, 1, (3, 3))
    Rt = A + A.T
    q = rng.uniform(-1, 1, 3)
    g = orc.grad_form(0.7, q, Rt, lib=lib)
    ok &= abs(g.sum() - 0.7) < 1e-13 and np.allclose(CI.T @ g, q, atol=1e-13)
    ok &= np.allclose(np.einsum("i,ia,ib->ab", g, CI, CI), Rt, atol=1e-13)
    return bool(ok)


def pin_collision(lib):
    prob = W.perturb_velocity(W.config1(nx=8, ny=3, nz=2), 0.02, 3)
    sim = orc.OracleSim(prob, lib=lib).init()
    pop, T = sim.state()
    pop = pop * (1.0 + 0.01 * np.random.default_rng(3).uniform(-1, 1, pop.shape))
    sim.set_state(pop, T)
    sim.step(1)
    post = sim.post()
    M = prob.M
    a, b = moments(pop, M), moments(post, M)
    X, rdot, du = sim.field(orc.F_X), sim.field(orc.F_RDOT), sim.field(orc.F_DU)
    u = a["j"] / a["rho"]
    ok = np.allclose(b["rho"], a["rho"], rtol=1e-13) and np.allclose(b["rhoE"], a["rhoE"], rtol=1e-12)
    ok &= np.allclose(b["j"], a["j"] + X, atol=1e-13)
    for s in range(M - 1):
        ok &= np.allclose(b["rho_a"][s], a["rho_a"][s] + rdot[s], rtol=1e-12)
        ok &= np.allclose(b["j_a"][s], 2 * a["rho_a"][s] * (u + du[s]) - a["j_a"][s] + rdot[s] * u, atol=1e-13)
    return bool(ok)


def pin_conservation(lib):
    prob = W.config1()
    x = np.arange(prob.N) % prob.nx
    prob.u[0] = 0.01 * np.sin(2 * math.pi * x / prob.nx)
    sim = orc.OracleSim(prob, lib=lib).init()
    mech = prob.mech

    def totals():
        mo = moments(sim.state()[0], prob.M)
        elem = (mech.elements.T @ (mo["rho_a"] / mech.molar_mass[:, None])).sum(1)
        return mo["rho"].sum(), mo["j"].sum(1), mo["rhoE"].sum(), elem

    t0 = totals()
    if sim.step(60) != 0:
        return False
    t1 = totals()
    return bool(abs(t1[0] - t0[0]) < 1e-12 * t0[0] and np.allclose(t1[1], t0[1], atol=1e-11)
                and abs(t1[2] - t0[2]) < 1e-11 * abs(t0[2]) and np.allclose(t1[3], t0[3], rtol=1e-11))


def pin_init_round_trip(lib):
    prob = W.perturb_velocity(W.config1(nx=6, ny=2, nz=2), 0.05, 4)
    mac = orc.OracleSim(prob, lib=lib).init().macros()
    return bool(np.allclose(mac["T"], prob.T, rtol=1e-12) and np.allclose(mac["u"], prob.u, atol=1e-14)
                and np.allclose(mac["Y"], prob.Y, rtol=1e-12) and np.allclose(mac["rho"], prob.rho, rtol=1e-14))


def _rate(sim, getter, L, n_meas, every):
    amps, ts = [], []
    for n in range(n_meas):
        amps.append(fourier_amp(getter(sim.macros()), L))
        ts.append(n * every)
        if sim.step(every):
            return float("nan")
    return -np.polyfit(ts, np.log(amps), 1)[0]


def pin_fick(lib):
    L, D = 48, 0.05
    X1 = 0.5 + 1e-3 * np.sin(2 * math.pi * np.arange(L) / L)
    prob = lattice_problem(two_species(), L, X=np.stack([X1, 1 - X1]), D=D)
    r = _rate(orc.OracleSim(prob, lib=lib).init(), lambda m: m["Y"][0] - m["Y"][0].mean(), L, 4, 200)
    return bool(abs(r / (D * (2 * math.pi / L) ** 2) - 1) < 0.02)


def pin_shear(lib):
    L = 48
    u = np.zeros((3, L))
    u[1] = 1e-3 * np.sin(2 * math.pi * np.arange(L) / L)
    prob = lattice_problem(two_species(), L, u=u, omega=1.4)
    nu = (1 / 1.4 - 0.5) * prob.kappa * W.R_U * 1000.0 / 28e-3
    r = _rate(orc.OracleSim(prob, lib=lib).init(), lambda m: m["u"][1], L, 4, 150)
    return bool(abs(r / (nu * (2 * math.pi / L) ** 2) - 1) < 0.02)


def pin_thermal(lib):
    L = 48
    Tf = 1000.0 * (1 + 2e-3 * np.sin(2 * math.pi * np.arange(L) / L))
    prob = lattice_problem(two_species(), L, T_field=Tf, omega=1.3)
    alpha = (1 / prob.omega1 - 0.5) * prob.kappa * W.R_U * 1000.0 / 28e-3
    r = _rate(orc.OracleSim(prob, lib=lib).init(), lambda m: m["T"] - 1000.0, L, 6, 100)
    return bool(abs(r / (alpha * (2 * math.pi / L) ** 2) - 1) < 0.05)


def pin_interdiffusion(lib):
    from test_oracle_step import interdiffusion_temperature_drift
    drift, scale = interdiffusion_temperature_drift(lambda p: orc.OracleSim(p, lib=lib), steps=300)
    return bool(drift < 2e-3 * scale)


def pin_reactor(lib):
    hC = -W.R_U * W.T_REF
    mech = W.abc_mechanism(A=2e8, Ta=6000.0, cp=(2.5, 2.5, 4.0), h_f=(0.0, 0.0, hC))
    prob = lattice_problem(mech, 1, 1, 1, X=[0.35, 0.25, 0.4], zeta_ref=0.05, dt_phys=0.05)
    sim = orc.OracleSim(prob, lib=lib).init()
    mac = sim.macros()
    c = mac["Y"][:, 0] * mac["rho"][0] * prob.rho_ref / mech.molar_mass
    k = 2e8 * math.exp(-6.0)
    for _ in range(20):
        q = k * c[0] * c[1] * prob.dt_phys
        c = c + np.array([-q, -q, q])
    sim.step(20)
    mac = sim.macros()
    co = mac["Y"][:, 0] * mac["rho"][0] * prob.rho_ref / mech.molar_mass
    return bool(np.allclose(co, c, rtol=1e-11))


def pin_equilibrium(lib):
    mech = W.abc_mechanism(reversible=True, cp=(2.5, 3.5, 4.5), A=3e8, Ta=4000)
    prob = W.config1()
    prob.mech = mech
    sim = orc.OracleSim(prob, lib=lib)
    T = 1400.0
    g = mech.nasa7[:, 0] * (1 - math.log(T)) + mech.nasa7[:, 5] / T - mech.nasa7[:, 6]
    nu = np.array([-1, -1, 1])
    Kc = math.exp(-(nu * g).sum()) * (W.P_ATM / (W.R_U * T) * 1e-6) ** nu.sum()
    conc = np.array([2e-6, 3e-6, Kc * 6e-12])
    rd = sim.rates(conc * mech.molar_mass / prob.rho_ref, T)
    fwd = 2 * 3e8 * math.exp(-4000 / T) * 6e-12 * prob.dt_phys / prob.rho_ref
    return bool(np.abs(rd).max() < 1e-10 * fwd)


def pin_iso_grad(lib):
    prob = W.config1(nx=16, ny=3, nz=2)
    sim = orc.OracleSim(prob, lib=lib)
    x = np.arange(prob.N) % 16
    k = 2 * math.pi * 3 / 16
    g = sim.iso_grad(np.sin(k * x))
    return bool(np.allclose(g[0], math.sin(k) * np.cos(k * x), atol=1e-13))


def pin_advection(lib):
    """A composition bump carried by a uniform flow moves downstream at u."""
    L = 64
    x = np.arange(L)
    X1 = 0.5 + 0.05 * np.exp(-((x - 20.0) / 4.0) ** 2)
    u = np.zeros((3, L))
    u[0] = 0.05
    prob = lattice_problem(two_species(), L, X=np.stack([X1, 1 - X1]), u=u, D=0.2)
    sim = orc.OracleSim(prob, lib=lib).init()
    sim.step(200)
    y = sim.macros()["Y"][0]
    y = y - y.min()
    centre = (x * y).sum() / y.sum()
    return bool(abs(centre - 30.0) < 1.5)


def pin_open_boundary(lib):
    """Uniform flow with open faces stays uniform; a zero-velocity face reflects it."""
    mech = W.abc_mechanism(R_count=0)
    N = 5 * 4 * 3
    u = np.tile(np.array([[0.03], [-0.02], [0.01]]), (1, N))
    prob = lattice_problem(mech, 5, 4, 3, bc=(1,) * 6, X=[0.3, 0.3, 0.4], u=u)
    sim = orc.OracleSim(prob, lib=lib).init()
    p0, _ = sim.state()
    sim.step(10)
    return bool(np.allclose(sim.state()[0], p0, atol=1e-13))


def pin_viscous_work(lib):
    from test_oracle_step import viscous_work_flux_after_collision
    f = lambda p: orc.OracleSim(p, lib=lib)
    q1, _ = viscous_work_flux_after_collision(1.2, f)
    q2, _ = viscous_work_flux_after_collision(0.8, f)
    return bool(np.allclose(q1, q2, rtol=0, atol=1e-12 * np.abs(q1).max()))


def pin_sound_galilean(lib):
    from test_oracle_step import sound_damping
    f = lambda p: orc.OracleSim(p, lib=lib)
    g0, g1 = sound_damping(0.0, f), sound_damping(0.1, f)
    return bool(g0 > 0 and abs(g1 / g0 - 1) < 0.15)


def pin_symmetry_face(lib):
    """A half lattice with a symmetry face against the mirror-symmetric full lattice."""
    from test_oracle_symmetry import _mirror_pair
    fm, hm, keep = _mirror_pair(0, L=4, other=(3, 2), steps=20, lib=lib)
    return bool(np.abs(hm["T"] - fm["T"][keep]).max() <= 1e-12 * fm["T"].max()
                and np.abs(hm["u"][0] - fm["u"][0][keep]).max() <= 1e-12 * np.sqrt(0.05))


def pin_transport_laws(lib):
    """Binary decay at D_ref (T/T_ref)^n k^2 and shear decay at (1/omega(T) - 1/2) R T k^2."""
    L, T = 48, 1000.0
    X1 = 0.5 + 1e-3 * np.sin(2 * math.pi * np.arange(L) / L)
    prob = lattice_problem(two_species(), L, X=np.stack([X1, 1 - X1]), D=0.02, T=T)
    prob.diff_T_ref, prob.diff_T_exp = 500.0, 1.5
    r = _rate(orc.OracleSim(prob, lib=lib).init(), lambda m: m["Y"][0] - m["Y"][0].mean(), L, 4, 200)
    ok = abs(r / (0.02 * 2.0 ** 1.5 * (2 * math.pi / L) ** 2) - 1) < 0.02
    u = np.zeros((3, L))
    u[1] = 1e-3 * np.sin(2 * math.pi * np.arange(L) / L)
    prob = lattice_problem(two_species(), L, u=u, omega=1.6, T=T)
    prob.visc_T_ref, prob.visc_T_exp = 500.0, 0.7
    nu = (1 / 1.6 - 0.5) * 2.0 ** 0.7 * prob.kappa * W.R_U * T / 28e-3
    r = _rate(orc.OracleSim(prob, lib=lib).init(), lambda m: m["u"][1], L, 4, 150)
    return bool(ok and abs(r / (nu * (2 * math.pi / L) ** 2) - 1) < 0.02)


def pin_front_speeds(lib):
    """S_d and S_a move the isotherms (the conduction and enthalpy-diffusion cases of the
    flame-speed pins)."""
    from test_oracle_flame_speeds import CASES, _run
    for case in ("conduction", "enthalpy diffusion"):
        make, settle, frac, tol = CASES[case]
        fs, g, u, dTdt, pw = _run(make(), settle, lib=lib)
        mag = np.abs(g)
        sel = mag > frac * mag.max()
        DTDt = dTdt + u * g
        if np.abs(fs["Sd"] * mag + pw - DTDt)[sel].max() > tol * np.abs(DTDt[sel]).max():
            return False
        if np.abs(fs["Sa"] * mag + pw - dTdt)[sel].max() > tol * np.abs(dTdt[sel]).max():
            return False
    return True


BATTERY = [pin_viscous_work, pin_sound_galilean, pin_moments, pin_collision, pin_conservation, pin_init_round_trip, pin_fick, pin_shear,
           pin_thermal, pin_interdiffusion, pin_reactor, pin_equilibrium, pin_iso_grad, pin_advection,
           pin_open_boundary, pin_symmetry_face, pin_transport_laws, pin_front_speeds]


def _run_battery(lib, stop_at_failure=False):
    """Results of the pins on lib; with stop_at_failure, up to the first pin that fails."""
    res = {}
    for pin in BATTERY:
        try:
            res[pin.__name__] = pin(lib)
        except (ValueError, FloatingPointError, np.linalg.LinAlgError):
            res[pin.__name__] = False
        if stop_at_failure and not res[pin.__name__]:
            break
    return res


def test_battery_holds_on_oracle():
    res = _run_battery(orc.load())
    assert all(res.values()), res


@pytest.fixture(scope="module")
def mutant_dir(tmp_path_factory):
    return tmp_path_factory.mktemp("mutants")


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_planted_mistake(name, mutant_dir):
    old, new = MUTANTS[name]
    src = open(os.path.join(obuild.HERE, "oracle.c")).read()
    assert src.count(old) == 1, f"mutation site for {name} not found exactly once"
    d = mutant_dir / name
    d.mkdir()
    shutil.copy(os.path.join(obuild.HERE, "oracle.h"), d / "oracle.h")
    (d / "oracle.c").write_text(src.replace(old, new))
    so = obuild.build(src=str(d / "oracle.c"), out=str(d / "liboracle_mutant.so"))
    with np.errstate(all="ignore"):
        res = _run_battery(orc.load(so), stop_at_failure=True)
    assert not all(res.values()), f"no pin caught mutant {name}"
