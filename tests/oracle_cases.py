"""Small lattice problems for the oracle pins (built from the shared workload helpers)."""
import math

import numpy as np

from paper_2101_01702_amd import workloads as W


def two_species(m=(28.0, 28.0), h_f=(0.0, 0.0), cp=(3.5, 3.5), s0=(200.0, 200.0)):
    names = ["P", "Q"]
    nasa = np.stack([W.nasa7_coeffs((cp[a], 0, 0, 0, 0), h_f[a], s0[a]) for a in range(2)])
    z = np.zeros((0, 2), np.int32)
    return W.Mechanism(names, np.array(m, float), np.eye(2, dtype=np.int32), nasa, 200.0, 4000.0,
                       z, z.copy(), np.zeros((0, 3)), np.zeros(0, np.uint8))


def lattice_problem(mech, nx, ny=1, nz=1, bc=(0,) * 6, D=0.05, T=1000.0, X=None, u=None,
                    zeta_ref=0.1, omega=1.6, prandtl=0.7, dt_phys=0.41, P=W.P_ATM, T_field=None):
    """Uniform-pressure lattice with mole fractions X [M, N] (or [M]) and temperature."""
    M = mech.M
    N = nx * ny * nz
    if X is None:
        X = np.full(M, 1.0 / M)
    X = np.asarray(X, float)
    if X.ndim == 1:
        X = np.repeat(X[:, None], N, axis=1)
    m = W.mean_molar_mass(X, mech.molar_mass)
    kappa, rho_ref = W.lattice_scales(zeta_ref, T, float(m.mean()), P)
    Tf = np.full(N, T) if T_field is None else np.asarray(T_field, float)
    rho = W.lattice_density(np.full(N, P), Tf, m, rho_ref)
    Y = W.mole_to_mass(X, mech.molar_mass)
    Dm = np.full((M, M), D) if np.isscalar(D) else np.asarray(D, float)
    Dm = Dm.copy()
    np.fill_diagonal(Dm, 0.0)
    uu = np.zeros((3, N)) if u is None else np.asarray(u, float)
    return W.Problem("test", nx, ny, nz, tuple(bc), mech, Dm, omega,
                     W.omega1_from_prandtl(omega, prandtl), kappa, dt_phys, rho_ref, P,
                     rho, uu, Tf, Y)


def fourier_amp(field, nx, mode=1):
    """Amplitude of sin/cos mode ``mode`` along x of a 1D field."""
    x = np.arange(nx)
    k = 2 * math.pi * mode / nx
    a = 2.0 / nx * (field * np.sin(k * x)).sum()
    b = 2.0 / nx * (field * np.cos(k * x)).sum()
    return math.hypot(a, b)


CI = np.array([[i % 3 - 1, (i // 3) % 3 - 1, i // 9 - 1] for i in range(27)], dtype=np.float64)


def moments(pop, M):
    """Per-node moments straight from the populations [S, 27, N] (definitions of Sec. 2/3)."""
    f = pop[M - 1]
    g = pop[M]
    rho = f.sum(0)
    j = np.einsum("in,ia->an", f, CI)
    rhoE = g.sum(0)
    rho_a = pop[: M - 1].sum(1)
    j_a = np.einsum("sin,ia->san", pop[: M - 1], CI)
    rho_all = np.concatenate([rho_a, (rho - rho_a.sum(0))[None]], 0)
    j_all = np.concatenate([j_a, (j - j_a.sum(0))[None]], 0)
    return dict(rho=rho, j=j, rhoE=rhoE, rho_a=rho_all, j_a=j_all)
