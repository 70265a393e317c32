"""Seeded synthetic workloads for the reactive-mixture LBM step.

This module only builds inputs: species tables, a reaction list, transport and
relaxation constants, lattice scales and initial fields (rho, u, T, Y).  It holds
none of the lattice Boltzmann arithmetic (no equilibria, no collision, no
temperature inversion, no production rates); both the HIP path and the CPU oracle
consume what it returns.

Units
-----
* Lattice units: dx = dt = 1, lattice density rho (1 lattice unit = ``rho_ref``
  g/cm^3), velocities in lattice units, temperature in Kelvin.
* ``kappa`` [s^2/m^2] scales specific energies: the lattice value of R_a*T is
  kappa * R_U * T / m_a with m_a in kg/mol.
* ``dt_phys`` [s] is the physical time of one step, used only by the chemistry.
* Arrhenius pre-exponentials are in CGS (cm^3, mol, s), activation temperatures
  in K.

Node ordering: n = x + nx*(y + ny*z) (x fastest).
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence, Tuple

import numpy as np

R_U = 8.314462618          # J/(mol K)
P_ATM = 101325.0           # Pa
T_REF = 298.15             # K, standard-state temperature of the thermo data

BC_PERIODIC = 0
BC_OPEN = 1                # zero-gradient, equilibrium ghost at the adjacent node
BC_OPEN_U0 = 2             # same, ghost velocity set to zero
BC_SYMMETRY = 3            # mirror plane half a cell outside the boundary nodes

STORE_F64 = 0
STORE_F32 = 1
STORE_F16_DEV = 2          # 16-bit deviations from the reference populations
STORE_BF16_DEV = 3

ELEMENTS = ("H", "O", "N")
ATOMIC_MASS = {"H": 1.0, "O": 16.0, "N": 14.0}   # integer masses: exact sums


@dataclasses.dataclass
class Mechanism:
    names: List[str]
    molar_mass: np.ndarray      # [M] g/mol
    elements: np.ndarray        # [M, n_el] atoms per molecule (tests only)
    nasa7: np.ndarray           # [M, 7] single-range NASA-7 coefficients
    t_lo: float
    t_hi: float
    nu_reac: np.ndarray         # [R, M] int32
    nu_prod: np.ndarray         # [R, M] int32
    arrhenius: np.ndarray       # [R, 3] A (CGS), b, Ta (K)
    reversible: np.ndarray      # [R] uint8

    @property
    def M(self) -> int:
        return len(self.names)

    @property
    def R(self) -> int:
        return int(self.nu_reac.shape[0])


@dataclasses.dataclass
class Problem:
    name: str
    nx: int
    ny: int
    nz: int
    bc: Tuple[int, int, int, int, int, int]   # -x,+x,-y,+y,-z,+z
    mech: Mechanism
    diff: np.ndarray            # [M, M] binary diffusivities, lattice units
    omega: float
    omega1: float
    kappa: float
    dt_phys: float
    rho_ref: float
    p0: float
    rho: np.ndarray             # [N]
    u: np.ndarray               # [3, N]
    T: np.ndarray               # [N]
    Y: np.ndarray               # [M, N]
    steps: int = 0
    storage: int = STORE_F64
    # quiescent reference state of the 16-bit deviation formats: [rho, T, Y_0..Y_M-1]
    ref_state: Optional[np.ndarray] = None
    # lengths along x of independent lattices side by side (a batch); None: one lattice
    segments: Optional[Tuple[int, ...]] = None
    # temperature-dependent diffusivities D_ab (T / diff_T_ref)^diff_T_exp (0: constant)
    diff_T_ref: float = 0.0
    diff_T_exp: float = 0.0
    # temperature-dependent viscosity and conductivity: 1/omega - 1/2 and 1/omega1 - 1/2
    # scale as (T / visc_T_ref)^visc_T_exp (0: constant omega, omega1)
    visc_T_ref: float = 0.0
    visc_T_exp: float = 0.0

    @property
    def N(self) -> int:
        return self.nx * self.ny * self.nz

    @property
    def M(self) -> int:
        return self.mech.M


# ----------------------------------------------------------------------------
# thermo data construction (input data, not the method)
# ----------------------------------------------------------------------------
def nasa7_coeffs(cp_poly: Sequence[float], h_f: float, s0: float) -> np.ndarray:
    """NASA-7 row whose cp/R polynomial is cp_poly=(a1..a5) and whose enthalpy and
    entropy at T_REF equal h_f [J/mol] and s0 [J/(mol K)]."""
    a1, a2, a3, a4, a5 = cp_poly
    t = T_REF
    h_poly = a1 * t + a2 * t**2 / 2 + a3 * t**3 / 3 + a4 * t**4 / 4 + a5 * t**5 / 5
    s_poly = a1 * math.log(t) + a2 * t + a3 * t**2 / 2 + a4 * t**3 / 3 + a5 * t**4 / 4
    a6 = h_f / R_U - h_poly
    a7 = s0 / R_U - s_poly
    return np.array([a1, a2, a3, a4, a5, a6, a7], dtype=np.float64)


def mole_to_mass(X: np.ndarray, molar_mass: np.ndarray) -> np.ndarray:
    """Mass fractions from mole fractions along axis 0."""
    w = X * molar_mass.reshape((-1,) + (1,) * (X.ndim - 1))
    return w / w.sum(axis=0, keepdims=True)


def mean_molar_mass(X: np.ndarray, molar_mass: np.ndarray) -> np.ndarray:
    return (X * molar_mass.reshape((-1,) + (1,) * (X.ndim - 1))).sum(axis=0)


def lattice_scales(zeta_ref: float, T_ref: float, m_ref: float, P_ref: float):
    """kappa and rho_ref such that a gas of molar mass m_ref [g/mol] at T_ref, P_ref
    has lattice R*T = zeta_ref and lattice density 1."""
    kappa = zeta_ref * (m_ref * 1e-3) / (R_U * T_ref)
    rho_si = P_ref * (m_ref * 1e-3) / (R_U * T_ref)         # kg/m^3
    rho_ref = rho_si * 1e-3                                  # g/cm^3
    return kappa, rho_ref


def lattice_density(P: np.ndarray, T: np.ndarray, m: np.ndarray, rho_ref: float) -> np.ndarray:
    """Lattice density of an ideal gas at pressure P [Pa], temperature T and molar
    mass m [g/mol] (input set-up: uniform-pressure initial fields)."""
    rho_si = P * (m * 1e-3) / (R_U * T)
    return rho_si * 1e-3 / rho_ref


def omega1_from_prandtl(omega: float, prandtl: float) -> float:
    """Relaxation rate of the energy flux for a given Prandtl number: the paper's
    viscosity and conductivity relations give nu/alpha = (1/w - 1/2)/(1/w1 - 1/2)."""
    return 1.0 / (0.5 + (1.0 / omega - 0.5) / prandtl)


def symmetric_uniform(rng: np.random.Generator, M: int, lo: float, hi: float) -> np.ndarray:
    D = rng.uniform(lo, hi, size=(M, M))
    D = 0.5 * (D + D.T)
    np.fill_diagonal(D, 0.0)
    return D


def _mech_arrays(M, reactions):
    R = len(reactions)
    nu_r = np.zeros((R, M), np.int32)
    nu_p = np.zeros((R, M), np.int32)
    arr = np.zeros((R, 3))
    rev = np.zeros(R, np.uint8)
    for k, (reac, prod, A, b, Ta, reversible) in enumerate(reactions):
        for a in reac:
            nu_r[k, a] += 1
        for a in prod:
            nu_p[k, a] += 1
        arr[k] = (A, b, Ta)
        rev[k] = 1 if reversible else 0
    return nu_r, nu_p, arr, rev


# ----------------------------------------------------------------------------
# configuration 1: A + B -> C on a 32x4x4 periodic lattice
# ----------------------------------------------------------------------------
def abc_mechanism(R_count: int = 1, A: float = 1e6, b: float = 0.0, Ta: float = 8000.0,
                  h_f=(0.0, 0.0, -50e3), s0=(200.0, 200.0, 200.0),
                  cp=(3.5, 3.5, 3.5), reversible: bool = False) -> Mechanism:
    """Three ideal-gas species A (2 g/mol), B (32 g/mol), C = AB (34 g/mol) with one
    irreversible reaction A + B -> C (or no reaction when R_count == 0)."""
    names = ["A", "B", "C"]
    mm = np.array([2.0, 32.0, 34.0])
    elements = np.array([[1, 0], [0, 1], [1, 1]], np.int32)   # element "a", element "b"
    nasa = np.stack([nasa7_coeffs((cp[a], 0, 0, 0, 0), h_f[a], s0[a]) for a in range(3)])
    reactions = [((0, 1), (2,), A, b, Ta, reversible)] if R_count else []
    nu_r, nu_p, arr, rev = _mech_arrays(3, reactions)
    if not R_count:
        nu_r = np.zeros((0, 3), np.int32)
        nu_p = np.zeros((0, 3), np.int32)
        arr = np.zeros((0, 3))
        rev = np.zeros(0, np.uint8)
    return Mechanism(names, mm, elements, nasa, 200.0, 4000.0, nu_r, nu_p, arr, rev)


def config1(seed: int = 1, nx: int = 32, ny: int = 4, nz: int = 4, steps: int = 200,
            zeta_ref: float = 0.05, omega: float = 1.6, prandtl: float = 0.7,
            dt_phys: float = 0.41, reacting: bool = True) -> Problem:
    """Plain method, FP64, D3Q27 32x4x4 periodic, M=3, A+B->C (A=1e6 CGS, b=0,
    Ta=8000 K), molar masses 2/32/34, D_ab ~ U[0.02, 0.08] lattice units, rest at
    1000 K, mole fractions 0.3/0.3/0.4 with a seeded sinusoid of amplitude 0.05
    along x (A up, C down), uniform pressure 1 atm."""
    rng = np.random.default_rng(seed)
    mech = abc_mechanism(R_count=1 if reacting else 0)
    M = 3
    D = symmetric_uniform(rng, M, 0.02, 0.08)
    phase = rng.uniform(0, 2 * math.pi)
    T0, P0 = 1000.0, P_ATM
    X_mean = np.array([0.3, 0.3, 0.4])
    m_mean = float(mean_molar_mass(X_mean, mech.molar_mass))
    kappa, rho_ref = lattice_scales(zeta_ref, T0, m_mean, P0)
    N = nx * ny * nz
    x = np.arange(N) % nx
    s = 0.05 * np.sin(2 * math.pi * x / nx + phase)
    X = np.stack([0.3 + s, np.full(N, 0.3), 0.4 - s])
    Y = mole_to_mass(X, mech.molar_mass)
    m = mean_molar_mass(X, mech.molar_mass)
    T = np.full(N, T0)
    rho = lattice_density(np.full(N, P0), T, m, rho_ref)
    u = np.zeros((3, N))
    return Problem("config1_abc_32x4x4", nx, ny, nz, (BC_PERIODIC,) * 6, mech, D, omega,
                   omega1_from_prandtl(omega, prandtl), kappa, dt_phys, rho_ref, P0,
                   rho, u, T, Y, steps=steps, storage=STORE_F64)


# ----------------------------------------------------------------------------
# synthetic 9-species hydrogen/air-like mechanism (configurations 2-5)
# ----------------------------------------------------------------------------
H2AIR_SPECIES = [
    # name, H, O, N   (the inert N2-like species is last: it is the slaved one)
    ("H2", 2, 0, 0), ("O2", 0, 2, 0), ("H", 1, 0, 0), ("O", 0, 1, 0),
    ("OH", 1, 1, 0), ("H2O", 2, 1, 0), ("HO2", 1, 2, 0), ("H2O2", 2, 2, 0),
    ("N2", 0, 0, 2),
]
_RADICALS = ("H", "O", "OH", "HO2")
_PRODUCTS = ("H2O", "H2O2")


def _candidate_reactions(comp: np.ndarray, n_reactive: int):
    """All element-balanced A+B<=>C+D and A+B<=>C among the reactive species."""
    cands = []
    pairs = [(a, b) for a in range(n_reactive) for b in range(a, n_reactive)]
    for (a, b) in pairs:
        lhs = comp[a] + comp[b]
        for c in range(n_reactive):
            if c not in (a, b) and np.array_equal(comp[c], lhs):
                cands.append(((a, b), (c,)))
        for (c, d) in pairs:
            if (c, d) <= (a, b) or {c, d} & {a, b}:
                continue
            if np.array_equal(comp[c] + comp[d], lhs):
                cands.append(((a, b), (c, d)))
    return cands


def _connected(reacs, n_reactive, src, dst):
    adj = {s: set() for s in range(n_reactive)}
    for lhs, rhs in reacs:
        for a in lhs:
            for c in rhs:
                adj[a].add(c)
                adj[c].add(a)
    seen, stack = {src}, [src]
    while stack:
        s = stack.pop()
        for t in adj[s]:
            if t not in seen:
                seen.add(t)
                stack.append(t)
    return dst in seen


# Seed of the synthetic mechanism used by the flame workloads, screened on the oracle:
# the homogeneous reactor at 1500 K ignites (above 2000 K within 3000 steps of 1e-9 s)
# while the 300 K premixture stays inert over 20000 steps, and with 3e-10 s of chemistry
# per step the quasi-1D flame propagates into the premixture at about 0.006 cells per
# step (longer chemistry steps overshoot the oxygen depletion at the front: the source
# is explicit).
FLAME_SEED = 156


def h2air_mechanism(seed: int = FLAME_SEED, n_reactions: int = 19) -> Mechanism:
    """Synthetic 9-species / 19-reaction reversible mechanism over the species set of
    the paper's hydrogen/air mechanism.  Reactions are sampled (seeded) from all
    element-balanced A+B<=>C+D and A+B<=>C templates over the 8 reactive species,
    with every species present and fuel connected to product; log10 A ~ U[8,14],
    b ~ U[-1,1], Ta ~ U[0,2e4] K.  NASA-7 rows are seeded: cp/R in [2.5, 8] on
    [250, 3500] K, h_f = 0 for H2/O2/N2, U[200,260] kJ/mol for the radical atoms,
    U[30,60] kJ/mol for the polyatomic radicals and U[-250,-100] kJ/mol for the two
    stable products, s0 in [100,240] J/(mol K) growing with the atom count."""
    rng = np.random.default_rng(seed)
    names = [s[0] for s in H2AIR_SPECIES]
    comp = np.array([s[1:] for s in H2AIR_SPECIES], np.int32)
    mm = comp @ np.array([ATOMIC_MASS[e] for e in ELEMENTS])
    M = len(names)
    nasa = np.zeros((M, 7))
    for a, nm in enumerate(names):
        atoms = int(comp[a].sum())
        while True:
            if atoms == 1:
                cp = (2.5, 0.0, 0.0, 0.0, 0.0)
            elif atoms == 2:
                cp = (rng.uniform(3.2, 3.6), rng.uniform(0, 6e-4), rng.uniform(-1.5e-7, 0),
                      rng.uniform(0, 1.5e-11), 0.0)
            else:
                cp = (rng.uniform(3.8, 4.5), rng.uniform(0, 1.2e-3), rng.uniform(-3e-7, 0),
                      rng.uniform(0, 3e-11), 0.0)
            tt = np.linspace(250, 3500, 200)
            cpv = cp[0] + cp[1] * tt + cp[2] * tt**2 + cp[3] * tt**3 + cp[4] * tt**4
            if cpv.min() >= 2.5 and cpv.max() <= 8.0:
                break
        if nm in ("H2", "O2", "N2"):
            h_f = 0.0
        elif nm in _RADICALS:
            # atoms are the most endothermic radicals
            h_f = rng.uniform(200e3, 260e3) if atoms == 1 else rng.uniform(30e3, 60e3)
        else:
            h_f = rng.uniform(-250e3, -100e3)
        # standard entropy grows with the number of atoms (bounded to [100, 240])
        s0 = {1: rng.uniform(110.0, 165.0), 2: rng.uniform(130.0, 210.0)}.get(atoms, rng.uniform(185.0, 235.0))
        nasa[a] = nasa7_coeffs(cp, h_f, s0)
    n_reactive = M - 1
    cands = _candidate_reactions(comp, n_reactive)
    fuel, prod = names.index("H2"), names.index("H2O")
    while True:
        pick = rng.choice(len(cands), size=n_reactions, replace=False)
        reacs = [cands[k] for k in sorted(pick)]
        present = set(a for lhs, rhs in reacs for a in lhs + rhs)
        if len(present) == n_reactive and _connected(reacs, n_reactive, fuel, prod):
            break
    h_form = np.array([nasa[a, 5] + nasa[a, 0] * T_REF for a in range(M)])  # h_f / R_U at T_REF
    reactions = []
    for lhs, rhs in reacs:
        # each reaction is written in its exothermic direction, so that the sampled
        # Arrhenius law is the fast direction and the reverse rate k_f/K_c stays bounded
        if sum(h_form[a] for a in rhs) > sum(h_form[a] for a in lhs):
            lhs, rhs = rhs, lhs
        A = 10.0 ** rng.uniform(8, 14)
        b = rng.uniform(-1, 1)
        Ta = rng.uniform(0, 2e4)
        reactions.append((lhs, rhs, A, b, Ta, True))
    nu_r, nu_p, arr, rev = _mech_arrays(M, reactions)
    return Mechanism(names, mm.astype(np.float64), comp, nasa, 250.0, 3500.0, nu_r, nu_p, arr, rev)


def premixed_h2air_X(mech: Mechanism, phi: float, floor: float = 1e-12) -> np.ndarray:
    """Mole fractions of a hydrogen/air premixture at equivalence ratio phi
    (stoichiometric X_F/X_O = 2, X_N/X_O = 3.76), absent species at ``floor``."""
    X = np.full(mech.M, floor)
    iH2, iO2, iN2 = mech.names.index("H2"), mech.names.index("O2"), mech.names.index("N2")
    xo = 1.0
    X[iO2] = xo
    X[iH2] = 2.0 * phi * xo
    X[iN2] = 3.76 * xo
    return X / X.sum()


def tanh_profile(dist: np.ndarray, width: float) -> np.ndarray:
    """0 inside (dist < 0), 1 outside, smooth over ``width`` cells."""
    return 0.5 * (1.0 + np.tanh(dist / width))


def _default_transport(M: int, rng: np.random.Generator, lo: float, hi: float) -> np.ndarray:
    return symmetric_uniform(rng, M, lo, hi)


def flame1d(nx: int = 4096, seed: int = FLAME_SEED, phi: float = 1.0, T_u: float = 300.0,
            T_hot: float = 2000.0, hot_cells: int = 64, zeta_ref: float = 0.003,
            omega: float = 1.0, prandtl: float = 0.7, dt_phys: float = 3e-10,
            diff_range=(0.02, 0.08), steps: int = 20000, edge: float = 8.0,
            storage: int = STORE_F64, mech: Optional[Mechanism] = None) -> Problem:
    """Quasi-1D premixed flame: nx x 1 x 1, periodic y/z, zero-velocity open end at
    -x (unburnt mixture at rest), open end at +x, hot slab of ``hot_cells`` cells at
    the +x end at T_hot with the unburnt composition, uniform pressure 1 atm.

    The slab has a tanh edge of ``edge`` cells.  With a sharp edge (2 cells) the
    ignition overshoots and the oxygen at the forming front goes negative for a few
    thousand steps, where the run is sensitive to rounding; with 8 cells every mass
    fraction stays positive and the front forms smoothly."""
    rng = np.random.default_rng(seed + 1000)
    mech = mech or h2air_mechanism(seed)
    M = mech.M
    X_u = premixed_h2air_X(mech, phi)
    m_u = float(mean_molar_mass(X_u, mech.molar_mass))
    kappa, rho_ref = lattice_scales(zeta_ref, T_u, m_u, P_ATM)
    x = np.arange(nx, dtype=np.float64)
    hot = tanh_profile(x - (nx - hot_cells - 0.5), edge)
    T = T_u + (T_hot - T_u) * hot
    X = np.repeat(X_u[:, None], nx, axis=1)
    Y = mole_to_mass(X, mech.molar_mass)
    m = mean_molar_mass(X, mech.molar_mass)
    rho = lattice_density(np.full(nx, P_ATM), T, m, rho_ref)
    u = np.zeros((3, nx))
    D = _default_transport(M, rng, *diff_range)
    Y_u = mole_to_mass(X_u, mech.molar_mass)
    ref = np.concatenate([[lattice_density(P_ATM, T_u, m_u, rho_ref), T_u], Y_u])
    return Problem(f"flame1d_{nx}", nx, 1, 1, (BC_OPEN_U0, BC_OPEN, 0, 0, 0, 0), mech, D, omega,
                   omega1_from_prandtl(omega, prandtl), kappa, dt_phys, rho_ref, P_ATM,
                   rho, u, T, Y, steps=steps, storage=storage, ref_state=ref)


def adjoint_flame(nx: int = 2048, storage: int = STORE_F64) -> Problem:
    """The flame of the discrete-adjoint workload: the quasi-1D premixed flame of
    ``flame1d`` on 2048 cells (9 species, 19 reactions, 64-cell hot slab), reversed over
    4000 steps with a snapshot every 100 steps."""
    prob = flame1d(nx=nx, storage=storage, steps=4000)
    prob.name = f"adjoint_flame1d_{nx}"
    return prob


def flame_batch(n_flames: int = 256, seed: int = FLAME_SEED, len_range=(512, 8192), phi_range=(0.5, 3.0),
                T_u: float = 300.0, T_hot: float = 2000.0, hot_cells: int = 64, zeta_ref: float = 0.003,
                omega: float = 1.0, prandtl: float = 0.7, dt_phys: float = 3e-10,
                diff_range=(0.02, 0.08), edge: float = 8.0, storage: int = STORE_F32,
                lengths: Optional[Sequence[int]] = None, phis: Optional[Sequence[float]] = None,
                mech: Optional[Mechanism] = None) -> Problem:
    """Batch of independent quasi-1D premixed flames side by side along x, each set up
    as ``flame1d`` (zero-velocity open end at its -x end, open end at +x, hot slab of
    ``hot_cells`` cells with a tanh edge at its +x end).  Lengths are drawn uniformly
    from the integers in ``len_range`` and equivalence ratios uniformly from
    ``phi_range`` (seeded), unless given.  All flames share the mechanism, the
    diffusivities and the lattice units; kappa and rho_ref come from the
    stoichiometric premixture at T_u, so a flame at another equivalence ratio has its
    own unburnt lattice R T (zeta_ref scaled by the mean molar mass ratio)."""
    rng = np.random.default_rng(seed + 3000)
    mech = mech or h2air_mechanism(seed)
    M = mech.M
    if lengths is None:
        lengths = rng.integers(len_range[0], len_range[1] + 1, size=n_flames)
    if phis is None:
        phis = rng.uniform(phi_range[0], phi_range[1], size=len(lengths))
    lengths = [int(v) for v in lengths]
    if len(phis) != len(lengths) or min(lengths) < 1:
        raise ValueError("one equivalence ratio per flame and lengths >= 1 are needed")
    m_st = float(mean_molar_mass(premixed_h2air_X(mech, 1.0), mech.molar_mass))
    kappa, rho_ref = lattice_scales(zeta_ref, T_u, m_st, P_ATM)
    rho_l, T_l, Y_l = [], [], []
    for nx, phi in zip(lengths, phis):
        X_u = premixed_h2air_X(mech, float(phi))
        x = np.arange(nx, dtype=np.float64)
        hot = tanh_profile(x - (nx - hot_cells - 0.5), edge)
        T = T_u + (T_hot - T_u) * hot
        X = np.repeat(X_u[:, None], nx, axis=1)
        Y_l.append(mole_to_mass(X, mech.molar_mass))
        m = mean_molar_mass(X, mech.molar_mass)
        rho_l.append(lattice_density(np.full(nx, P_ATM), T, m, rho_ref))
        T_l.append(T)
    N = int(sum(lengths))
    D = _default_transport(M, np.random.default_rng(seed + 1000), *diff_range)
    Y_st = mole_to_mass(premixed_h2air_X(mech, 1.0), mech.molar_mass)
    ref = np.concatenate([[lattice_density(P_ATM, T_u, m_st, rho_ref), T_u], Y_st])
    prob = Problem(f"flame_batch_{len(lengths)}x{N}", N, 1, 1, (BC_OPEN_U0, BC_OPEN, 0, 0, 0, 0), mech, D,
                   omega, omega1_from_prandtl(omega, prandtl), kappa, dt_phys, rho_ref, P_ATM,
                   np.concatenate(rho_l), np.zeros((3, N)), np.concatenate(T_l), np.concatenate(Y_l, axis=1),
                   storage=storage, ref_state=ref, segments=tuple(lengths))
    prob.phis = np.asarray(phis, np.float64)
    return prob


def split_batch(prob: Problem) -> List[Problem]:
    """The lattices of a batch (``Problem.segments``) as separate problems, in order:
    the x ranges of the batch lattice, each with the full cross-section."""
    if prob.segments is None:
        return [prob]
    shp = (prob.nz, prob.ny, prob.nx)

    def cut(a, sl):
        lead = a.shape[:-1]
        return np.ascontiguousarray(a.reshape(lead + shp)[..., sl]).reshape(lead + (-1,))

    out, x0 = [], 0
    for k, nx in enumerate(prob.segments):
        sl = slice(x0, x0 + nx)
        out.append(dataclasses.replace(prob, name=f"{prob.name}[{k}]", nx=nx, rho=cut(prob.rho, sl),
                                       u=cut(prob.u, sl), T=cut(prob.T, sl), Y=cut(prob.Y, sl),
                                       segments=None))
        x0 += nx
    return out


def batch_nodes(prob: Problem, k: int) -> np.ndarray:
    """Node indices (of the whole batch lattice) of segment k, in that segment's own
    node order."""
    x0 = int(sum(prob.segments[:k]))
    nx = prob.segments[k]
    z, y, x = np.meshgrid(np.arange(prob.nz), np.arange(prob.ny), np.arange(x0, x0 + nx), indexing="ij")
    return (x + prob.nx * (y + prob.ny * z)).reshape(-1)


def sphere3d(n: int = 256, seed: int = FLAME_SEED, phi: float = 0.8, T_u: float = 300.0,
             T_ig: float = 1500.0, radius: float = 12.0, zeta_ref: float = 0.003,
             omega: float = 1.0, prandtl: float = 0.7, dt_phys: float = 3e-10,
             diff_range=(0.02, 0.08), edge: float = 8.0, storage: int = STORE_F32,
             shape: Optional[Tuple[int, int, int]] = None,
             mech: Optional[Mechanism] = None) -> Problem:
    """3D expanding spherical flame: n^3 lattice, all faces open, quiescent premixture
    at T_u and equivalence ratio phi, ignition sphere at T_ig of the given radius
    centred with a seeded sub-cell offset, tanh edge of ``edge`` cells.  With a 2-cell
    edge the run goes non-finite within 100 steps (FP64); with 8 cells it stays finite
    and positive over the 500 steps checked."""
    rng = np.random.default_rng(seed + 2000)
    mech = mech or h2air_mechanism(seed)
    nx, ny, nz = shape or (n, n, n)
    M = mech.M
    X_u = premixed_h2air_X(mech, phi)
    m_u = float(mean_molar_mass(X_u, mech.molar_mass))
    kappa, rho_ref = lattice_scales(zeta_ref, T_u, m_u, P_ATM)
    off = rng.uniform(-0.5, 0.5, size=3)
    c = np.array([(nx - 1) / 2, (ny - 1) / 2, (nz - 1) / 2]) + off
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    r = np.sqrt((x - c[0]) ** 2 + (y - c[1]) ** 2 + (z - c[2]) ** 2).reshape(-1)
    cold = tanh_profile(r - radius, edge)
    T = T_ig + (T_u - T_ig) * cold
    N = nx * ny * nz
    m = np.full(N, m_u)
    rho = lattice_density(np.full(N, P_ATM), T, m, rho_ref)
    Y = np.repeat(mole_to_mass(X_u, mech.molar_mass)[:, None], N, axis=1)
    u = np.zeros((3, N))
    D = _default_transport(M, np.random.default_rng(seed + 1000), *diff_range)
    Y_u = mole_to_mass(X_u, mech.molar_mass)
    ref = np.concatenate([[lattice_density(P_ATM, T_u, m_u, rho_ref), T_u], Y_u])
    return Problem(f"sphere3d_{nx}x{ny}x{nz}", nx, ny, nz, (BC_OPEN,) * 6, mech, D, omega,
                   omega1_from_prandtl(omega, prandtl), kappa, dt_phys, rho_ref, P_ATM,
                   rho, u, T, Y, steps=5000, storage=storage, ref_state=ref)


def cylinder3d(n: int = 256, nz: Optional[int] = None, seed: int = FLAME_SEED, phi: float = 0.8,
               T_u: float = 300.0, T_ig: float = 2000.0, radius: float = 32.0, zeta_ref: float = 0.003,
               omega: float = 1.0, prandtl: float = 0.7, dt_phys: float = 3e-10,
               diff_range=(0.02, 0.08), edge: float = 8.0, storage: int = STORE_F32,
               mech: Optional[Mechanism] = None) -> Problem:
    """Expanding circular flame (the geometry of Sec. 5.2) extruded along z: an n x n x nz
    lattice (nz = n by default), open x and y faces, periodic z, quiescent premixture at
    T_u and equivalence ratio phi, and an ignition cylinder along z at T_ig of the given
    radius, its axis at a seeded sub-cell offset from the centre of the x-y plane, with a
    tanh edge of ``edge`` cells.  At T_ig = 2000 K and radius 24 to 48 it ignites (2440 to
    2510 K) and the burnt area grows over the 3000 steps checked; spherical kernels of the
    same parameters go non-finite."""
    rng = np.random.default_rng(seed + 3000)
    mech = mech or h2air_mechanism(seed)
    nz = n if nz is None else nz
    nx, ny = n, n
    M = mech.M
    X_u = premixed_h2air_X(mech, phi)
    m_u = float(mean_molar_mass(X_u, mech.molar_mass))
    kappa, rho_ref = lattice_scales(zeta_ref, T_u, m_u, P_ATM)
    off = rng.uniform(-0.5, 0.5, size=2)
    c = np.array([(nx - 1) / 2, (ny - 1) / 2]) + off
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    r = np.sqrt((x - c[0]) ** 2 + (y - c[1]) ** 2).reshape(-1)
    cold = tanh_profile(r - radius, edge)
    T = T_ig + (T_u - T_ig) * cold
    N = nx * ny * nz
    rho = lattice_density(np.full(N, P_ATM), T, np.full(N, m_u), rho_ref)
    Y = np.repeat(mole_to_mass(X_u, mech.molar_mass)[:, None], N, axis=1)
    u = np.zeros((3, N))
    D = _default_transport(M, np.random.default_rng(seed + 1000), *diff_range)
    Y_u = mole_to_mass(X_u, mech.molar_mass)
    ref = np.concatenate([[lattice_density(P_ATM, T_u, m_u, rho_ref), T_u], Y_u])
    return Problem(f"cylinder3d_{nx}x{ny}x{nz}", nx, ny, nz, (BC_OPEN, BC_OPEN, BC_OPEN, BC_OPEN, BC_PERIODIC, BC_PERIODIC),
                   mech, D, omega, omega1_from_prandtl(omega, prandtl), kappa, dt_phys, rho_ref, P_ATM,
                   rho, u, T, Y, steps=5000, storage=storage, ref_state=ref)


def perturb_velocity(prob: Problem, amp: float, seed: int) -> Problem:
    """Add a seeded random velocity field (parity cases that exercise every term)."""
    rng = np.random.default_rng(seed)
    prob.u = prob.u + amp * rng.uniform(-1, 1, size=prob.u.shape)
    return prob
