"""Helpers shared by the GPU parity tests: oracle runs and field comparisons."""
import math

import numpy as np

from oracle import oracle as orc
from paper_2101_01702_amd import workloads as W


def field_errors(gpu, ref, zeta_ref):
    """Normwise relative errors per field: ||a - b||_inf / ||b||_inf, with the floor
    max(||u||_inf, sqrt(zeta_ref)) for velocity components (a velocity is a difference
    of populations of unit lattice speed, so its rounding is absolute; errors are
    measured against the lattice sound-speed scale) and max(||Y_a||, 1e-12) for mass
    fractions."""
    err = {}
    for k in ("rho", "T", "P"):
        err[k] = float(np.abs(gpu[k] - ref[k]).max() / np.abs(ref[k]).max())
    ufloor = math.sqrt(zeta_ref)
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
