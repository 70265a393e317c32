"""Symmetry faces of the oracle (the mirror boundary of the quarter-domain flame,
Sec. 5.2), pinned against its own full-domain dynamics.

A lattice whose fields are mirror-symmetric about the plane between cells L-1 and L
keeps that symmetry: its half [0, L) with a symmetry face at the mirror plane must
evolve exactly like the half of the full lattice.  The full lattice has no symmetry
face, so it checks the mirror streaming and the mirrored vector components of the
gradient stencils from outside."""
import dataclasses

import numpy as np
import pytest

from oracle import oracle as orc
from paper_2101_01702_amd import workloads as W


def mirror_problems(axis, L, other=(4, 2), seed=3):
    """Full lattice (2L along `axis`, open faces there) with fields mirror-symmetric
    about its middle, the half lattice [0, L) with a symmetry face at +axis, and the
    mask of the full lattice's nodes that the half holds."""
    shape = [0, 0, 0]
    shape[axis] = 2 * L
    rest = [a for a in range(3) if a != axis]
    shape[rest[0]], shape[rest[1]] = other
    base = W.config1(nx=shape[0], ny=shape[1], nz=shape[2])
    nx, ny, nz = shape
    rng = np.random.default_rng(seed)
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    c = [x, y, z][axis].astype(float)
    r = np.minimum(c, 2 * L - 1 - c)                  # distance index from the outer face
    k = 2 * np.pi / (2 * L)
    oth = sum(np.cos(2 * np.pi * [x, y, z][a] / shape[a] + rng.uniform(0, 6)) for a in rest)
    T = (1000.0 + 60.0 * np.cos(k * r + 0.3) + 10.0 * oth).reshape(-1)
    u = np.zeros((3, x.size))
    sgn = np.where(c < L, 1.0, -1.0).reshape(-1)
    u[axis] = 2e-3 * np.sin(k * (r + 0.5)).reshape(-1) * sgn      # odd under the mirror
    for a in rest:
        u[a] = 1e-3 * np.cos(k * r + a).reshape(-1) + 5e-4 * oth.reshape(-1)
    Y = np.repeat(base.Y.mean(axis=1)[:, None], x.size, axis=1)   # config 1's own profile is not mirrored
    dY = 0.03 * np.cos(k * r + 1.0).reshape(-1)
    Y[0] += dY
    Y[2] -= dY
    rho = base.rho.mean() * (1.0 + 0.02 * np.sin(k * r + 0.7).reshape(-1))
    bc = [W.BC_PERIODIC] * 6
    bc[2 * axis], bc[2 * axis + 1] = W.BC_OPEN, W.BC_OPEN
    full = dataclasses.replace(base, bc=tuple(bc), rho=rho, u=u, T=T, Y=Y, name="mirror_full")
    half_shape = list(shape)
    half_shape[axis] = L
    keep = (c < L).reshape(-1)
    bch = list(bc)
    bch[2 * axis + 1] = W.BC_SYMMETRY
    half = dataclasses.replace(base, nx=half_shape[0], ny=half_shape[1], nz=half_shape[2], bc=tuple(bch),
                               rho=rho[keep], u=u[:, keep], T=T[keep], Y=Y[:, keep], name="mirror_half")
    return full, half, keep


def _mirror_pair(axis, L, other=(4, 2), seed=3, steps=40, lib=None):
    full, half, keep = mirror_problems(axis, L, other, seed)
    fs = orc.OracleSim(full, lib=lib).init()
    hs = orc.OracleSim(half, lib=lib).init()
    assert fs.step(steps, 4) == 0 and hs.step(steps, 4) == 0
    return fs.macros(), hs.macros(), keep


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_symmetry_face_reproduces_the_mirrored_full_lattice(axis):
    fm, hm, keep = _mirror_pair(axis, L=6)
    for key in ("rho", "T", "P"):
        a, b = hm[key], fm[key][keep]
        assert np.abs(a - b).max() <= 1e-12 * np.abs(b).max(), key
    # a velocity is a difference of populations of unit lattice speed: its rounding is
    # absolute, at the scale of the lattice sound speed sqrt(zeta) (config 1: 0.05)
    for d in range(3):
        a, b = hm["u"][d], fm["u"][d][keep]
        assert np.abs(a - b).max() <= 1e-12 * max(np.abs(b).max(), np.sqrt(0.05)), ("u", d)
    for s in range(hm["Y"].shape[0]):
        a, b = hm["Y"][s], fm["Y"][s][keep]
        assert np.abs(a - b).max() <= 1e-12 * np.abs(b).max(), ("Y", s)


def test_full_lattice_keeps_its_mirror_symmetry():
    """The mirror case itself: the full lattice stays symmetric, u along the axis odd."""
    fm, _, keep = _mirror_pair(0, L=6)
    nx = 12
    T = fm["T"].reshape(2, 4, nx)
    assert np.abs(T - T[:, :, ::-1]).max() <= 1e-12 * T.max()
    ux = fm["u"][0].reshape(2, 4, nx)
    assert np.abs(ux + ux[:, :, ::-1]).max() <= 1e-12 * np.sqrt(0.05)
    assert np.abs(ux).max() > 1e-5
