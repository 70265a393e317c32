"""Symmetry faces (the mirror boundary of the quarter-domain flame, Sec. 5.2), HIP
path against the FP64 oracle through the C ABI.  The oracle's own symmetry faces are
pinned against the mirrored full lattice in tests/test_oracle_symmetry.py."""
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


def sym_problem(shape, bc, seed=5):
    """Config-1 chemistry on a small lattice with smooth seeded fields and flow in all
    three directions, so that every population, correction and mirrored component is
    exercised at the faces.  Relaxation omega = 1.3: at config 1's 1.6 any content
    across a cross-section this thin grows until the run breaks down (periodic faces
    too), within about 100 steps.  The mixture self-heats (A + B -> C, about 1000 K to
    1550 K in 500 steps) and runs away near step 650, so the runs stop at 500."""
    nx, ny, nz = shape
    base = W.config1(nx=nx, ny=ny, nz=nz)
    rng = np.random.default_rng(seed)
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    def wave(amp):
        ph = rng.uniform(0, 2 * np.pi, 3)
        return amp * (np.cos(2 * np.pi * x / nx + ph[0]) * np.cos(np.pi * y / ny + ph[1]) +
                      np.sin(np.pi * z / nz + ph[2])).reshape(-1)
    T = 1000.0 + wave(20.0)
    u = np.stack([wave(1e-3), wave(8e-4), wave(6e-4)])
    Y = np.repeat(base.Y.mean(axis=1)[:, None], x.size, axis=1)
    dY = wave(0.005)                     # the heavy species: both stay well above zero
    Y[1] += dY
    Y[2] -= dY
    rho = base.rho.mean() * (1.0 + wave(0.002))
    return dataclasses.replace(base, bc=tuple(bc), rho=rho, u=u, T=T, Y=Y, omega=1.3,
                               omega1=W.omega1_from_prandtl(1.3, 0.7), name=f"sym_{nx}x{ny}x{nz}")


S, O, P, U0 = W.BC_SYMMETRY, W.BC_OPEN, W.BC_PERIODIC, W.BC_OPEN_U0
CASES = [
    ((9, 4, 3), (O, S, P, P, P, P)),            # one symmetry face
    ((8, 7, 3), (S, O, S, O, P, P)),            # quarter domain: symmetry and open edges
    ((6, 5, 4), (S, S, S, U0, O, S)),           # corners of two and three symmetry faces
]


@pytest.mark.parametrize("shape,bc", CASES)
def test_symmetry_faces_fp64(lbm_mod, shape, bc):
    prob = sym_problem(shape, bc)
    s = lbm_mod.Solver(prob, storage=W.STORE_F64).init()
    s.step(100)
    mac = s.macros()
    sim, anom = oracle_run(prob, 100)
    assert s.status() == 0 and anom == 0
    check_fp64(field_errors(mac, sim.macros(), zeta_of(prob)), f"{prob.name} {bc}")
    pop, _ = s.populations(np.arange(prob.N))
    assert max(pop_errors(pop, sim.state()[0])) <= TOL64
    s.close()


@pytest.mark.parametrize("shape,bc", CASES[1:2])
def test_symmetry_faces_fp32(lbm_mod, shape, bc):
    prob = sym_problem(shape, bc)
    s = lbm_mod.Solver(prob, storage=W.STORE_F32).init()
    s.step(500)
    mac = s.macros()
    sim, anom = oracle_run(prob, 500)
    assert s.status() == 0 and anom == 0
    check_fp32(field_errors(mac, sim.macros(), zeta_of(prob)), prob.name)
    s.close()


@pytest.mark.parametrize("axis", [0, 2])
def test_symmetry_face_matches_mirrored_full_lattice_on_gpu(lbm_mod, axis):
    """The half lattice with a symmetry face against the full mirror-symmetric lattice,
    both on the GPU in FP64 (the oracle's own pin of the face, repeated on the HIP path)."""
    import test_oracle_symmetry as TS
    full, half, keep = TS.mirror_problems(axis, L=6)
    out = []
    for prob in (full, half):
        s = lbm_mod.Solver(prob, storage=W.STORE_F64).init()
        s.step(40)
        assert s.status() == 0
        out.append(s.macros())
        s.close()
    fm, hm = out
    err = field_errors(hm, {k: (v[..., keep] if k in ("u", "Y") else v[keep]) for k, v in fm.items()},
                       zeta_of(full))
    check_fp64(err, f"mirror axis {axis}")
