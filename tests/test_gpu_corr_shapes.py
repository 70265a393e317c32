"""The tile shapes of the correction stencil (eqs. X and the energy-flux correction, with
psi of the isotropy correction), which lbm_create times and from which it keeps the
fastest: k_corr after k_psi in three tiles (0-2), or in a flat one (9) on lattices one
node thick in z, and k_corr_march (6),
which forms psi itself from phi while it walks a column of the lattice along z, so
that psi never goes through HBM.  Every shape reads the same values and sums them in
the same order: a run gives the same bits whichever shape it takes.  Covered: chunks
of z planes with wrapped and clamped z neighbours, ragged tiles, symmetry faces,
temperature-dependent relaxation rates (psi's factor 1/omega - 1/2 per node), lattices
one node thick in z or in y, batches of 3D segments, and the seeded random lattices;
the marching shape is also held to the oracle directly."""
import dataclasses

import numpy as np
import pytest

from paper_2101_01702_amd import workloads as W
from gpu_cases import check_fp64, field_errors, oracle_run, pop_errors, zeta_of, TOL64
from test_gpu_random_cases import random_case
from test_gpu_species_counts import problem as species_problem
from test_gpu_symmetry import sym_problem

pytestmark = pytest.mark.gpu

S, O, P, U0 = W.BC_SYMMETRY, W.BC_OPEN, W.BC_PERIODIC, W.BC_OPEN_U0
SPLIT = (0, 1, 2)        # k_psi, then k_corr
MARCH = (6,)             # k_corr_march
FLAT = (9,)              # k_psi, then k_corr on a 32 x 8 x 1 tile (lattices one node thick in z)


@pytest.fixture(scope="module")
def lbm_mod():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2101_01702_amd import lbm
    lbm.load()
    return lbm


def lattice(name):
    if name == "chunks_wrapped_z_rates_of_T":
        # 70 planes: 3 chunks of 32 planes; 35 x 19
        # leaves ragged tiles in x and y
        prob = sym_problem((35, 19, 70), (O, U0, S, O, P, P), seed=7)
        return dataclasses.replace(prob, visc_T_ref=900.0, visc_T_exp=0.5, name="chunks_35x19x70_vt")
    if name == "symmetry_and_clamped_z":
        return dataclasses.replace(sym_problem((20, 11, 37), (S, O, S, U0, S, O), seed=8), name="sym_20x11x37")
    if name == "all_periodic":
        return dataclasses.replace(sym_problem((33, 9, 17), (P, P, P, P, P, P), seed=9), name="per_33x9x17")
    if name == "one_plane":
        return dataclasses.replace(sym_problem((40, 33, 1), (O, S, U0, O, P, P), seed=10), name="plane_40x33x1")
    if name == "one_row_in_y":
        return dataclasses.replace(sym_problem((37, 1, 40), (O, O, P, P, S, U0), seed=11), name="y1_37x1x40")
    if name == "segments_3d":
        base = W.perturb_velocity(W.sphere3d(shape=(22, 4, 35), radius=3.0, storage=W.STORE_F64), 1e-3, 4)
        return dataclasses.replace(base, bc=(O, S, P, P, O, U0), segments=(5, 9, 1, 7), name="segments_22x4x35")
    raise KeyError(name)


LATTICES = ["chunks_wrapped_z_rates_of_T", "symmetry_and_clamped_z", "all_periodic", "one_plane",
            "one_row_in_y", "segments_3d"]


def _run(lbm_mod, prob, storage, tile, steps, monkeypatch):
    monkeypatch.setenv("LBM_CORR_TILE", str(tile))
    print(f"[{prob.name} storage={storage} tile={tile} steps={steps}]", flush=True)
    s = lbm_mod.Solver(prob, storage=storage).init()
    s.step(steps)
    mac = s.macros()
    pops, T = s.populations(np.arange(0, prob.N, 3))
    assert s.status() == 0
    s.close()
    monkeypatch.delenv("LBM_CORR_TILE")
    return mac, pops, T


def _same(a, b, what):
    for k in ("rho", "u", "T", "P", "Y"):
        assert np.array_equal(a[0][k], b[0][k]), (what, k)
    assert np.array_equal(a[1], b[1]) and np.array_equal(a[2], b[2]), (what, "populations")


@pytest.mark.parametrize("name", LATTICES)
def test_marching_shapes_give_the_same_bits_fp64(lbm_mod, name, monkeypatch):
    prob = lattice(name)
    ref = _run(lbm_mod, prob, W.STORE_F64, 0, 20, monkeypatch)
    for tile in SPLIT[1:] + MARCH + (FLAT if prob.nz == 1 else ()):
        _same(_run(lbm_mod, prob, W.STORE_F64, tile, 20, monkeypatch), ref, (name, tile))


@pytest.mark.parametrize("name", ["chunks_wrapped_z_rates_of_T", "segments_3d"])
def test_marching_shapes_give_the_same_bits_fp32(lbm_mod, name, monkeypatch):
    prob = lattice(name)
    ref = _run(lbm_mod, prob, W.STORE_F32, 0, 20, monkeypatch)
    for tile in MARCH:
        _same(_run(lbm_mod, prob, W.STORE_F32, tile, 20, monkeypatch), ref, (name, tile))


def test_marching_shapes_on_random_lattices(lbm_mod, monkeypatch):
    """The seeded random lattices (every boundary type, segments, sizes 1..9) that have
    a cross-section: tiles 0 and 6 give the same bits after 10 steps."""
    n = 0
    for seed in range(40):
        prob = random_case(seed)
        if prob.ny == 1 and prob.nz == 1:
            continue
        ref = _run(lbm_mod, prob, W.STORE_F64, 0, 10, monkeypatch)
        for tile in MARCH + (FLAT if prob.nz == 1 else ()):
            _same(_run(lbm_mod, prob, W.STORE_F64, tile, 10, monkeypatch), ref, (prob.name, tile))
        n += 1
    assert n >= 30


@pytest.mark.parametrize("M", range(2, 11))
def test_marching_shape_every_species_count(lbm_mod, M, monkeypatch):
    """Every species count the library builds (its own instance of the marching kernel,
    with M mass-fraction planes in LDS), on the ragged 7x5x4 lattice with open,
    zero-velocity and symmetry faces: the same bits as k_psi + k_corr, FP64 and FP32."""
    prob = species_problem(M)
    for storage in (W.STORE_F64, W.STORE_F32):
        ref = _run(lbm_mod, prob, storage, 0, 20, monkeypatch)
        for tile in MARCH:
            _same(_run(lbm_mod, prob, storage, tile, 20, monkeypatch), ref, (prob.name, storage, tile))


@pytest.mark.parametrize("tile", MARCH)
def test_marching_shape_against_oracle_fp64(lbm_mod, tile, monkeypatch):
    """Symmetry, open and zero-velocity faces on a lattice of two z chunks: the marching
    shape against the oracle to 1e-12 (fields and populations) after 30 steps."""
    prob = lattice("symmetry_and_clamped_z")
    monkeypatch.setenv("LBM_CORR_TILE", str(tile))
    print(f"[{prob.name} tile={tile} against the oracle]", flush=True)
    s = lbm_mod.Solver(prob, storage=W.STORE_F64).init()
    s.step(30)
    mac = s.macros()
    pops, _ = s.populations(np.arange(prob.N))
    assert s.status() == 0
    s.close()
    sim, anom = oracle_run(prob, 30)
    assert anom == 0
    check_fp64(field_errors(mac, sim.macros(), zeta_of(prob)), f"{prob.name} tile {tile}")
    assert max(pop_errors(pops, sim.state()[0])) <= TOL64
