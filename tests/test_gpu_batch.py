"""Batches of independent lattices side by side along x (lbm_desc.n_segments): ragged
quasi-1D flames, each set up as the flame of Sec. 5.1, advanced in one launch per
kernel.  A batch computes what its lattices compute one by one: every segment is
compared with the FP64 oracle run on that lattice alone, and with the same lattice
run alone on the GPU (bitwise: no arithmetic of a node depends on the layout)."""
import dataclasses

import numpy as np
import pytest

from paper_2101_01702_amd import workloads as W
from gpu_cases import check_fp32, check_fp64, field_errors, oracle_run, pop_errors, zeta_of

pytestmark = pytest.mark.gpu

TOL64 = 1e-12
TOL32 = 1e-5
# mass fractions of igniting flames after 1000 FP32 steps: the bar of the single
# quasi-1D flame (storage rounding amplified by the flame's pinned linear response)


@pytest.fixture(scope="module")
def lbm_mod():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2101_01702_amd import lbm
    lbm.load()
    return lbm


def _run(lbm_mod, prob, steps, storage):
    s = lbm_mod.Solver(prob, storage=storage).init()
    s.step(steps)
    mac = s.macros()
    bits = s.status()
    return s, mac, bits


def _seg(mac, idx):
    return {k: (v[..., idx] if np.ndim(v) > 1 else v[idx]) for k, v in mac.items()}


def test_ragged_flame_batch_fp64(lbm_mod):
    """Six flames of 1 to 160 cells (a one-node flame: both ghost ends on one node)."""
    prob = W.flame_batch(lengths=[96, 1, 2, 33, 160, 65], phis=[0.6, 1.0, 2.5, 3.0, 0.5, 1.4], hot_cells=16,
                         storage=W.STORE_F64)
    s, mac, bits = _run(lbm_mod, prob, 200, W.STORE_F64)
    assert bits == 0
    pops, _ = s.populations(np.arange(prob.N))
    for k, part in enumerate(W.split_batch(prob)):
        idx = W.batch_nodes(prob, k)
        sim, anom = oracle_run(part, 200)
        assert anom == 0
        check_fp64(field_errors(_seg(mac, idx), sim.macros(), zeta_of(part)), f"{part.name} nx={part.nx}")
        assert max(pop_errors(pops[..., idx], sim.state()[0])) <= TOL64, k


def test_flame_batch_fp32_1000_steps(lbm_mod):
    prob = W.flame_batch(lengths=[200, 37, 128], phis=[1.0, 2.2, 0.7], hot_cells=32, storage=W.STORE_F32)
    s, mac, bits = _run(lbm_mod, prob, 1000, W.STORE_F32)
    assert bits == 0
    errs = []
    for k, part in enumerate(W.split_batch(prob)):
        sim, anom = oracle_run(part, 1000)
        assert anom == 0
        errs.append(field_errors(_seg(mac, W.batch_nodes(prob, k)), sim.macros(), zeta_of(part)))
    worst = {key: max(e[key] for e in errs) for key in errs[0]}
    check_fp32(worst, "flame batch of 3, fp32 1000")


def test_batch_of_3d_lattices_with_symmetry_fp64(lbm_mod):
    """Segments with a cross-section (periodic y, open and zero-velocity z faces) and a
    symmetry face at each segment's +x end: x ghost cells of every segment, and the
    edges and corners where they meet the z ghost layer."""
    base = W.perturb_velocity(W.sphere3d(shape=(22, 4, 3), radius=3.0, storage=W.STORE_F64), 1e-3, 4)
    prob = dataclasses.replace(base, bc=(W.BC_OPEN, W.BC_SYMMETRY, 0, 0, W.BC_OPEN, W.BC_OPEN_U0),
                               segments=(5, 9, 1, 7))
    s, mac, bits = _run(lbm_mod, prob, 60, W.STORE_F64)
    assert bits == 0
    pops, _ = s.populations(np.arange(prob.N))
    for k, part in enumerate(W.split_batch(prob)):
        idx = W.batch_nodes(prob, k)
        sim, anom = oracle_run(part, 60)
        assert anom == 0
        check_fp64(field_errors(_seg(mac, idx), sim.macros(), zeta_of(part)), part.name)
        assert max(pop_errors(pops[..., idx], sim.state()[0])) <= TOL64, k


def test_full_batch_equals_separate_lattices(lbm_mod):
    """The batch of 256 flames of 512..8192 cells (FP32 storage) against the same 256
    lattices run one by one on the GPU: identical bits after 20 steps; and its two
    shortest flames against the oracle."""
    prob = W.flame_batch()
    assert len(prob.segments) == 256 and min(prob.segments) >= 512 and max(prob.segments) <= 8192
    s, mac, bits = _run(lbm_mod, prob, 20, W.STORE_F32)
    assert bits == 0
    s.close()
    parts = W.split_batch(prob)
    for k, part in enumerate(parts):
        sk, mk, bk = _run(lbm_mod, part, 20, W.STORE_F32)
        assert bk == 0
        idx = W.batch_nodes(prob, k)
        for key in ("rho", "T", "u", "Y"):
            assert np.array_equal(mk[key], mac[key][..., idx]), (k, key)
        sk.close()
    for k in np.argsort(prob.segments)[:2]:
        sim, anom = oracle_run(parts[k], 20)
        assert anom == 0
        check_fp32(field_errors(_seg(mac, W.batch_nodes(prob, int(k))), sim.macros(), zeta_of(parts[k])),
                   f"{parts[k].name} nx={parts[k].nx}")
