"""Seeded random lattices against the oracle: sizes 1..9 per axis, every boundary type
on every face (periodic faces in pairs), batches of segments along an open x axis, and
smooth seeded fields in all three directions (config-1 chemistry at omega = 1.3, as in
the symmetry cases).  FP64 storage to 1e-12 after 30 steps (fields and populations),
FP32 storage to 1e-5; each segment of a batch against the oracle run on that lattice
alone."""
import dataclasses

import numpy as np
import pytest

from paper_2101_01702_amd import workloads as W
from gpu_cases import check_fp32, check_fp64, field_errors, oracle_run, pop_errors, zeta_of
from test_gpu_symmetry import sym_problem

pytestmark = pytest.mark.gpu

TOL64 = 1e-12
BCS = (W.BC_OPEN, W.BC_OPEN_U0, W.BC_SYMMETRY)


def random_case(seed):
    rng = np.random.default_rng(1000 + seed)
    shape = [int(v) for v in rng.integers(1, 10, size=3)]
    bc = []
    for a in range(3):
        if rng.random() < 0.3:
            bc += [W.BC_PERIODIC, W.BC_PERIODIC]
        else:
            bc += [int(rng.choice(BCS)), int(rng.choice(BCS))]
    segments = None
    if bc[0] != W.BC_PERIODIC and rng.random() < 0.5:
        k = int(rng.integers(2, 4))
        lens = rng.integers(1, 6, size=k)
        shape[0] = int(lens.sum())
        segments = tuple(int(v) for v in lens)
    prob = sym_problem(tuple(shape), tuple(bc), seed=seed)
    return dataclasses.replace(prob, segments=segments, name=f"random{seed}_{shape}_{bc}_{segments}")


@pytest.fixture(scope="module")
def lbm_mod():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2101_01702_amd import lbm
    lbm.load()
    return lbm


@pytest.mark.parametrize("seed", range(40))
def test_random_lattice_fp64(lbm_mod, seed):
    _check(lbm_mod, random_case(seed), W.STORE_F64, TOL64, pops=True)


@pytest.mark.parametrize("seed", range(40, 52))
def test_random_lattice_fp32(lbm_mod, seed):
    _check(lbm_mod, random_case(seed), W.STORE_F32, 1e-5, pops=False)


def _check(lbm_mod, prob, storage, tol, pops):
    print(f"[{prob.name} storage={storage}]", flush=True)
    s = lbm_mod.Solver(prob, storage=storage).init()
    s.step(30)
    mac = s.macros()
    allpop, _ = s.populations(np.arange(prob.N))
    assert s.status() == 0
    worst = 0.0
    for k, part in enumerate(W.split_batch(prob)):
        idx = W.batch_nodes(prob, k) if prob.segments else np.arange(prob.N)
        sim, anom = oracle_run(part, 30)
        assert anom == 0
        err = field_errors({key: (v[..., idx] if np.ndim(v) > 1 else v[idx]) for key, v in mac.items()},
                           sim.macros(), zeta_of(part))
        worst = max(worst, max(err.values()))
        (check_fp64 if storage == W.STORE_F64 else check_fp32)(err, f"{prob.name} part {k}")
        if pops:
            assert max(pop_errors(allpop[..., idx], sim.state()[0])) <= tol, k
    s.close()
    print(f"  worst field error {worst:.2e}", flush=True)
