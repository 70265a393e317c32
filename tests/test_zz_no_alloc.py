"""lbm_flame_speeds_static (the entry point that allocates nothing: its work fields and
partial sums live in the library's per-GPU scratch array) against lbm_flame_speeds with
a caller-allocated work buffer, through the C ABI: two calls in a row, the second on a
smaller lattice, and the size limit."""
import ctypes as C

import numpy as np
import pytest

from paper_2101_01702_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lbm_mod():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2101_01702_amd import lbm
    lbm.load()
    return lbm


def _compare(a, b, label):
    for k in ("Sd", "Sa", "w"):
        den = max(float(np.abs(b[k]).max()), 1e-300)
        err = float(np.abs(a[k] - b[k]).max()) / den
        print(f"[{label}] {k}: {err:.3e}", flush=True)
        assert err <= 1e-12, (label, k, err)
    den = np.maximum(np.abs(b["totals"]), 1e-300)
    err = float((np.abs(a["totals"] - b["totals"]) / den).max())
    print(f"[{label}] totals: {err:.3e}", flush=True)
    assert err <= 1e-12, (label, err)


def test_static_scratch_matches_work_buffer_two_calls(lbm_mod):
    # first call: quasi-1D flame of 512 cells with a front (FP64 storage)
    big = W.flame1d(nx=512, hot_cells=64)
    s1 = lbm_mod.Solver(big, storage=W.STORE_F64).init()
    s1.step(300)
    assert s1.status() == 0
    ref1 = s1.flame_speeds(900.0)
    got1 = s1.flame_speeds_static(900.0)
    assert ref1["totals"][0] > 0
    _compare(got1, ref1, "flame1d 512, first call")
    # second call, smaller lattice: a ragged 3D ignition kernel (FP32 storage); the
    # scratch array still holds the first call's fields
    small = W.perturb_velocity(W.sphere3d(shape=(13, 10, 9), radius=3.0, storage=W.STORE_F32), 2e-3, 9)
    s2 = lbm_mod.Solver(small, storage=W.STORE_F32).init()
    s2.step(20)
    assert s2.status() == 0
    centre = (6.0, 4.5, 4.0)
    ref2 = s2.flame_speeds(600.0, centre)
    got2 = s2.flame_speeds_static(600.0, centre)
    _compare(got2, ref2, "sphere 13x10x9, second call")
    # and the first lattice again, after the smaller one
    got1b = s1.flame_speeds_static(900.0)
    _compare(got1b, ref1, "flame1d 512, third call")
    s1.close()
    s2.close()


def test_static_scratch_rejects_large_lattices(lbm_mod):
    prob = W.flame1d(nx=lbm_mod.FLAME_STATIC_MAX_NODES + 1, hot_cells=64)
    s = lbm_mod.Solver(prob, storage=W.STORE_F32).init()
    with pytest.raises(lbm_mod.LbmError) as ei:
        s.flame_speeds_static(900.0)
    assert ei.value.status == -1
    assert "at most" in str(ei.value)
    # a lattice at the limit is accepted
    s.close()
    prob = W.flame1d(nx=lbm_mod.FLAME_STATIC_MAX_NODES, hot_cells=64)
    s = lbm_mod.Solver(prob, storage=W.STORE_F32).init()
    s.step(2)
    ref = s.flame_speeds(900.0)
    got = s.flame_speeds_static(900.0)
    _compare(got, ref, "flame1d at the limit")
    s.close()
