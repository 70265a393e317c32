"""lbm_step_graph: steps replayed from a recorded HIP graph give the bits of lbm_step.
Every replay is checked against the eager run, with eager work (macros, populations)
and synchronisations between the replays; an odd step count alternates between the
recordings of both ping-pong parities."""
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


def _same(a, b):
    for k in ("rho", "u", "T", "P", "Y"):
        assert np.array_equal(a[k], b[k]), k


@pytest.mark.parametrize("n", [10, 3])
def test_graph_replays_match_eager_steps(lbm_mod, n):
    prob = W.flame_batch(lengths=[300, 17, 129, 64], phis=[1.0, 0.7, 2.4, 1.6], hot_cells=24,
                         storage=W.STORE_F32)
    eager = lbm_mod.Solver(prob).init()
    graph = lbm_mod.Solver(prob).init()
    nodes = np.arange(0, prob.N, 7)
    for rep in range(4):
        eager.step(n)
        graph.step_graph(n)
        _same(graph.macros(), eager.macros())
        pg, Tg = graph.populations(nodes)
        pe, Te = eager.populations(nodes)
        assert np.array_equal(pg, pe) and np.array_equal(Tg, Te), rep
    assert graph.status() == 0 and eager.status() == 0
    # eager steps in between keep the parity bookkeeping
    eager.step(1)
    graph.step(1)
    eager.step(n)
    graph.step_graph(n)
    _same(graph.macros(), eager.macros())
    graph.close()
    eager.close()


def test_graph_on_3d_lattice_with_all_kernels(lbm_mod):
    """Open, symmetry and periodic faces: the ghost, mirror-correction, psi and
    correction kernels all take part in the recording."""
    prob = W.perturb_velocity(W.sphere3d(shape=(13, 10, 9), radius=3.0, storage=W.STORE_F64), 1e-3, 5)
    prob.bc = (W.BC_SYMMETRY, W.BC_OPEN, 0, 0, W.BC_OPEN_U0, W.BC_SYMMETRY)
    eager = lbm_mod.Solver(prob, storage=W.STORE_F64).init()
    graph = lbm_mod.Solver(prob, storage=W.STORE_F64).init()
    for rep in range(3):
        eager.step(4)
        graph.step_graph(4)
        _same(graph.macros(), eager.macros())
    graph.close()
    eager.close()


def test_graph_step_counts(lbm_mod):
    """Zero steps change nothing; a negative count is an argument error."""
    prob = W.flame_batch(lengths=[40, 9], phis=[1.0, 2.0], hot_cells=8, storage=W.STORE_F64)
    s = lbm_mod.Solver(prob, storage=W.STORE_F64).init()
    before = s.macros()
    s.step_graph(0)
    _same(s.macros(), before)
    with pytest.raises(lbm_mod.LbmError):
        s.step_graph(-1)
    s.close()


@pytest.mark.parametrize("kind,tiles", [("3d", (0, 1, 2, 6)), ("thin", (3, 4, 5))])
def test_correction_tile_shapes_give_the_same_bits(lbm_mod, kind, tiles, monkeypatch):
    """lbm_create times the tile shapes of the correction stencil and keeps the fastest;
    every shape reads the same values in the same order, so the state after a run is
    the same bit for bit whichever is chosen."""
    if kind == "3d":
        prob = W.perturb_velocity(W.sphere3d(shape=(37, 10, 9), radius=3.0, storage=W.STORE_F64), 1e-3, 3)
    else:
        prob = W.flame_batch(lengths=[300, 45, 700], phis=[1.0, 2.0, 0.6], hot_cells=24, storage=W.STORE_F64)
    out = []
    for k in tiles:
        monkeypatch.setenv("LBM_CORR_TILE", str(k))
        s = lbm_mod.Solver(prob, storage=W.STORE_F64).init()
        s.step(30)
        out.append(s.macros())
        assert s.status() == 0
        s.close()
    monkeypatch.delenv("LBM_CORR_TILE")
    s = lbm_mod.Solver(prob, storage=W.STORE_F64).init()    # the timed choice
    s.step(30)
    out.append(s.macros())
    s.close()
    for m in out[1:]:
        _same(m, out[0])
