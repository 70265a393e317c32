"""Pins of the oracle's reverse sweep (oracle/oracle_ad.cpp: oracle.c compiled on a
recording arithmetic type, reversed over its tape).  Nothing here compares the reverse
sweep with itself: every vector-Jacobian product is checked against FP64 central
differences of the plain oracle (the dot-product test <lam, J v> = <J^T lam, v>), and
the taped forward is checked bitwise against the plain oracle.  A planted mistake in a
derivative rule of the tape is caught by the same checks."""
import os
import shutil

import numpy as np
import pytest

from oracle import oracle as orc
from paper_2101_01702_amd import workloads as W


def _cases():
    flame = W.flame1d(nx=24, hot_cells=8)
    sphere = W.perturb_velocity(W.sphere3d(shape=(5, 4, 3), radius=1.5, storage=W.STORE_F64), 2e-3, 5)
    periodic = W.config1(nx=8, ny=2, nz=2)
    return [("flame1d_24", flame), ("sphere_5x4x3", sphere), ("config1_8x2x2", periodic)]


def _advance(prob, steps):
    """State after a few plain oracle steps (with a non-equilibrium part)."""
    s = orc.OracleSim(prob).init()
    s.step(steps)
    return s.state()


def _fd_step(prob, pop, T, v, h, arrhenius=None):
    """Central difference of one step along the population direction v."""
    s = orc.OracleSim(prob, arrhenius=arrhenius).init()
    s.set_state(pop + h * v, T)
    s.step(1)
    p1 = s.state()[0]
    s.set_state(pop - h * v, T)
    s.step(1)
    return (p1 - s.state()[0]) / (2 * h)


def test_taped_forward_is_the_plain_oracle():
    for name, prob in _cases():
        a = orc.OracleSim(prob).init()
        a.step(4)
        b = orc.OracleAdjoint(prob).init()
        assert b._lib.orc_step(b._h, 4, 1) == 0
        pa, Ta = a.state()
        pb, Tb = b.state()
        assert np.array_equal(pa, pb), name
        assert np.array_equal(Ta, Tb), name


@pytest.mark.parametrize("case", range(3))
def test_step_vjp_matches_central_differences(case):
    name, prob = _cases()[case]
    pop, T = _advance(prob, 3)
    rng = np.random.default_rng(11 + case)
    v = rng.standard_normal(pop.shape) * pop          # relative perturbation of every population
    lam = rng.standard_normal(pop.shape)
    adj = orc.OracleAdjoint(prob).init()
    adj.set_state(pop, T)
    lam_prev, _, anom = adj.step_vjp(lam)
    assert anom == 0
    ad_dot = float((lam_prev * v).sum())
    fd_dot = float((lam * _fd_step(prob, pop, T, v, 1e-5)).sum())
    rel = abs(fd_dot - ad_dot) / abs(ad_dot)
    print(f"[{name}] <lam, J v>: fd {fd_dot:.12e} ad {ad_dot:.12e} rel {rel:.2e}", flush=True)
    assert rel < 1e-7, (name, rel)
    # the step advanced the recorded state exactly as the plain oracle does
    plain = orc.OracleSim(prob).init()
    plain.set_state(pop, T)
    plain.step(1)
    assert np.array_equal(adj.state()[0], plain.state()[0])


@pytest.mark.parametrize("case", [0, 1])
def test_parameter_gradient_matches_central_differences(case):
    name, prob = _cases()[case]
    pop, T = _advance(prob, 3)
    rng = np.random.default_rng(5 + case)
    scale = np.abs(pop).max(axis=(1, 2), keepdims=True)
    lam = rng.standard_normal(pop.shape) / scale
    adj = orc.OracleAdjoint(prob).init()
    adj.set_state(pop, T)
    _, grad, _ = adj.step_vjp(lam)
    A = prob.mech.arrhenius
    worst = 0.0
    # the three reactions that move the step most (others can be frozen at these states)
    for k in np.argsort(-np.abs(grad[:, 0]))[:3]:
        for c, h in ((0, 1e-6), (1, 1e-6), (2, 1e-2)):
            def run(sign):
                arr = A.copy()
                if c == 0:
                    arr[k, 0] *= np.exp(sign * h)
                else:
                    arr[k, c] += sign * h
                s = orc.OracleSim(prob, arrhenius=arr).init()
                s.set_state(pop, T)
                s.step(1)
                return s.state()[0]
            fd = float((lam * (run(1) - run(-1))).sum() / (2 * h))
            den = max(abs(fd), abs(grad[k, c]), 1e-300)
            rel = abs(fd - grad[k, c]) / den
            worst = max(worst, rel)
            assert rel < 1e-5, (name, k, c, fd, grad[k, c])
    print(f"[{name}] parameter gradient vs central differences: worst rel {worst:.2e}", flush=True)


def test_macros_vjp_matches_central_differences():
    name, prob = _cases()[1]
    pop, T = _advance(prob, 3)
    rng = np.random.default_rng(3)
    N, M = prob.N, prob.M
    w = dict(w_rho=rng.standard_normal(N), w_u=rng.standard_normal((3, N)), w_T=rng.standard_normal(N) * 1e-3,
             w_P=rng.standard_normal(N) * 10, w_Y=rng.standard_normal((M, N)))
    adj = orc.OracleAdjoint(prob).init()
    adj.set_state(pop, T)
    lam = adj.macros_vjp(**w)
    v = rng.standard_normal(pop.shape) * pop
    h = 1e-6

    def J(p):
        s = orc.OracleSim(prob).init()
        s.set_state(p, T)
        m = s.macros()
        return sum(float((w["w_" + k] * m[k]).sum()) for k in ("rho", "u", "T", "P", "Y"))
    fd = (J(pop + h * v) - J(pop - h * v)) / (2 * h)
    ad = float((lam * v).sum())
    assert abs(fd - ad) / abs(ad) < 1e-7, (fd, ad)


def test_init_vjp_matches_central_differences():
    name, prob = _cases()[0]
    rng = np.random.default_rng(8)
    S, N, M = prob.M + 1, prob.N, prob.M
    lam0 = rng.standard_normal((S, 27, N))
    adj = orc.OracleAdjoint(prob)
    g = adj.init_vjp(lam0)
    for key, h in (("T", 1e-4), ("rho", 1e-8), ("u", 1e-7), ("Y", 1e-8)):
        base = getattr(prob, key)
        d = rng.standard_normal(base.shape)

        def pop0(sign):
            kw = {key: base + sign * h * d}
            return orc.OracleSim(prob).init(**kw).state()[0]
        fd = float((lam0 * (pop0(1) - pop0(-1))).sum() / (2 * h))
        ad = float((g[key] * d).sum())
        assert abs(fd - ad) / abs(ad) < 1e-6, (key, fd, ad)


def _front_objective(prob, steps, arrhenius=None, T0=None):
    """The smooth front position sum_x (T - T_u) / (T_b - T_u) after `steps` steps."""
    s = orc.OracleSim(prob, arrhenius=arrhenius).init(T=T0)
    s.step(steps)
    return float(((s.macros()["T"] - 300.0) / (2000.0 - 300.0)).sum())


def _reverse_sweep(prob, steps, lib_path=None):
    """dJ/d(ln A, b, Ta) and dJ/dT0 of the front objective by the oracle's reverse sweep:
    forward states kept, then one recorded step per state in reverse order."""
    fwd = orc.OracleSim(prob).init()
    states = [fwd.state()]
    for _ in range(steps):
        fwd.step(1)
        states.append(fwd.state())
    lib = orc.load_ad(lib_path) if lib_path else None
    adj = orc.OracleAdjoint(prob) if lib is None else _adjoint_on(prob, lib)
    adj.set_state(*states[-1])
    lam = adj.macros_vjp(w_T=np.full(prob.N, 1.0 / (2000.0 - 300.0)))
    grad = np.zeros((prob.mech.R, 3))
    for n in range(steps - 1, -1, -1):
        adj.set_state(*states[n])
        lam, g, _ = adj.step_vjp(lam)
        grad += g
    gT0 = adj.init_vjp(lam)["T"]
    return grad, gT0


def _adjoint_on(prob, lib):
    a = orc.OracleAdjoint.__new__(orc.OracleAdjoint)
    orc.OracleSim.__init__(a, prob, lib=lib)
    return a


def test_multistep_gradient_matches_central_differences():
    prob = W.flame1d(nx=20, hot_cells=6)
    steps = 25
    grad, gT0 = _reverse_sweep(prob, steps)
    A = prob.mech.arrhenius
    worst = 0.0
    big = np.argsort(-np.abs(grad[:, 0]))[:2]
    for k in big:
        for c, h in ((0, 1e-5), (1, 1e-5), (2, 1e-1)):
            arr_p, arr_m = A.copy(), A.copy()
            if c == 0:
                arr_p[k, 0] *= np.exp(h)
                arr_m[k, 0] *= np.exp(-h)
            else:
                arr_p[k, c] += h
                arr_m[k, c] -= h
            fd = (_front_objective(prob, steps, arr_p) - _front_objective(prob, steps, arr_m)) / (2 * h)
            rel = abs(fd - grad[k, c]) / max(abs(fd), 1e-300)
            worst = max(worst, rel)
            assert rel < 1e-5, (k, c, fd, grad[k, c])
    d = np.random.default_rng(2).standard_normal(prob.N)
    h = 1e-3
    fd = (_front_objective(prob, steps, T0=prob.T + h * d) - _front_objective(prob, steps, T0=prob.T - h * d)) / (2 * h)
    ad = float((gT0 * d).sum())
    assert abs(fd - ad) / abs(ad) < 1e-6, (fd, ad)
    print(f"multistep: parameter gradient worst rel {worst:.2e}; T0 direction fd {fd:.10e} ad {ad:.10e}", flush=True)


def test_planted_derivative_mistake_is_caught(tmp_path):
    """A wrong derivative rule in the tape (d/db of x^b without its log factor, the rule
    the Arrhenius temperature exponent goes through) must fail the central-difference
    check of the parameter gradient."""
    src = os.path.join(os.path.dirname(orc.__file__), "oracle_ad.cpp")
    text = open(src).read()
    bad = text.replace("b, r * std::log(a.v));", "b, r);")
    assert bad != text
    work = tmp_path / "mut"
    work.mkdir()
    shutil.copy(os.path.join(os.path.dirname(src), "oracle.c"), work / "oracle.c")
    shutil.copy(os.path.join(os.path.dirname(src), "oracle.h"), work / "oracle.h")
    (work / "oracle_ad.cpp").write_text(bad)
    from oracle import build
    lib_path = build.build_ad(src=str(work / "oracle_ad.cpp"), out=str(work / "liboracle_ad_mut.so"))
    prob = W.flame1d(nx=20, hot_cells=6)
    steps = 10
    grad_bad, _ = _reverse_sweep(prob, steps, lib_path=lib_path)
    grad_ok, _ = _reverse_sweep(prob, steps)
    k = int(np.argmax(np.abs(grad_ok[:, 1])))
    h = 1e-5
    A = prob.mech.arrhenius
    arr_p, arr_m = A.copy(), A.copy()
    arr_p[k, 1] += h
    arr_m[k, 1] -= h
    fd = (_front_objective(prob, steps, arr_p) - _front_objective(prob, steps, arr_m)) / (2 * h)
    assert abs(fd - grad_ok[k, 1]) / abs(fd) < 1e-5
    assert abs(fd - grad_bad[k, 1]) / abs(fd) > 1e-2
