"""ctypes wrapper of the FP64 CPU oracle (test infrastructure only)."""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")
LIB_AD_PATH = os.path.join(HERE, "liboracle_ad.so")

F_T, F_RDOT, F_DU, F_BETA, F_X, F_GRADY, F_PHI, F_PSI, F_NEWTON = range(9)

_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int32)
_up = C.POINTER(C.c_uint8)


class _Problem(C.Structure):
    _fields_ = [
        ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
        ("bc", C.c_int32 * 6),
        ("M", C.c_int32), ("R", C.c_int32),
        ("molar_mass", _dp), ("nasa7", _dp), ("diff", _dp),
        ("nu_reac", _ip), ("nu_prod", _ip), ("arrhenius", _dp), ("reversible", _up),
        ("omega", C.c_double), ("omega1", C.c_double),
        ("kappa", C.c_double), ("dt_phys", C.c_double), ("rho_ref", C.c_double),
        ("p0", C.c_double),
        ("diff_T_ref", C.c_double), ("diff_T_exp", C.c_double),
        ("visc_T_ref", C.c_double), ("visc_T_exp", C.c_double),
    ]


_libs = {}


def load(path=None):
    """Load the oracle library (``path`` selects another build of the same source)."""
    path = path or LIB_PATH
    if path in _libs:
        return _libs[path]
    if path == LIB_PATH and not os.path.exists(LIB_PATH):
        from . import build as _b
        _b.build()
    lib = C.CDLL(path)
    lib.orc_create.restype = C.c_void_p
    lib.orc_create.argtypes = [C.POINTER(_Problem)]
    lib.orc_destroy.argtypes = [C.c_void_p]
    lib.orc_init.argtypes = [C.c_void_p, _dp, _dp, _dp, _dp]
    lib.orc_step.restype = C.c_uint32
    lib.orc_step.argtypes = [C.c_void_p, C.c_int32, C.c_int32]
    lib.orc_macros.restype = C.c_uint32
    lib.orc_macros.argtypes = [C.c_void_p, _dp, _dp, _dp, _dp, _dp]
    lib.orc_flame_speeds.restype = C.c_uint32
    lib.orc_flame_speeds.argtypes = [C.c_void_p, C.c_double, _dp, _dp, _dp]
    lib.orc_get_state.argtypes = [C.c_void_p, _dp, _dp]
    lib.orc_set_state.argtypes = [C.c_void_p, _dp, _dp]
    lib.orc_get_post.argtypes = [C.c_void_p, _dp]
    lib.orc_get_field.argtypes = [C.c_void_p, C.c_int32, _dp]
    lib.orc_product_form.argtypes = [C.c_double, _dp, C.c_double, _dp]
    lib.orc_grad_form.argtypes = [C.c_double, _dp, _dp, _dp]
    lib.orc_thermo.argtypes = [C.c_void_p, C.c_int32, C.c_double, _dp]
    lib.orc_temperature.restype = C.c_int32
    lib.orc_temperature.argtypes = [C.c_void_p, _dp, C.c_double, C.c_double, _dp]
    lib.orc_rates.argtypes = [C.c_void_p, _dp, C.c_double, _dp]
    lib.orc_diffusion.argtypes = [C.c_void_p, _dp, C.c_double, _dp, _dp, _dp]
    lib.orc_iso_grad.argtypes = [C.c_void_p, _dp, _dp]
    _libs[path] = lib
    return lib


def load_ad(path=None):
    """Load the reverse sweep of the oracle (liboracle_ad.so: the same source on a
    recording arithmetic type; see oracle_ad.cpp)."""
    path = path or LIB_AD_PATH
    if path in _libs:
        return _libs[path]
    if path == LIB_AD_PATH and not os.path.exists(LIB_AD_PATH):
        from . import build as _b
        _b.build_ad()
    lib = C.CDLL(path)
    lib.orc_create.restype = C.c_void_p
    lib.orc_create.argtypes = [C.POINTER(_Problem)]
    lib.orc_destroy.argtypes = [C.c_void_p]
    lib.orc_step.restype = C.c_uint32
    lib.orc_step.argtypes = [C.c_void_p, C.c_int32, C.c_int32]
    lib.orc_get_state.argtypes = [C.c_void_p, _dp, _dp]
    lib.orc_set_state.argtypes = [C.c_void_p, _dp, _dp]
    lib.orc_ad_step_vjp.restype = C.c_uint32
    lib.orc_ad_step_vjp.argtypes = [C.c_void_p, _dp, _dp, _dp]
    lib.orc_ad_macros_vjp.restype = C.c_uint32
    lib.orc_ad_macros_vjp.argtypes = [C.c_void_p, _dp, _dp, _dp, _dp, _dp, _dp]
    lib.orc_ad_init_vjp.argtypes = [C.c_void_p, _dp, _dp, _dp, _dp, _dp, _dp, _dp, _dp, _dp]
    lib.orc_ad_tape_entries.restype = C.c_int64
    _libs[path] = lib
    return lib


def _d(a):
    return a.ctypes.data_as(_dp)


def _c64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def product_form(dens, v, zeta, lib=None):
    out = np.zeros(27)
    (lib or load()).orc_product_form(float(dens), _d(_c64(v)), float(zeta), _d(out))
    return out


def grad_form(rhoE, q, Rt, lib=None):
    out = np.zeros(27)
    (lib or load()).orc_grad_form(float(rhoE), _d(_c64(q)), _d(_c64(Rt).reshape(9)), _d(out))
    return out


class OracleSim:
    """One lattice held by the oracle; arrays in the layouts of oracle.h."""

    def __init__(self, prob, lib=None, arrhenius=None):
        lib = lib or load()
        self.prob = prob
        mech = prob.mech
        self.M = mech.M
        self.S = self.M + 1
        self.N = prob.N
        keep = dict(
            molar_mass=_c64(mech.molar_mass), nasa7=_c64(mech.nasa7), diff=_c64(prob.diff),
            nu_reac=np.ascontiguousarray(mech.nu_reac, np.int32).reshape(-1),
            nu_prod=np.ascontiguousarray(mech.nu_prod, np.int32).reshape(-1),
            arrhenius=_c64(mech.arrhenius if arrhenius is None else arrhenius).reshape(-1),
            reversible=np.ascontiguousarray(mech.reversible, np.uint8))
        if keep["nu_reac"].size == 0:
            keep["nu_reac"] = np.zeros(1, np.int32)
            keep["nu_prod"] = np.zeros(1, np.int32)
            keep["arrhenius"] = np.zeros(3)
            keep["reversible"] = np.zeros(1, np.uint8)
        self._keep = keep
        p = _Problem()
        p.nx, p.ny, p.nz = prob.nx, prob.ny, prob.nz
        p.bc = (C.c_int32 * 6)(*prob.bc)
        p.M, p.R = mech.M, mech.R
        p.molar_mass = _d(keep["molar_mass"])
        p.nasa7 = _d(keep["nasa7"])
        p.diff = _d(keep["diff"])
        p.nu_reac = keep["nu_reac"].ctypes.data_as(_ip)
        p.nu_prod = keep["nu_prod"].ctypes.data_as(_ip)
        p.arrhenius = _d(keep["arrhenius"])
        p.reversible = keep["reversible"].ctypes.data_as(_up)
        p.omega, p.omega1 = prob.omega, prob.omega1
        p.kappa, p.dt_phys, p.rho_ref, p.p0 = prob.kappa, prob.dt_phys, prob.rho_ref, prob.p0
        p.diff_T_ref = getattr(prob, "diff_T_ref", 0.0)
        p.diff_T_exp = getattr(prob, "diff_T_exp", 0.0)
        p.visc_T_ref = getattr(prob, "visc_T_ref", 0.0)
        p.visc_T_exp = getattr(prob, "visc_T_exp", 0.0)
        self._p = p
        h = lib.orc_create(C.byref(p))
        if not h:
            raise ValueError("oracle rejected the problem description")
        self._h = h
        self._lib = lib

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            self._lib.orc_destroy(h)
            self._h = None

    def init(self, rho=None, u=None, T=None, Y=None):
        pr = self.prob
        rho = _c64(pr.rho if rho is None else rho)
        u = _c64(pr.u if u is None else u)
        T = _c64(pr.T if T is None else T)
        Y = _c64(pr.Y if Y is None else Y)
        self._lib.orc_init(self._h, _d(rho), _d(u), _d(T), _d(Y))
        return self

    def step(self, n=1, threads=1):
        return int(self._lib.orc_step(self._h, int(n), int(threads)))

    def macros(self):
        N, M = self.N, self.M
        rho, u, T, P, Y = np.zeros(N), np.zeros((3, N)), np.zeros(N), np.zeros(N), np.zeros((M, N))
        anom = self._lib.orc_macros(self._h, _d(rho), _d(u), _d(T), _d(P), _d(Y))
        return dict(rho=rho, u=u, T=T, P=P, Y=Y, anomaly=int(anom))

    def flame_speeds(self, T_iso, centre=(0.0, 0.0, 0.0)):
        """S_d, S_a (eq. sd) and isosurface weights w per node of the current state, and
        the sums [w, w S_d, w S_a, w rho S_d, w |x - centre|]."""
        out = np.zeros((3, self.N))
        tot = np.zeros(5)
        c = _c64(np.asarray(centre, np.float64))
        anom = self._lib.orc_flame_speeds(self._h, float(T_iso), _d(c), _d(out), _d(tot))
        return dict(Sd=out[0], Sa=out[1], w=out[2], totals=tot, anomaly=int(anom))

    def state(self):
        pop = np.zeros((self.S, 27, self.N))
        T = np.zeros(self.N)
        self._lib.orc_get_state(self._h, _d(pop), _d(T))
        return pop, T

    def set_state(self, pop, T):
        pop = _c64(pop).reshape(self.S, 27, self.N)
        T = _c64(T).reshape(self.N)
        self._lib.orc_set_state(self._h, _d(pop), _d(T))

    def post(self):
        out = np.zeros((self.S, 27, self.N))
        self._lib.orc_get_post(self._h, _d(out))
        return out

    def field(self, which):
        N, M = self.N, self.M
        shapes = {F_T: (N,), F_RDOT: (M, N), F_DU: (M, 3, N), F_BETA: (M, N), F_X: (3, N),
                  F_GRADY: (M, 3, N), F_PHI: (3, N), F_PSI: (3, N), F_NEWTON: (N,)}
        out = np.zeros(shapes[which])
        self._lib.orc_get_field(self._h, int(which), _d(out))
        return out

    # ---- pieces of the method --------------------------------------------------------
    def thermo(self, a, T):
        out = np.zeros(6)
        self._lib.orc_thermo(self._h, int(a), float(T), _d(out))
        return dict(cp_R=out[0], h_RT=out[1], s_R=out[2], U=out[3], H=out[4], Cv=out[5])

    def temperature(self, Y, e_target, T_start):
        T = np.zeros(1)
        it = self._lib.orc_temperature(self._h, _d(_c64(Y)), float(e_target), float(T_start), _d(T))
        return float(T[0]), int(it)

    def rates(self, rho_a, T):
        out = np.zeros(self.M)
        self._lib.orc_rates(self._h, _d(_c64(rho_a)), float(T), _d(out))
        return out

    def diffusion(self, Y, T, rhs):
        du = np.zeros((self.M, 3))
        beta = np.zeros(self.M)
        self._lib.orc_diffusion(self._h, _d(_c64(Y)), float(T), _d(_c64(rhs).reshape(-1)), _d(du),
                                _d(beta))
        return du, beta

    def iso_grad(self, field):
        out = np.zeros((3, self.N))
        self._lib.orc_iso_grad(self._h, _d(_c64(field)), _d(out))
        return out


class OracleAdjoint(OracleSim):
    """The oracle on its recording arithmetic type: the same forward steps, plus the
    vector-Jacobian products of one step, of the macroscopic fields and of the
    equilibrium initial state, by a reverse pass over the recorded operations."""

    def __init__(self, prob, arrhenius=None):
        super().__init__(prob, lib=load_ad(), arrhenius=arrhenius)

    def init(self, rho=None, u=None, T=None, Y=None):
        self.init_vjp(np.zeros((self.S, 27, self.N)), rho, u, T, Y)
        return self

    def macros(self):
        raise NotImplementedError("use OracleSim for forward fields")

    def step_vjp(self, lam_next):
        """(lam_prev [S, 27, N], grad [R, 3] w.r.t. (ln A, b, Ta), anomaly bits); the
        state advances by one step."""
        lam_next = _c64(lam_next).reshape(self.S, 27, self.N)
        lam_prev = np.zeros_like(lam_next)
        R = self.prob.mech.R
        grad = np.zeros((max(R, 1), 3))
        anom = self._lib.orc_ad_step_vjp(self._h, _d(lam_next), _d(lam_prev), _d(grad))
        return lam_prev, grad[:R], int(anom)

    def macros_vjp(self, w_rho=None, w_u=None, w_T=None, w_P=None, w_Y=None):
        """Adjoint populations [S, 27, N] of sum(w_rho rho + w_u u + w_T T + w_P P + w_Y Y)
        over the lattice, at the current state."""
        lam = np.zeros((self.S, 27, self.N))
        ws = [None if w is None else _c64(w) for w in (w_rho, w_u, w_T, w_P, w_Y)]
        ptrs = [C.cast(None, _dp) if w is None else _d(w) for w in ws]
        self._lib.orc_ad_macros_vjp(self._h, *ptrs, _d(lam))
        return lam

    def init_vjp(self, lam0, rho=None, u=None, T=None, Y=None):
        """Gradients (rho [N], u [3, N], T [N], Y [M, N]) of sum(lam0 * pop_0) for the
        equilibrium initial state of the given fields; sets that state."""
        pr = self.prob
        N, M = self.N, self.M
        f = [_c64(pr.rho if rho is None else rho), _c64(pr.u if u is None else u),
             _c64(pr.T if T is None else T), _c64(pr.Y if Y is None else Y)]
        g = [np.zeros(N), np.zeros((3, N)), np.zeros(N), np.zeros((M, N))]
        lam0 = _c64(lam0).reshape(self.S, 27, N)
        self._lib.orc_ad_init_vjp(self._h, *(_d(a) for a in f), _d(lam0), *(_d(a) for a in g))
        return dict(rho=g[0], u=g[1], T=g[2], Y=g[3])

    def tape_entries(self):
        return int(self._lib.orc_ad_tape_entries())
