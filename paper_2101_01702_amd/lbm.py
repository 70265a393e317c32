"""Python binding of the C ABI in include/lbm.h (argument marshalling only).

Device memory (the workspace and the field buffers) and the stream come from
PyTorch; every step of the method runs in the HIP library liblbm.so.  There is no
fallback: if the library is missing or no HIP device is present, the calls raise.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Dict, Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblbm.so")

LBM_OK = 0
STATUS_NAMES = {0: "LBM_OK", -1: "LBM_ERR_ARG", -2: "LBM_ERR_UNSUPPORTED", -3: "LBM_ERR_HIP",
                -4: "LBM_ERR_WORKSPACE", -5: "LBM_ERR_DEVICE_ANOMALY"}
STORE_F64, STORE_F32, STORE_F16_DEV, STORE_BF16_DEV = 0, 1, 2, 3
NUM_KERNELS = 4
KERNEL_NAMES = ("step", "psi", "corr", "ghost")
ANOM_NONFINITE, ANOM_NEWTON, ANOM_NEG_DENSITY = 1, 2, 4
MAX_SPECIES = 10
MAX_REACTIONS = 64

_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int32)
_up = C.POINTER(C.c_uint8)


class LbmDesc(C.Structure):
    _fields_ = [
        ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
        ("bc", C.c_int32 * 6),
        ("n_species", C.c_int32), ("n_reactions", C.c_int32),
        ("molar_mass", _dp), ("nasa7", _dp), ("diff_ab", _dp),
        ("nu_reac", _ip), ("nu_prod", _ip), ("arrhenius", _dp), ("reversible", _up),
        ("omega", C.c_double), ("omega1", C.c_double),
        ("kappa", C.c_double), ("dt_phys", C.c_double), ("rho_ref", C.c_double), ("p0", C.c_double),
        ("storage", C.c_int32), ("adjoint", C.c_int32), ("ref_state", C.c_void_p),
        ("n_segments", C.c_int32), ("reserved2", C.c_int32), ("segment_lengths", _ip),
        ("diff_T_ref", C.c_double), ("diff_T_exp", C.c_double),
        ("visc_T_ref", C.c_double), ("visc_T_exp", C.c_double),
    ]


class LbmError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


_lib = None

EXPORTS = ("lbm_workspace_size", "lbm_create", "lbm_destroy", "lbm_init_fields", "lbm_step",
           "lbm_step_timed", "lbm_step_graph", "lbm_macros", "lbm_populations", "lbm_diagnostics",
           "lbm_flame_speeds", "lbm_flame_speeds_static", "lbm_state_size", "lbm_state_save",
           "lbm_state_load", "lbm_set_arrhenius", "lbm_adjoint_step", "lbm_adjoint_macros", "lbm_adjoint_init",
           "lbm_stream_copy", "lbm_growth_fit",
           "lbm_status_sync", "lbm_last_error")
DIAG_TOTALS = 4   # heat release rate, nodes with T >= T_iso, mass, total energy
FLAME_WORK = 17   # FP64 work fields per node of lbm_flame_speeds
FLAME_TOTALS = 5  # sum w, sum w S_d, sum w S_a, sum w rho S_d, sum w |x - centre|
FLAME_STATIC_MAX_NODES = 65536   # largest lattice of lbm_flame_speeds_static


def load(path: Optional[str] = None):
    """Load liblbm.so (built by ``python -m paper_2101_01702_amd.build``)."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise ImportError(f"{p} is missing: build it with `python -m paper_2101_01702_amd.build`")
    lib = C.CDLL(p)
    vp = C.c_void_p
    lib.lbm_workspace_size.argtypes = [C.POINTER(LbmDesc), C.POINTER(C.c_size_t)]
    lib.lbm_create.argtypes = [C.POINTER(LbmDesc), vp, C.c_size_t, C.POINTER(vp)]
    lib.lbm_destroy.argtypes = [vp]
    lib.lbm_init_fields.argtypes = [vp, vp, vp, vp, vp, vp]
    lib.lbm_step.argtypes = [vp, C.c_int32, vp]
    lib.lbm_step_timed.argtypes = [vp, C.c_int32, vp, C.POINTER(C.c_float)]
    lib.lbm_step_graph.argtypes = [vp, C.c_int32, vp]
    lib.lbm_macros.argtypes = [vp, vp, vp, vp, vp, vp, vp]
    lib.lbm_populations.argtypes = [vp, vp, C.c_int64, vp, vp, vp]
    lib.lbm_diagnostics.argtypes = [vp, C.c_double, vp, vp, vp]
    lib.lbm_flame_speeds.argtypes = [vp, C.c_double, C.POINTER(C.c_double), vp, vp, vp, vp]
    lib.lbm_flame_speeds_static.argtypes = [vp, C.c_double, C.POINTER(C.c_double), vp, vp, vp]
    lib.lbm_state_size.argtypes = [vp, C.POINTER(C.c_size_t)]
    lib.lbm_state_save.argtypes = [vp, vp, vp]
    lib.lbm_state_load.argtypes = [vp, vp, vp]
    lib.lbm_set_arrhenius.argtypes = [vp, C.POINTER(C.c_double), vp]
    lib.lbm_adjoint_step.argtypes = [vp, vp, vp, vp, vp]
    lib.lbm_adjoint_macros.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp, vp]
    lib.lbm_adjoint_init.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp]
    lib.lbm_stream_copy.argtypes = [vp, vp, C.c_size_t, vp]
    lib.lbm_growth_fit.argtypes = [_dp, _dp, C.c_int64, _dp, _dp]
    lib.lbm_status_sync.argtypes = [vp, vp, C.POINTER(C.c_uint32)]
    lib.lbm_last_error.argtypes = [vp]
    lib.lbm_last_error.restype = C.c_char_p
    for name in EXPORTS:
        if name != "lbm_last_error":
            getattr(lib, name).restype = C.c_int
    if path is None:
        _lib = lib
    return lib


def _c64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def make_desc(prob, storage: Optional[int] = None, adjoint: bool = False):
    """lbm_desc of a workloads.Problem; returns (desc, arrays kept alive)."""
    mech = prob.mech
    keep = dict(molar_mass=_c64(mech.molar_mass), nasa7=_c64(mech.nasa7), diff=_c64(prob.diff),
                nu_reac=np.ascontiguousarray(mech.nu_reac, np.int32).reshape(-1),
                nu_prod=np.ascontiguousarray(mech.nu_prod, np.int32).reshape(-1),
                arrhenius=_c64(mech.arrhenius).reshape(-1),
                reversible=np.ascontiguousarray(mech.reversible, np.uint8))
    d = LbmDesc()
    d.nx, d.ny, d.nz = prob.nx, prob.ny, prob.nz
    d.bc = (C.c_int32 * 6)(*prob.bc)
    d.n_species, d.n_reactions = mech.M, mech.R
    d.molar_mass = keep["molar_mass"].ctypes.data_as(_dp)
    d.nasa7 = keep["nasa7"].ctypes.data_as(_dp)
    d.diff_ab = keep["diff"].ctypes.data_as(_dp)
    if mech.R:
        d.nu_reac = keep["nu_reac"].ctypes.data_as(_ip)
        d.nu_prod = keep["nu_prod"].ctypes.data_as(_ip)
        d.arrhenius = keep["arrhenius"].ctypes.data_as(_dp)
        d.reversible = keep["reversible"].ctypes.data_as(_up)
    d.omega, d.omega1 = prob.omega, prob.omega1
    d.kappa, d.dt_phys, d.rho_ref, d.p0 = prob.kappa, prob.dt_phys, prob.rho_ref, prob.p0
    d.storage = prob.storage if storage is None else storage
    d.adjoint = 1 if adjoint else 0
    d.diff_T_ref = float(getattr(prob, "diff_T_ref", 0.0))
    d.diff_T_exp = float(getattr(prob, "diff_T_exp", 0.0))
    d.visc_T_ref = float(getattr(prob, "visc_T_ref", 0.0))
    d.visc_T_exp = float(getattr(prob, "visc_T_exp", 0.0))
    segs = getattr(prob, "segments", None)
    if segs is not None and len(segs) > 1:
        keep["segments"] = np.ascontiguousarray(segs, np.int32)
        d.n_segments = len(segs)
        d.segment_lengths = keep["segments"].ctypes.data_as(_ip)
    if d.storage in (STORE_F16_DEV, STORE_BF16_DEV):
        ref = prob.ref_state
        if ref is None:
            # mean state of the initial fields: density, temperature, mass-weighted Y
            rho = np.asarray(prob.rho, np.float64)
            Y = (np.asarray(prob.Y, np.float64) * rho).sum(axis=1) / rho.sum()
            ref = np.concatenate([[rho.mean(), np.asarray(prob.T, np.float64).mean()], Y / Y.sum()])
        keep["ref_state"] = _c64(ref)
        d.ref_state = keep["ref_state"].ctypes.data_as(C.c_void_p)
    return d, keep


def workspace_size(prob, storage: Optional[int] = None) -> int:
    lib = load()
    d, _keep = make_desc(prob, storage)
    n = C.c_size_t(0)
    st = lib.lbm_workspace_size(C.byref(d), C.byref(n))
    if st != LBM_OK:
        raise LbmError(st, lib.lbm_last_error(None).decode())
    return int(n.value)


class Solver:
    """One lattice on one HIP device, advanced by the HIP library."""

    def __init__(self, prob, storage: Optional[int] = None, device=None, adjoint: bool = False):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("no HIP device: the reactive LBM step runs only on the GPU")
        self.torch = torch
        self.lib = load()
        self.prob = prob
        self.M = prob.mech.M
        self.S = self.M + 1
        self.N = prob.N
        self.device = (torch.device(device) if device is not None
                       else torch.device("cuda", torch.cuda.current_device()))
        self.desc, self._keep = make_desc(prob, storage, adjoint)
        self.adjoint = bool(adjoint)
        self.storage = self.desc.storage
        self.ref_state = self._keep.get("ref_state")
        n = C.c_size_t(0)
        self._check(self.lib.lbm_workspace_size(C.byref(self.desc), C.byref(n)), None)
        self.ws_bytes = int(n.value)
        with torch.cuda.device(self.device):
            self._ws_raw = torch.empty(self.ws_bytes + 256, dtype=torch.uint8, device=self.device)
            base = self._ws_raw.data_ptr()
            self._ws_ptr = (base + 255) // 256 * 256
            h = C.c_void_p()
            self._check(self.lib.lbm_create(C.byref(self.desc), C.c_void_p(self._ws_ptr), C.c_size_t(self.ws_bytes),
                                            C.byref(h)), None)
        self.h = h

    # ------------------------------------------------------------------------------
    def _check(self, st, h):
        if st != LBM_OK:
            msg = self.lib.lbm_last_error(h)
            raise LbmError(st, msg.decode() if msg else "")

    def _stream(self):
        return C.c_void_p(self.torch.cuda.current_stream(self.device).cuda_stream)

    def _dev(self, a, dtype=None):
        t = self.torch
        if isinstance(a, t.Tensor):
            return a.to(device=self.device, dtype=dtype or t.float64).contiguous()
        return t.as_tensor(np.ascontiguousarray(a), dtype=dtype or t.float64, device=self.device).contiguous()

    def close(self):
        if getattr(self, "h", None) and self.h.value:
            self.lib.lbm_destroy(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------------------------
    def init(self, rho=None, u=None, T=None, Y=None):
        p = self.prob
        N, M = self.N, self.M
        r = self._dev(p.rho if rho is None else rho).reshape(N)
        uu = self._dev(p.u if u is None else u).reshape(3, N)
        TT = self._dev(p.T if T is None else T).reshape(N)
        YY = self._dev(p.Y if Y is None else Y).reshape(M, N)
        self._init_keep = (r, uu, TT, YY)
        self._check(self.lib.lbm_init_fields(self.h, C.c_void_p(r.data_ptr()), C.c_void_p(uu.data_ptr()),
                                             C.c_void_p(TT.data_ptr()), C.c_void_p(YY.data_ptr()),
                                             self._stream()), self.h)
        return self

    def step(self, n: int = 1):
        self._check(self.lib.lbm_step(self.h, int(n), self._stream()), self.h)

    def step_graph(self, n: int = 1):
        """n steps replayed from a HIP graph recorded at the first call of that n."""
        self._check(self.lib.lbm_step_graph(self.h, int(n), self._stream()), self.h)

    def step_timed(self, n: int = 1) -> Dict[str, float]:
        ms = (C.c_float * NUM_KERNELS)()
        self._check(self.lib.lbm_step_timed(self.h, int(n), self._stream(), ms), self.h)
        return {KERNEL_NAMES[k]: float(ms[k]) for k in range(NUM_KERNELS)}

    def macros(self, to_numpy: bool = True):
        t = self.torch
        N, M = self.N, self.M
        rho = t.empty(N, dtype=t.float64, device=self.device)
        u = t.empty(3, N, dtype=t.float64, device=self.device)
        T = t.empty(N, dtype=t.float64, device=self.device)
        P = t.empty(N, dtype=t.float64, device=self.device)
        Y = t.empty(M, N, dtype=t.float64, device=self.device)
        self._check(self.lib.lbm_macros(self.h, *(C.c_void_p(a.data_ptr()) for a in (rho, u, T, P, Y)),
                                        self._stream()), self.h)
        out = dict(rho=rho, u=u, T=T, P=P, Y=Y)
        if to_numpy:
            t.cuda.synchronize(self.device)
            out = {k: v.cpu().numpy() for k, v in out.items()}
        return out

    def diagnostics(self, T_iso: float, to_numpy: bool = True):
        """Heat release rate field [N] and the sums (heat release, nodes with
        T >= T_iso, mass, total energy) of the current state (``lbm_diagnostics``)."""
        t = self.torch
        hrr = t.empty(self.N, dtype=t.float64, device=self.device)
        tot = t.empty(DIAG_TOTALS, dtype=t.float64, device=self.device)
        self._check(self.lib.lbm_diagnostics(self.h, C.c_double(T_iso), C.c_void_p(hrr.data_ptr()),
                                             C.c_void_p(tot.data_ptr()), self._stream()), self.h)
        if to_numpy:
            t.cuda.synchronize(self.device)
            return hrr.cpu().numpy(), tot.cpu().numpy()
        return hrr, tot

    def flame_speeds(self, T_iso: float, centre=(0.0, 0.0, 0.0), to_numpy: bool = True):
        """S_d, S_a (eq. sd) and isosurface weights w per node [3, N] of the current state,
        and the sums [w, w S_d, w S_a, w rho S_d, w |x - centre|]."""
        t = self.torch
        work = t.empty(FLAME_WORK * self.N, dtype=t.float64, device=self.device)
        out = t.empty(3, self.N, dtype=t.float64, device=self.device)
        tot = t.empty(FLAME_TOTALS, dtype=t.float64, device=self.device)
        c = (C.c_double * 3)(*[float(v) for v in centre])
        self._check(self.lib.lbm_flame_speeds(self.h, float(T_iso), c, C.c_void_p(work.data_ptr()),
                                              C.c_void_p(out.data_ptr()), C.c_void_p(tot.data_ptr()),
                                              self._stream()), self.h)
        if to_numpy:
            t.cuda.synchronize(self.device)
            o = out.cpu().numpy()
            return dict(Sd=o[0], Sa=o[1], w=o[2], totals=tot.cpu().numpy())
        return dict(Sd=out[0], Sa=out[1], w=out[2], totals=tot)

    def flame_speeds_static(self, T_iso: float, centre=(0.0, 0.0, 0.0), to_numpy: bool = True):
        """``flame_speeds`` through lbm_flame_speeds_static: no work buffer is passed, the
        library's per-GPU scratch array holds the work fields (lattices of at most
        FLAME_STATIC_MAX_NODES nodes)."""
        t = self.torch
        out = t.empty(3, self.N, dtype=t.float64, device=self.device)
        tot = t.empty(FLAME_TOTALS, dtype=t.float64, device=self.device)
        c = (C.c_double * 3)(*[float(v) for v in centre])
        self._check(self.lib.lbm_flame_speeds_static(self.h, float(T_iso), c, C.c_void_p(out.data_ptr()),
                                                     C.c_void_p(tot.data_ptr()), self._stream()), self.h)
        if to_numpy:
            t.cuda.synchronize(self.device)
            o = out.cpu().numpy()
            return dict(Sd=o[0], Sa=o[1], w=o[2], totals=tot.cpu().numpy())
        return dict(Sd=out[0], Sa=out[1], w=out[2], totals=tot)

    def mean_radius(self, T_iso: float, centre=(0.0, 0.0, 0.0)) -> float:
        """Mean distance from ``centre`` over the isosurface T = T_iso (eq. rmean), from
        the isosurface sums of lbm_flame_speeds; nan when no node lies on the surface."""
        tot = self.flame_speeds(T_iso, centre)["totals"]
        return float(tot[4] / tot[0]) if tot[0] > 0 else float("nan")

    def populations(self, nodes: Sequence[int], to_numpy: bool = True):
        """Pre-collision populations [S, 27, k] and stored temperatures at node ids."""
        t = self.torch
        idx = self._dev(np.asarray(nodes, dtype=np.int64), dtype=t.int64).reshape(-1)
        k = idx.numel()
        out = t.empty(self.S, 27, max(k, 1), dtype=t.float64, device=self.device)
        Tn = t.empty(max(k, 1), dtype=t.float64, device=self.device)
        self._check(self.lib.lbm_populations(self.h, C.c_void_p(idx.data_ptr()), C.c_int64(k),
                                             C.c_void_p(out.data_ptr()), C.c_void_p(Tn.data_ptr()),
                                             self._stream()), self.h)
        out, Tn = out[:, :, :k], Tn[:k]
        if to_numpy:
            t.cuda.synchronize(self.device)
            return out.cpu().numpy(), Tn.cpu().numpy()
        return out, Tn

    # ---- state snapshots and the discrete adjoint -------------------------------------
    def state_size(self) -> int:
        n = C.c_size_t(0)
        self._check(self.lib.lbm_state_size(self.h, C.byref(n)), self.h)
        return int(n.value)

    def new_state_buffer(self):
        """A device buffer for one state snapshot (256-byte aligned view of a uint8 tensor)."""
        t = self.torch
        n = self.state_size()
        raw = t.empty(n + 256, dtype=t.uint8, device=self.device)
        off = (-raw.data_ptr()) % 256
        return raw[off:off + n]

    def state_save(self, buf=None):
        buf = self.new_state_buffer() if buf is None else buf
        self._check(self.lib.lbm_state_save(self.h, C.c_void_p(buf.data_ptr()), self._stream()), self.h)
        return buf

    def state_load(self, buf):
        self._check(self.lib.lbm_state_load(self.h, C.c_void_p(buf.data_ptr()), self._stream()), self.h)

    def set_arrhenius(self, arrhenius):
        """Replace the reactions' (A, b, Ta) [R, 3] (host values)."""
        arr = np.ascontiguousarray(arrhenius, dtype=np.float64).reshape(-1)
        self._keep["arrhenius_set"] = arr
        self._check(self.lib.lbm_set_arrhenius(self.h, arr.ctypes.data_as(_dp), self._stream()), self.h)

    def _ptr(self, a):
        return C.c_void_p(0) if a is None else C.c_void_p(a.data_ptr())

    def adjoint_macros(self, state=None, w_rho=None, w_u=None, w_T=None, w_P=None, w_Y=None):
        """Adjoint populations [S, 27, N] (device FP64) of sum over nodes of the weighted
        macroscopic fields at a snapshot (None: the current state)."""
        t = self.torch
        ws = [None if w is None else self._dev(w) for w in (w_rho, w_u, w_T, w_P, w_Y)]
        out = t.empty(self.S, 27, self.N, dtype=t.float64, device=self.device)
        self._check(self.lib.lbm_adjoint_macros(self.h, self._ptr(state), *(self._ptr(w) for w in ws),
                                                C.c_void_p(out.data_ptr()), self._stream()), self.h)
        return out

    def adjoint_step(self, lam, state=None, grad=None):
        """lambda_n from lambda_{n+1} (device FP64 [S, 27, N], updated in place) at the
        snapshot of step n; grad [R, 3] (device FP64) is incremented."""
        self._check(self.lib.lbm_adjoint_step(self.h, self._ptr(state), C.c_void_p(lam.data_ptr()),
                                              self._ptr(grad), self._stream()), self.h)
        return lam

    def adjoint_init(self, lam0, rho=None, u=None, T=None, Y=None):
        """Gradients (rho, u, T, Y) of sum(lam0 * pop_0) through the equilibrium initial
        state of the given fields (default: the problem's)."""
        t = self.torch
        p = self.prob
        N, M = self.N, self.M
        f = [self._dev(p.rho if rho is None else rho).reshape(N), self._dev(p.u if u is None else u).reshape(3, N),
             self._dev(p.T if T is None else T).reshape(N), self._dev(p.Y if Y is None else Y).reshape(M, N)]
        g = [t.empty_like(a) for a in f]
        self._check(self.lib.lbm_adjoint_init(self.h, *(C.c_void_p(a.data_ptr()) for a in f),
                                              C.c_void_p(lam0.data_ptr()), *(C.c_void_p(a.data_ptr()) for a in g),
                                              self._stream()), self.h)
        return dict(rho=g[0], u=g[1], T=g[2], Y=g[3])

    def status(self) -> int:
        bits = C.c_uint32(0)
        st = self.lib.lbm_status_sync(self.h, self._stream(), C.byref(bits))
        if st not in (LBM_OK, -5):
            self._check(st, self.h)
        return int(bits.value)


def growth_exponent(t: Sequence[float], r: Sequence[float]):
    """Least-squares fit of R = a t^alpha to samples of a mean radius (the growth law of
    the expanding flame, Sec. 5.2), by lbm_growth_fit: returns (a, alpha)."""
    lib = load()
    tt = np.ascontiguousarray(t, dtype=np.float64).reshape(-1)
    rr = np.ascontiguousarray(r, dtype=np.float64).reshape(-1)
    if tt.size != rr.size:
        raise ValueError("t and r must have the same length")
    a, alpha = C.c_double(0.0), C.c_double(0.0)
    st = lib.lbm_growth_fit(tt.ctypes.data_as(_dp), rr.ctypes.data_as(_dp), tt.size, C.byref(a), C.byref(alpha))
    if st != LBM_OK:
        raise ValueError(lib.lbm_last_error(None).decode())
    return float(a.value), float(alpha.value)
