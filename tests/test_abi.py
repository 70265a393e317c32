"""C ABI contract checks that need no GPU: the library loads, exports every entry
point the header declares, and rejects invalid descriptors with explicit errors."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_2101_01702_amd import lbm
from paper_2101_01702_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lbm.h")


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(lbm.LIB_PATH):
        from paper_2101_01702_amd import build
        build.build()
    return lbm.load()


def declared_functions():
    src = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:lbm_status|const char \*)\s*(lbm_\w+)\s*\(", src, re.M)))


def test_header_declares_entry_points():
    names = declared_functions()
    for n in ("lbm_create", "lbm_init_fields", "lbm_step", "lbm_macros", "lbm_adjoint_step"):
        assert n in names
    assert set(names) == set(lbm.EXPORTS)


def test_library_exports_every_declared_symbol(lib):
    for name in declared_functions():
        assert hasattr(lib, name), name


def _desc(prob, **kw):
    d, keep = lbm.make_desc(prob)
    for k, v in kw.items():
        setattr(d, k, v)
    return d, keep


def _ws(lib, d):
    n = C.c_size_t(0)
    st = lib.lbm_workspace_size(C.byref(d), C.byref(n))
    return st, n.value, lib.lbm_last_error(None).decode()


def test_workspace_size_config1(lib):
    prob = W.config1()
    d, keep = _desc(prob)
    st, n, _ = _ws(lib, d)
    assert st == 0
    S, N, M = 4, 512, 3
    pops = 2 * S * 27 * N * 8
    # beyond the two population copies: temperature, side channel (2M + 7 words),
    # psi (3) and corrections (6) words per node, plus the constant tables
    per_node = 8 * (1 + 2 * M + 7 + 3 + 6)
    assert pops + per_node * N < n < pops + per_node * N + 200_000


def test_workspace_grows_with_ghost_layer(lib):
    per = W.config1(nx=16, ny=4, nz=4)
    opn = W.config1(nx=16, ny=4, nz=4)
    opn.bc = (1, 1, 0, 0, 0, 0)
    d1, k1 = _desc(per)
    d2, k2 = _desc(opn)
    assert _ws(lib, d2)[1] - _ws(lib, d1)[1] >= 2 * 4 * 27 * (2 * 4 * 4) * 8


@pytest.mark.parametrize("field,value,needle", [
    ("nx", 0, "lattice sizes"),
    ("n_species", 1, "n_species"),
    ("n_species", 11, "n_species"),
    ("n_reactions", -1, "n_reactions"),
    ("omega", 2.0, "omega"),
    ("omega1", 0.0, "omega1"),
    ("kappa", 0.0, "kappa"),
    ("rho_ref", -1.0, "rho_ref"),
    ("storage", 7, "storage"),
])
def test_invalid_descriptor_rejected(lib, field, value, needle):
    d, keep = _desc(W.config1(), **{field: value})
    st, _, msg = _ws(lib, d)
    assert st == -1
    assert needle in msg


def test_unpaired_periodic_face_rejected(lib):
    d, keep = _desc(W.config1())
    d.bc = (C.c_int32 * 6)(0, 1, 0, 0, 0, 0)
    st, _, msg = _ws(lib, d)
    assert st == -1 and "pairs" in msg


def test_asymmetric_diffusivity_rejected(lib):
    prob = W.config1()
    prob.diff = prob.diff.copy()
    prob.diff[0, 1] *= 1.5
    d, keep = _desc(prob)
    st, _, msg = _ws(lib, d)
    assert st == -1 and "symmetric" in msg


def test_mass_unbalanced_reaction_rejected(lib):
    prob = W.config1()
    prob.mech.nu_prod = prob.mech.nu_prod * 2
    d, keep = _desc(prob)
    st, _, msg = _ws(lib, d)
    assert st == -1 and "mass" in msg


def test_reaction_order_limit(lib):
    """Stoichiometric coefficients 0..3 and at most LBM_MAX_ORDER (8) molecules on
    each side of a reaction (the checks do not need the reaction to be physical)."""
    prob = W.config1()
    prob.mech.nu_reac = np.array([[3, 3, 0]], np.int32)
    prob.mech.nu_prod = np.array([[0, 0, 3]], np.int32)
    d, keep = _desc(prob)
    st, _, msg = _ws(lib, d)
    assert st == 0, msg
    prob.mech.nu_reac = np.array([[3, 3, 3]], np.int32)
    prob.mech.nu_prod = np.array([[0, 0, 6]], np.int32)
    d, keep = _desc(prob)
    st, _, msg = _ws(lib, d)
    assert st == -1 and "coefficients" in msg      # 6 exceeds the per-species 0..3
    prob.mech.nu_reac = np.array([[3, 3, 3]], np.int32)
    prob.mech.nu_prod = np.array([[3, 3, 3]], np.int32)      # 9 molecules on each side
    d, keep = _desc(prob)
    st, _, msg = _ws(lib, d)
    assert st == -1 and "molecules" in msg


def test_deviation_formats_need_a_valid_reference_state(lib):
    """LBM_STORE_F16_DEV / _BF16_DEV store populations in 2 bytes and need ref_state
    (density > 0, temperature > 0, mass fractions >= 0 summing to 1)."""
    prob = W.config1()
    sizes = {}
    for st in (W.STORE_F64, W.STORE_F32, W.STORE_F16_DEV, W.STORE_BF16_DEV):
        d, keep = lbm.make_desc(prob, st)
        code, n, msg = _ws(lib, d)
        assert code == 0, msg
        sizes[st] = n
    S, N = 4, 512
    assert sizes[W.STORE_F32] - sizes[W.STORE_F16_DEV] >= 2 * S * 27 * N * 2
    d, keep = lbm.make_desc(prob, W.STORE_F16_DEV)
    d.ref_state = None
    code, _, msg = _ws(lib, d)
    assert code == -1 and "ref_state" in msg
    for bad, needle in [([0.0, 1000.0, 0.3, 0.3, 0.4], "density"), ([1.0, -5.0, 0.3, 0.3, 0.4], "temperature"),
                        ([1.0, 1000.0, 0.5, 0.3, 0.4], "sum"), ([1.0, 1000.0, -0.1, 0.7, 0.4], "Y[0]")]:
        ref = np.array(bad, np.float64)
        d.ref_state = ref.ctypes.data_as(C.c_void_p)
        code, _, msg = _ws(lib, d)
        assert code == -1 and needle in msg, (bad, msg)
    d.storage = 4
    code, _, msg = _ws(lib, d)
    assert code == -1 and "storage" in msg


def test_plane_offsets_stay_32_bit(lib):
    """One padded plane times the element size must stay below 2 GiB (8 bytes for FP64
    storage, 4 otherwise): 700^3 periodic fits in FP32 and not in FP64."""
    for storage, ok in ((W.STORE_F32, True), (W.STORE_F64, False)):
        d, keep = lbm.make_desc(W.config1(), storage)
        d.nx = d.ny = d.nz = 700
        code, n, msg = _ws(lib, d)
        if ok:
            assert code == 0, msg
            assert n > 2 * 4 * 27 * 700 ** 3 * 4
        else:
            assert code == -1 and "2 GiB" in msg, msg


def test_create_rejects_bad_workspace_without_device(lib):
    d, keep = _desc(W.config1())
    h = C.c_void_p()
    assert lib.lbm_create(C.byref(d), None, 0, C.byref(h)) == -1
    assert lib.lbm_create(C.byref(d), C.c_void_p(0x1001), 1 << 30, C.byref(h)) == -4
    assert "aligned" in lib.lbm_last_error(None).decode()
    assert lib.lbm_create(C.byref(d), C.c_void_p(0x100000), 1024, C.byref(h)) == -4
    assert "needed" in lib.lbm_last_error(None).decode()
    assert not h.value


def test_null_handle_calls_fail_cleanly(lib):
    assert lib.lbm_step(None, 1, None) == -1
    assert lib.lbm_macros(None, None, None, None, None, None, None) == -1
    assert lib.lbm_init_fields(None, None, None, None, None, None) == -1
    assert lib.lbm_status_sync(None, None, None) == -1
    assert lib.lbm_diagnostics(None, 1000.0, None, None, None) == -1
    assert lib.lbm_step_graph(None, 2, None) == -1
    assert lib.lbm_flame_speeds(None, 900.0, None, None, None, None, None) == -1
    assert lib.lbm_flame_speeds_static(None, 900.0, None, None, None, None) == -1
    assert lib.lbm_adjoint_step(None, None, None, None, None) == -1
    assert lib.lbm_adjoint_macros(None, None, None, None, None, None, None, None, None) == -1
    assert lib.lbm_adjoint_init(None, None, None, None, None, None, None, None, None, None, None) == -1
    assert lib.lbm_state_save(None, None, None) == -1
    assert lib.lbm_state_load(None, None, None) == -1
    assert lib.lbm_state_size(None, None) == -1
    assert lib.lbm_set_arrhenius(None, None, None) == -1


def test_adjoint_workspace_and_scope(lib):
    """The adjoint's work buffers enlarge the workspace; descriptors outside its scope
    (16-bit storage, symmetry faces, batches, temperature-dependent transport) are
    refused with LBM_ERR_UNSUPPORTED."""
    prob = W.flame1d(nx=64, hot_cells=8)
    d, keep = lbm.make_desc(prob)
    code, plain, msg = _ws(lib, d)
    assert code == 0, msg
    d.adjoint = 1
    code, with_adj, msg = _ws(lib, d)
    assert code == 0, msg
    S, N, M = prob.M + 1, prob.N, prob.M
    assert with_adj - plain >= (2 * S * 27 + 6 * M + 9) * N * 8
    for field, value in (("storage", W.STORE_F16_DEV), ("diff_T_exp", 0.5), ("visc_T_exp", 0.5)):
        d2, keep2 = lbm.make_desc(prob, storage=value if field == "storage" else None, adjoint=True)
        setattr(d2, field, value)
        if field == "diff_T_exp":
            d2.diff_T_ref = 300.0
        if field == "visc_T_exp":
            d2.visc_T_ref = 300.0
        code, _, msg = _ws(lib, d2)
        assert code == -2, (field, code, msg)
    sym = W.sphere3d(shape=(6, 5, 4), radius=1.5, storage=W.STORE_F64)
    sym.bc = (W.BC_SYMMETRY, W.BC_OPEN, W.BC_OPEN, W.BC_OPEN, W.BC_OPEN, W.BC_OPEN)
    d3, keep3 = lbm.make_desc(sym, adjoint=True)
    code, _, msg = _ws(lib, d3)
    assert code == -2 and "symmetry" in msg
    batch = W.flame_batch(lengths=[7, 5], phis=[1.0, 1.0], hot_cells=3, storage=W.STORE_F64)
    d4, keep4 = lbm.make_desc(batch, adjoint=True)
    code, _, msg = _ws(lib, d4)
    assert code == -2 and "segments" in msg


def test_large_slab_needs_no_24_bit_products(lib):
    """A slab of more than 2^24 padded rows is a valid lattice: the step kernel forms row
    and cell indices with full 32-bit products."""
    prob = W.config1(nx=1, ny=4, nz=4)
    d, keep = lbm.make_desc(prob)
    d.ny, d.nz = 4100, 4100
    d.bc = (C.c_int32 * 6)(W.BC_PERIODIC, W.BC_PERIODIC, W.BC_OPEN, W.BC_OPEN, W.BC_OPEN, W.BC_OPEN)
    code, n, msg = _ws(lib, d)
    assert code == 0, msg


def test_segment_descriptors(lib):
    """A batch of lattices along x: lengths >= 1 summing to nx, non-periodic x faces;
    two x ghost cells per segment and row, plus the segment table.  Planes are padded to
    multiples of 64 cells: 62 cells with 2 ghosts fill one such block, with 6 ghosts two."""
    prob = W.flame_batch(lengths=[30, 1, 31], phis=[1.0, 1.0, 1.0], hot_cells=4, storage=W.STORE_F64)
    d, keep = lbm.make_desc(prob)
    assert d.n_segments == 3
    code, n3, msg = _ws(lib, d)
    assert code == 0, msg
    one = W.flame_batch(lengths=[62], phis=[1.0], hot_cells=4, storage=W.STORE_F64)
    d1, k1 = lbm.make_desc(one)
    assert d1.n_segments == 0
    code, n1, msg = _ws(lib, d1)
    assert code == 0, msg
    S = prob.M + 1
    assert n3 - n1 >= 2 * S * 27 * 64 * 8           # one more 64-cell block per plane, two copies
    for lens, needle in (([30, 1, 30], "sum"), ([30, 0, 32], "segment_lengths[1]")):
        arr = np.array(lens, np.int32)
        d.segment_lengths = arr.ctypes.data_as(C.POINTER(C.c_int32))
        code, _, msg = _ws(lib, d)
        assert code == -1 and needle in msg, msg
    d.segment_lengths = None
    code, _, msg = _ws(lib, d)
    assert code == -1 and "NULL" in msg
    d, keep = lbm.make_desc(prob)
    d.n_segments = -2
    code, _, msg = _ws(lib, d)
    assert code == -1 and "n_segments" in msg
    d, keep = lbm.make_desc(prob)
    d.bc = (C.c_int32 * 6)(0, 0, 0, 0, 0, 0)
    code, _, msg = _ws(lib, d)
    assert code == -1 and "periodic" in msg
    d, keep = lbm.make_desc(prob)
    d.n_segments = prob.nx + 1
    code, _, msg = _ws(lib, d)
    assert code == -1 and "exceeds" in msg


def test_split_batch_keeps_every_node():
    prob = W.flame_batch(n_flames=5, len_range=(3, 9), seed=11)
    parts = W.split_batch(prob)
    assert [p.nx for p in parts] == list(prob.segments)
    for k, p in enumerate(parts):
        idx = W.batch_nodes(prob, k)
        assert np.array_equal(p.T, prob.T[idx]) and np.array_equal(p.Y, prob.Y[:, idx])
        assert np.array_equal(p.rho, prob.rho[idx])
    assert np.array_equal(np.sort(np.concatenate([W.batch_nodes(prob, k) for k in range(5)])), np.arange(prob.N))


def test_diffusivity_exponent_validation(lib):
    prob = W.config1()
    for ref, ex, ok, needle in ((500.0, 1.5, True, ""), (0.0, 0.0, True, ""), (0.0, 1.0, False, "diff_T_ref"),
                                (500.0, 4.5, False, "diff_T_exp"), (500.0, float("nan"), False, "diff_T_exp")):
        prob.diff_T_ref, prob.diff_T_exp = ref, ex
        d, keep = lbm.make_desc(prob)
        code, _, msg = _ws(lib, d)
        assert (code == 0) == ok and needle in msg, (ref, ex, msg)


def test_viscosity_exponent_validation(lib):
    prob = W.config1()
    for ref, ex, ok, needle in ((300.0, 0.7, True, ""), (0.0, 0.7, False, "visc_T_ref"),
                                (300.0, -5.0, False, "visc_T_exp")):
        prob.visc_T_ref, prob.visc_T_exp = ref, ex
        d, keep = lbm.make_desc(prob)
        code, _, msg = _ws(lib, d)
        assert (code == 0) == ok and needle in msg, (ref, ex, msg)


def test_growth_exponent_fit():
    """R = a t^alpha is recovered exactly from noiseless samples."""
    t = np.array([200.0, 400.0, 800.0, 1600.0, 3200.0])
    a, alpha = lbm.growth_exponent(t, 0.37 * t ** 1.16)
    assert abs(alpha - 1.16) < 1e-12 and abs(a - 0.37) < 1e-12
    with pytest.raises(ValueError):
        lbm.growth_exponent([1.0], [2.0])
    with pytest.raises(ValueError):
        lbm.growth_exponent([1.0, 2.0], [1.0, -1.0])
    with pytest.raises(ValueError):
        lbm.growth_exponent([3.0, 3.0], [1.0, 2.0])
    # against the plain least-squares line through the logs of seeded noisy samples
    rng = np.random.default_rng(5)
    tn = np.sort(rng.uniform(100.0, 5000.0, 12))
    rn = 0.5 * tn ** 0.9 * np.exp(rng.normal(0.0, 0.05, 12))
    a, alpha = lbm.growth_exponent(tn, rn)
    ref_alpha, ref_ln_a = np.polyfit(np.log(tn), np.log(rn), 1)
    assert abs(alpha - ref_alpha) < 1e-12 and abs(np.log(a) - ref_ln_a) < 1e-12


def test_stream_copy_rejects_unaligned_arguments(lib):
    """Size and pointers must be multiples of 16 bytes; the check comes before any device
    work (the pointers here are never dereferenced)."""
    assert lib.lbm_stream_copy(C.c_void_p(4096), C.c_void_p(8192), 24, None) == -1
    assert b"16" in lib.lbm_last_error(None)
    assert lib.lbm_stream_copy(C.c_void_p(4100), C.c_void_p(8192), 32, None) == -1
    assert lib.lbm_stream_copy(None, C.c_void_p(8192), 32, None) == -1
