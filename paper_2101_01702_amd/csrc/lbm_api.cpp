// Host side of the C ABI: descriptor validation, workspace layout, table upload and
// the launch sequence of one step.  No device memory is allocated here: the
// workspace belongs to the caller.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "lbm_internal.h"

using namespace lbm;

namespace {

constexpr double R_UNIV = 8.314462618;
constexpr size_t ALIGN = 256;

thread_local std::string g_last_error;

size_t round_up(size_t v) { return (v + ALIGN - 1) / ALIGN * ALIGN; }

struct Layout {
  size_t status, tables, consts, segs, pop0, pop1, T, side_Y, side_w, side_phi, side_rho, side_u, psi, corr, diag,
      total;
  size_t corr_bytes, pop_bytes;
  // discrete adjoint (lbm_desc.adjoint != 0)
  size_t adj_P, adj_Ln, adj_fY, adj_fw, adj_lX, adj_lgY, adj_lpsi, adj_lphi, adj_lYs, adj_part, adj_nodes;
};

// sections of a state snapshot (lbm_state_save): populations, corrections, temperature
struct StateLayout {
  size_t pop, corr, T, total;
};

Geom make_geom(const lbm_desc &d) {
  Geom g{};
  g.M = d.n_species;
  g.nx = d.nx; g.ny = d.ny; g.nz = d.nz;
  const int n[3] = {d.nx, d.ny, d.nz};
  int pad[3];
  for (int a = 0; a < 3; ++a) {
    g.per[a] = d.bc[2 * a] == LBM_BC_PERIODIC ? 1 : 0;
    pad[a] = g.per[a] ? 0 : 1;
  }
  for (int k = 0; k < 6; ++k) g.bc[k] = d.bc[k];
  g.px = 0; g.py = pad[1]; g.pz = pad[2];
  g.NX = n[0]; g.NY = n[1] + 2 * pad[1]; g.NZ = n[2] + 2 * pad[2];
  g.xg = pad[0];
  g.nseg = d.n_segments > 1 ? d.n_segments : 1;
  g.vt = d.visc_T_exp != 0.0 ? 1 : 0;
  g.N = (int64_t)d.nx * d.ny * d.nz;
  g.XG = (int64_t)g.NX * g.NY * g.NZ;
  // Planes are padded to a multiple of 64 cells, so that every plane starts on a 256-byte
  // boundary; from 65536 cells on, to a multiple of 1024 cells plus 64 more, so that
  // each plane also starts 256 bytes (modulo 4 KiB) after the previous one.  Packed
  // planes started a few words off a cache line, so that each wave's stretch of a row
  // touched one more line: the 256^3 step ran 5-10% slower.
  const int64_t used = g.XG + (g.xg ? 2LL * g.nseg * g.NY * g.NZ : 0);
  g.NPAD = used >= 65536 ? (used + 1023) / 1024 * 1024 + 64 : (used + 63) / 64 * 64;
  return g;
}

Layout make_layout(const lbm_desc &d, const Geom &g) {
  const size_t st = d.storage == LBM_STORE_F64 ? 8 : (d.storage == LBM_STORE_F32 ? 4 : 2);  // populations
#ifndef LBM_SIDE_F64_FOR_F32
#define LBM_SIDE_F64_FOR_F32 0
#endif
  const size_t ct = (d.storage == LBM_STORE_F64 || (LBM_SIDE_F64_FOR_F32 && d.storage == LBM_STORE_F32))
                        ? 8 : 4;   // side channel, psi and corrections
  const size_t S = (size_t)d.n_species + 1;
  const size_t N = (size_t)g.N, M = (size_t)d.n_species;
  Layout L{};
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t at = off;
    off += round_up(bytes);
    return at;
  };
  L.status = take(64);
  L.tables = take(sizeof(Tables));
  L.consts = take(sizeof(CollideConsts));
  L.segs = take(g.nseg > 1 ? ((size_t)d.nx + g.nseg + 1) * 4 : 0);   // x -> segment, segment offsets
  L.pop0 = take(S * Q * (size_t)g.NPAD * st);
  L.pop1 = take(S * Q * (size_t)g.NPAD * st);
  L.T = take(N * 8);
  L.side_Y = take(M * N * ct);
  L.side_w = take(M * N * ct);
  L.side_phi = take(3 * N * ct);
  L.side_rho = take(N * ct);
  L.side_u = take(3 * N * ct);
  L.psi = take(3 * N * ct);
  L.corr_bytes = 6 * (size_t)g.NPAD * ct;   // deferred corrections, padded planes
  L.corr = take(L.corr_bytes);
  L.diag = take((size_t)8 * ((N + 127) / 128) * 8);   // partial sums of the diagnostics (up to 8 totals)
  L.pop_bytes = S * Q * (size_t)g.NPAD * st;
  if (d.adjoint) {
    const size_t R = (size_t)d.n_reactions;
    L.adj_P = take(S * Q * N * 8);
    L.adj_Ln = take(S * Q * N * 8);
    L.adj_fY = take(M * N * 8);
    L.adj_fw = take(M * N * 8);
    L.adj_lX = take(3 * N * 8);
    L.adj_lgY = take(3 * M * N * 8);
    L.adj_lpsi = take(3 * N * 8);
    L.adj_lphi = take(3 * N * 8);
    L.adj_lYs = take(M * N * 8);
    L.adj_part = take(3 * (R > 0 ? R : 1) * ((N + 7) / 8) * 8);
    L.adj_nodes = take(N * 8);
  }
  L.total = off;
  return L;
}

StateLayout make_state_layout(const Layout &L, const Geom &g) {
  StateLayout S{};
  S.pop = 0;
  S.corr = round_up(L.pop_bytes);
  S.T = S.corr + round_up(L.corr_bytes);
  S.total = S.T + round_up((size_t)g.N * 8);
  return S;
}

bool fail(std::string *where, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  *where = buf;
  return false;
}

bool validate(const lbm_desc *d, std::string *err) {
  if (!d) return fail(err, "descriptor is NULL");
  if (d->nx < 1 || d->ny < 1 || d->nz < 1) return fail(err, "lattice sizes must be >= 1 (got %d x %d x %d)", d->nx, d->ny, d->nz);
  const double nodes = (double)d->nx * d->ny * d->nz;
  if (nodes > 1073741824.0) return fail(err, "lattice has %.0f nodes; at most 2^30 are supported", nodes);
  for (int a = 0; a < 3; ++a) {
    for (int s = 0; s < 2; ++s) {
      const int b = d->bc[2 * a + s];
      if (b != LBM_BC_PERIODIC && b != LBM_BC_OPEN_EQ && b != LBM_BC_OPEN_EQ_U0 && b != LBM_BC_SYMMETRY)
        return fail(err, "bc[%d] = %d is not a boundary type", 2 * a + s, b);
    }
    if ((d->bc[2 * a] == LBM_BC_PERIODIC) != (d->bc[2 * a + 1] == LBM_BC_PERIODIC))
      return fail(err, "axis %d: periodic faces must come in pairs", a);
  }
  const int M = d->n_species, R = d->n_reactions;
  if (M < 2 || M > LBM_MAX_SPECIES) return fail(err, "n_species = %d outside [2, %d]", M, LBM_MAX_SPECIES);
  if (R < 0 || R > LBM_MAX_REACTIONS) return fail(err, "n_reactions = %d outside [0, %d]", R, LBM_MAX_REACTIONS);
  if (!d->molar_mass || !d->nasa7 || !d->diff_ab) return fail(err, "species arrays must not be NULL");
  if (R > 0 && (!d->nu_reac || !d->nu_prod || !d->arrhenius || !d->reversible))
    return fail(err, "reaction arrays must not be NULL when n_reactions > 0");
  for (int a = 0; a < M; ++a) {
    if (!(d->molar_mass[a] > 0.0) || !std::isfinite(d->molar_mass[a])) return fail(err, "molar_mass[%d] must be > 0", a);
    for (int k = 0; k < 7; ++k)
      if (!std::isfinite(d->nasa7[a * 7 + k])) return fail(err, "nasa7[%d][%d] is not finite", a, k);
    for (int b = 0; b < M; ++b) {
      if (a == b) continue;
      const double D = d->diff_ab[a * M + b], Dt = d->diff_ab[b * M + a];
      if (!(D > 0.0) || !std::isfinite(D)) return fail(err, "diff_ab[%d][%d] must be > 0", a, b);
      if (std::fabs(D - Dt) > 1e-12 * std::fabs(D)) return fail(err, "diff_ab is not symmetric at (%d, %d)", a, b);
    }
  }
  for (int k = 0; k < R; ++k) {
    double mass_in = 0.0, mass_out = 0.0;
    int ord_in = 0, ord_out = 0;
    for (int a = 0; a < M; ++a) {
      const int nr = d->nu_reac[k * M + a], np = d->nu_prod[k * M + a];
      if (nr < 0 || nr > 3 || np < 0 || np > 3) return fail(err, "reaction %d: stoichiometric coefficients must be in 0..3", k);
      mass_in += nr * d->molar_mass[a];
      mass_out += np * d->molar_mass[a];
      ord_in += nr;
      ord_out += np;
    }
    if (ord_in > LBM_MAX_ORDER || ord_out > LBM_MAX_ORDER)
      return fail(err, "reaction %d: more than %d molecules on one side", k, LBM_MAX_ORDER);
    if (std::fabs(mass_in - mass_out) > 1e-9 * (mass_in + mass_out))
      return fail(err, "reaction %d does not conserve mass", k);
    const double A = d->arrhenius[k * 3], b = d->arrhenius[k * 3 + 1], Ta = d->arrhenius[k * 3 + 2];
    if (!(A >= 0.0) || !std::isfinite(A) || !std::isfinite(b) || !std::isfinite(Ta))
      return fail(err, "reaction %d: Arrhenius parameters must be finite with A >= 0", k);
  }
  if (!(d->omega > 0.0 && d->omega < 2.0)) return fail(err, "omega = %g outside (0, 2)", d->omega);
  if (!(d->omega1 > 0.0 && d->omega1 < 2.0)) return fail(err, "omega1 = %g outside (0, 2)", d->omega1);
  if (!(d->kappa > 0.0) || !std::isfinite(d->kappa)) return fail(err, "kappa must be > 0");
  if (!(d->dt_phys >= 0.0) || !std::isfinite(d->dt_phys)) return fail(err, "dt_phys must be >= 0");
  if (!(d->rho_ref > 0.0) || !std::isfinite(d->rho_ref)) return fail(err, "rho_ref must be > 0");
  if (!(d->p0 > 0.0) || !std::isfinite(d->p0)) return fail(err, "p0 must be > 0");
  if (d->storage < LBM_STORE_F64 || d->storage > LBM_STORE_BF16_DEV)
    return fail(err, "storage = %d is not supported", d->storage);
  if (d->storage == LBM_STORE_F16_DEV || d->storage == LBM_STORE_BF16_DEV) {
    if (!d->ref_state) return fail(err, "the deviation formats need ref_state");
    const double *r = d->ref_state;
    if (!(r[0] > 0.0) || !std::isfinite(r[0])) return fail(err, "ref_state: density must be > 0");
    if (!(r[1] > 0.0) || !std::isfinite(r[1])) return fail(err, "ref_state: temperature must be > 0");
    double ys = 0.0;
    for (int a = 0; a < M; ++a) {
      if (!(r[2 + a] >= 0.0) || !std::isfinite(r[2 + a])) return fail(err, "ref_state: Y[%d] must be >= 0", a);
      ys += r[2 + a];
    }
    if (std::fabs(ys - 1.0) > 1e-9) return fail(err, "ref_state: mass fractions sum to %.17g, not 1", ys);
  }
  if (!std::isfinite(d->diff_T_exp) || std::fabs(d->diff_T_exp) > 4.0)
    return fail(err, "diff_T_exp = %g must be finite and within [-4, 4]", d->diff_T_exp);
  if (d->diff_T_exp != 0.0 && (!(d->diff_T_ref > 0.0) || !std::isfinite(d->diff_T_ref)))
    return fail(err, "diff_T_ref must be > 0 when diff_T_exp != 0");
  if (!std::isfinite(d->visc_T_exp) || std::fabs(d->visc_T_exp) > 4.0)
    return fail(err, "visc_T_exp = %g must be finite and within [-4, 4]", d->visc_T_exp);
  if (d->visc_T_exp != 0.0 && (!(d->visc_T_ref > 0.0) || !std::isfinite(d->visc_T_ref)))
    return fail(err, "visc_T_ref must be > 0 when visc_T_exp != 0");
  if (d->visc_T_exp != 0.0 && d->storage != LBM_STORE_F64 && d->storage != LBM_STORE_F32)
    return fail(err, "visc_T_exp != 0 needs LBM_STORE_F64 or LBM_STORE_F32 storage");
  if (d->n_segments < 0) return fail(err, "n_segments = %d must be >= 0", d->n_segments);
  if (d->n_segments > 1) {
    if (d->bc[0] == LBM_BC_PERIODIC) return fail(err, "segments along x need non-periodic x faces");
    if (d->n_segments > d->nx) return fail(err, "n_segments = %d exceeds nx = %d", d->n_segments, d->nx);
    if (!d->segment_lengths) return fail(err, "segment_lengths must not be NULL when n_segments > 1");
    int64_t sum = 0;
    for (int s = 0; s < d->n_segments; ++s) {
      if (d->segment_lengths[s] < 1) return fail(err, "segment_lengths[%d] = %d must be >= 1", s, d->segment_lengths[s]);
      sum += d->segment_lengths[s];
    }
    if (sum != d->nx) return fail(err, "segment lengths sum to %lld, not nx = %d", (long long)sum, d->nx);
  }
  {
    // the step kernel addresses one padded plane with 32-bit byte offsets
    const double xghost = d->bc[0] == LBM_BC_PERIODIC ? 0.0 : 2.0 * (d->n_segments > 1 ? d->n_segments : 1);
    const double padded = (d->nx + xghost) *
                          (d->ny + (d->bc[2] == LBM_BC_PERIODIC ? 0 : 2)) *
                          (d->nz + (d->bc[4] == LBM_BC_PERIODIC ? 0 : 2));
    const double word = d->storage == LBM_STORE_F64 ? 8.0 : 4.0;   // largest element of a plane
    if (padded * word > 2147483647.0)
      return fail(err, "lattice has %.0f padded nodes; a plane of %.0f-byte values must stay below 2 GiB",
                  padded, word);
  }
  return true;
}

// The discrete adjoint covers FP64 and FP32 storage, constant transport, and periodic,
// open and zero-velocity faces of one lattice.
bool adjoint_supported(const lbm_desc *d, std::string *err) {
  if (!d->adjoint) return true;
  if (d->storage != LBM_STORE_F64 && d->storage != LBM_STORE_F32)
    return fail(err, "the adjoint needs LBM_STORE_F64 or LBM_STORE_F32 storage");
  for (int k = 0; k < 6; ++k)
    if (d->bc[k] == LBM_BC_SYMMETRY) return fail(err, "the adjoint does not cover symmetry faces");
  if (d->n_segments > 1) return fail(err, "the adjoint does not cover batches of segments");
  if (d->diff_T_exp != 0.0 || d->visc_T_exp != 0.0)
    return fail(err, "the adjoint covers constant diffusivities, viscosity and conductivity only");
  return true;
}

void build_tables(const lbm_desc &d, Tables &t) {
  std::memset(&t, 0, sizeof(t));
  const int M = d.n_species, R = d.n_reactions;
  t.M = M;
  t.R = R;
  t.S = M + 1;
  t.open_any = (d.bc[0] != LBM_BC_PERIODIC) || (d.bc[2] != LBM_BC_PERIODIC) || (d.bc[4] != LBM_BC_PERIODIC);
  for (int a = 0; a < M; ++a) {
    const double *n = d.nasa7 + a * 7;
    const double Ra = d.kappa * R_UNIV / (d.molar_mass[a] * 1e-3);
    t.Ra[a] = Ra;
    for (int k = 0; k < 7; ++k) t.nasa[a][k] = n[k];
    // U_a = Ra (T h - T) with T h = a1 T + a2 T^2/2 + ... + a5 T^5/5 + a6
    t.ucoef[a][0] = Ra * n[5];
    t.ucoef[a][1] = Ra * (n[0] - 1.0);
    t.ucoef[a][2] = Ra * n[1] / 2.0;
    t.ucoef[a][3] = Ra * n[2] / 3.0;
    t.ucoef[a][4] = Ra * n[3] / 4.0;
    t.ucoef[a][5] = Ra * n[4] / 5.0;
    t.cvcoef[a][0] = Ra * (n[0] - 1.0);
    for (int k = 1; k < 5; ++k) t.cvcoef[a][k] = Ra * n[k];
    for (int b = 0; b < M; ++b) {
      t.invD[a][b] = (a == b) ? 0.0 : 1.0 / d.diff_ab[a * M + b];
      t.invDf[a][b] = (float)t.invD[a][b];
    }
    for (int b = a + 1; b < M; ++b) {
      const int k = a * M - a * (a + 1) / 2 + (b - a - 1);
      t.invDp[k] = 1.0 / d.diff_ab[a * M + b];
      t.invDpf[k] = (float)t.invDp[k];
    }
    t.conc_scale[a] = d.rho_ref / d.molar_mass[a];
    t.rdot_scale[a] = d.molar_mass[a] * d.dt_phys / d.rho_ref;
  }
  for (int k = 0; k < R; ++k) {
    const double A = d.arrhenius[k * 3];
    t.lnA[k] = A > 0.0 ? std::log(A) : -HUGE_VAL;
    t.bexp[k] = d.arrhenius[k * 3 + 1];
    t.Ta[k] = d.arrhenius[k * 3 + 2];
    t.rev[k] = d.reversible[k] ? 1 : 0;
    int dn = 0;
    for (int a = 0; a < M; ++a) {
      t.nu_r[k][a] = d.nu_reac[k * M + a];
      t.nu_p[k][a] = d.nu_prod[k * M + a];
      dn += t.nu_p[k][a] - t.nu_r[k][a];
      t.dnu_a[k][a] = double(t.nu_p[k][a] - t.nu_r[k][a]);
    }
    t.dnu[k] = dn;
    // species of each side repeated by their coefficient, ascending; unused slots
    // point at the constant 1 that follows the concentrations
    int nr = 0, np = 0;
    for (int a = 0; a < M; ++a) {
      for (int r = 0; r < t.nu_r[k][a]; ++r) t.reac_idx[k][nr++] = a;
      for (int r = 0; r < t.nu_p[k][a]; ++r) t.prod_idx[k][np++] = a;
    }
    t.nreac[k] = nr;
    t.nprod[k] = np;
    for (int r = nr; r < MAXORD; ++r) t.reac_idx[k][r] = M;
    for (int r = np; r < MAXORD; ++r) t.prod_idx[k][r] = M;
  }
  t.ln_c0_const = std::log(d.p0 * 1e-6 / R_UNIV);
  t.omega = d.omega;
  t.omega1 = d.omega1;
  t.dexp = d.diff_T_exp;
  t.ln_dTref = d.diff_T_exp != 0.0 ? std::log(d.diff_T_ref) : 0.0;
  t.vexp = d.visc_T_exp;
  t.ln_vTref = d.visc_T_exp != 0.0 ? std::log(d.visc_T_ref) : 0.0;
  t.c_om = 1.0 / d.omega - 0.5;
  t.c_om1 = 1.0 / d.omega1 - 0.5;
}

// Reference populations of the deviation formats: the equilibria (eqs. feq, gieq) of
// every set at the caller's reference state at rest, and per set the scale of the
// stored deviations.  The scale is 1e-3 of the set's reference magnitude (the mixture
// density for f and for every species, so that a species absent from the reference
// can still grow to the mixture density without leaving the 16-bit range).
void build_reference(const lbm_desc &d, const Tables &t, CollideConsts &kc) {
  const int M = d.n_species;
  for (int s = 0; s <= MAXM; ++s) {
    kc.sc[s] = 1.0f;
    kc.isc[s] = 1.0f;
    for (int i = 0; i < Q; ++i) kc.ref[s][i] = 0.0f;
  }
  if (d.storage != LBM_STORE_F16_DEV && d.storage != LBM_STORE_BF16_DEV) return;
  const double rho = d.ref_state[0], T = d.ref_state[1];
  const double *Y = d.ref_state + 2;
  double zeta = 0.0, U = 0.0, H = 0.0, za[MAXM];
  for (int a = 0; a < M; ++a) {
    const double *n = t.nasa[a];
    za[a] = t.Ra[a] * T;
    const double hRT = n[0] + n[1] * T / 2.0 + n[2] * T * T / 3.0 + n[3] * T * T * T / 4.0 +
                       n[4] * T * T * T * T / 5.0 + n[5] / T;
    zeta += Y[a] * za[a];
    U += Y[a] * za[a] * (hRT - 1.0);
    H += Y[a] * za[a] * hRT;
  }
  auto psi0 = [](int c, double z) { return c == 0 ? 1.0 - z : 0.5 * z; };
  auto w1 = [](int c) { return c == 0 ? 2.0 / 3.0 : 1.0 / 6.0; };
  const double theta = 1.0 / 3.0, rhoE = rho * U;
  double gmag = 0.0;
  for (int i = 0; i < Q; ++i) {
    const int cx = i % 3 - 1, cy = (i / 3) % 3 - 1, cz = i / 9 - 1;
    for (int a = 0; a < M - 1; ++a)
      kc.ref[a][i] = (float)(rho * Y[a] * psi0(cx, za[a]) * psi0(cy, za[a]) * psi0(cz, za[a]));
    kc.ref[M - 1][i] = (float)(rho * psi0(cx, zeta) * psi0(cy, zeta) * psi0(cz, zeta));
    // Grad form at rest: R^eq = H rho zeta I, so (R^eq - rho E theta I) : (c c - theta I)
    // = (H rho zeta - rho E theta)(c^2 - 3 theta)
    const double c2 = cx * cx + cy * cy + cz * cz;
    const double g = w1(cx) * w1(cy) * w1(cz) *
                     (rhoE + (H * rho * zeta - rhoE * theta) * (c2 - 3.0 * theta) / (2.0 * theta * theta));
    kc.ref[M][i] = (float)g;
    gmag += std::fabs(g);
  }
  for (int s = 0; s < M; ++s) kc.sc[s] = (float)(1e-3 * rho);
  kc.sc[M] = (float)(1e-3 * gmag);
  for (int s = 0; s <= M; ++s) kc.isc[s] = 1.0f / kc.sc[s];
}

}  // namespace

// a recorded sequence of steps: n_steps steps from a state of the given ping-pong parity
struct GraphEntry {
  int32_t n_steps;
  int parity;
  hipGraph_t graph;
  hipGraphExec_t exec;
};

struct lbm_ctx {
  lbm_desc d{};
  std::vector<double> molar_mass, nasa7, diff;
  std::vector<int32_t> nu_r, nu_p;
  std::vector<double> arrh;
  std::vector<uint8_t> rev;
  std::vector<double> ref_state;
  std::vector<int32_t> seg_len;
  Geom g{};
  Layout L{};
  Buffers b{};
  CollideConsts kc{};
  int cur = 0;
  int device = 0;
  std::string err;
  std::vector<GraphEntry> graphs;   // lbm_step_graph recordings, most recent last
  hipStream_t capture = nullptr;    // stream the recordings are captured on
  AdjBufHost adj{};                 // work buffers of the adjoint (lbm_desc.adjoint != 0)
  int64_t *adj_nodes = nullptr;
  Tables tab_host{};                // host copy of the tables (lbm_set_arrhenius)
};

namespace {

// Tile shape of the correction stencil for this lattice: each valid shape is timed over
// three launches (after one untimed) on a non-blocking stream of its own, created and
// destroyed here (so the timing neither waits for nor holds up work the caller has on
// other streams), with the stencil's inputs (and the temperature) cleared, and the
// fastest kept.  A shape that takes psi from k_psi is timed with k_psi before it.
// LBM_CORR_TILE=k in the environment picks shape k when it is valid for the lattice.
// The stencil's output (the corrections) is cleared again by lbm_init_fields.
hipError_t tune_corr_tile(lbm_ctx *h, char *ws) {
  int cand[LBM_CORR_TILES_MAX];
  const int nc = corr_tile_candidates(h->g, cand);
  h->g.corr_tile = cand[0];
  if (const char *env = std::getenv("LBM_CORR_TILE")) {
    const int k = std::atoi(env);
    for (int i = 0; i < nc; ++i)
      if (cand[i] == k) {
        h->g.corr_tile = k;
        return hipSuccess;
      }
  }
  const Layout &L = h->L;
  hipStream_t st = nullptr;
  hipError_t e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
  if (e == hipSuccess) e = launch_zero(ws + L.T, (int64_t)((L.corr - L.T) / 4), st);
  hipEvent_t ev[2] = {nullptr, nullptr};
  if (e == hipSuccess) e = hipEventCreate(&ev[0]);
  if (e == hipSuccess) e = hipEventCreate(&ev[1]);
  float best = 0.f;
  int choice = cand[0];
  for (int i = 0; i < nc && e == hipSuccess; ++i) {
    h->g.corr_tile = cand[i];
    auto once = [&] {
      hipError_t r = hipSuccess;
      if (!corr_forms_psi(cand[i])) r = launch_psi(h->g, h->b, h->d.storage, st);
      return r == hipSuccess ? launch_corr_only(h->g, h->b, h->d.storage, st) : r;
    };
    e = once();
    if (e == hipSuccess) e = hipEventRecord(ev[0], st);
    for (int r = 0; r < 3 && e == hipSuccess; ++r) e = once();
    if (e == hipSuccess) e = hipEventRecord(ev[1], st);
    if (e == hipSuccess) e = hipEventSynchronize(ev[1]);
    float t = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&t, ev[0], ev[1]);
    if (e == hipSuccess && (i == 0 || t < best)) {
      best = t;
      choice = cand[i];
    }
  }
  if (st) {
    const hipError_t es = hipStreamSynchronize(st);
    if (e == hipSuccess) e = es;
  }
  for (hipEvent_t x : ev)
    if (x) (void)hipEventDestroy(x);
  if (st) (void)hipStreamDestroy(st);
  h->g.corr_tile = choice;
  return e;
}

lbm_status hip_fail(lbm_ctx *h, hipError_t e, const char *what) {
  std::string msg = std::string(what) + ": " + hipGetErrorString(e);
  if (h) h->err = msg; else g_last_error = msg;
  return LBM_ERR_HIP;
}

lbm_status arg_fail(lbm_ctx *h, const char *msg) {
  if (h) h->err = msg; else g_last_error = msg;
  return LBM_ERR_ARG;
}

}  // namespace

extern "C" {

lbm_status lbm_workspace_size(const lbm_desc *desc, size_t *bytes) {
  std::string err;
  if (!bytes) return arg_fail(nullptr, "bytes is NULL");
  if (!validate(desc, &err)) {
    g_last_error = err;
    return LBM_ERR_ARG;
  }
  if (!adjoint_supported(desc, &err)) {
    g_last_error = err;
    return LBM_ERR_UNSUPPORTED;
  }
  const Geom g = make_geom(*desc);
  *bytes = make_layout(*desc, g).total;
  return LBM_OK;
}

lbm_status lbm_create(const lbm_desc *desc, void *d_workspace, size_t bytes, lbm_handle *out) {
  std::string err;
  if (!out) return arg_fail(nullptr, "out is NULL");
  *out = nullptr;
  if (!validate(desc, &err)) {
    g_last_error = err;
    return LBM_ERR_ARG;
  }
  if (!adjoint_supported(desc, &err)) {
    g_last_error = err;
    return LBM_ERR_UNSUPPORTED;
  }
  if (!d_workspace) return arg_fail(nullptr, "workspace is NULL");
  if (reinterpret_cast<uintptr_t>(d_workspace) % ALIGN != 0) {
    g_last_error = "workspace must be 256-byte aligned";
    return LBM_ERR_WORKSPACE;
  }
  lbm_ctx *h = new lbm_ctx();
  const int M = desc->n_species, R = desc->n_reactions;
  h->d = *desc;
  h->molar_mass.assign(desc->molar_mass, desc->molar_mass + M);
  h->nasa7.assign(desc->nasa7, desc->nasa7 + 7 * M);
  h->diff.assign(desc->diff_ab, desc->diff_ab + M * M);
  if (R > 0) {
    h->nu_r.assign(desc->nu_reac, desc->nu_reac + R * M);
    h->nu_p.assign(desc->nu_prod, desc->nu_prod + R * M);
    h->arrh.assign(desc->arrhenius, desc->arrhenius + 3 * R);
    h->rev.assign(desc->reversible, desc->reversible + R);
  }
  h->d.molar_mass = h->molar_mass.data();
  h->d.nasa7 = h->nasa7.data();
  h->d.diff_ab = h->diff.data();
  h->d.nu_reac = R ? h->nu_r.data() : nullptr;
  h->d.nu_prod = R ? h->nu_p.data() : nullptr;
  h->d.arrhenius = R ? h->arrh.data() : nullptr;
  h->d.reversible = R ? h->rev.data() : nullptr;
  if (desc->ref_state) {
    h->ref_state.assign(desc->ref_state, desc->ref_state + 2 + M);
    h->d.ref_state = h->ref_state.data();
  }
  if (desc->n_segments > 1) {
    h->seg_len.assign(desc->segment_lengths, desc->segment_lengths + desc->n_segments);
    h->d.segment_lengths = h->seg_len.data();
  } else {
    h->d.segment_lengths = nullptr;
  }
  h->g = make_geom(h->d);
  h->L = make_layout(h->d, h->g);
  if (bytes < h->L.total) {
    char buf[160];
    snprintf(buf, sizeof(buf), "workspace has %zu bytes, %zu needed", bytes, h->L.total);
    g_last_error = buf;
    delete h;
    return LBM_ERR_WORKSPACE;
  }
  hipError_t e = hipGetDevice(&h->device);
  if (e != hipSuccess) {
    lbm_status s = hip_fail(nullptr, e, "hipGetDevice");
    delete h;
    return s;
  }
  char *ws = static_cast<char *>(d_workspace);
  const Layout &L = h->L;
  Buffers &b = h->b;
  b.status = reinterpret_cast<uint32_t *>(ws + L.status);
  b.tab = reinterpret_cast<const Tables *>(ws + L.tables);
  b.pop[0] = ws + L.pop0;
  b.pop[1] = ws + L.pop1;
  b.T = reinterpret_cast<double *>(ws + L.T);
  b.side_Y = ws + L.side_Y;
  b.side_w = ws + L.side_w;
  b.side_phi = ws + L.side_phi;
  b.side_rho = ws + L.side_rho;
  b.side_u = ws + L.side_u;
  b.psi = ws + L.psi;
  b.corr = ws + L.corr;
  b.kc = reinterpret_cast<const CollideConsts *>(ws + L.consts);
  b.diag = reinterpret_cast<double *>(ws + L.diag);
  if (h->d.adjoint) {
    AdjBufHost &a = h->adj;
    a.P = reinterpret_cast<double *>(ws + L.adj_P);
    a.Ln = reinterpret_cast<double *>(ws + L.adj_Ln);
    a.T0 = nullptr;
    a.fY = reinterpret_cast<double *>(ws + L.adj_fY);
    a.fw = reinterpret_cast<double *>(ws + L.adj_fw);
    a.lX = reinterpret_cast<double *>(ws + L.adj_lX);
    a.lgY = reinterpret_cast<double *>(ws + L.adj_lgY);
    a.lpsi = reinterpret_cast<double *>(ws + L.adj_lpsi);
    a.lphi = reinterpret_cast<double *>(ws + L.adj_lphi);
    a.lYs = reinterpret_cast<double *>(ws + L.adj_lYs);
    a.part = reinterpret_cast<double *>(ws + L.adj_part);
    h->adj_nodes = reinterpret_cast<int64_t *>(ws + L.adj_nodes);
  }
  if (h->g.nseg > 1) {
    h->g.x_seg = reinterpret_cast<const int32_t *>(ws + L.segs);
    h->g.seg_off = h->g.x_seg + h->d.nx;
  }
  Tables &t = h->tab_host;
  build_tables(h->d, t);
  h->kc.omega = t.omega;
  h->kc.vexp = t.vexp;
  h->kc.ln_vTref = t.ln_vTref;
  h->kc.c_om = t.c_om;
  for (int a = 0; a < MAXM; ++a) {
    h->kc.Ra[a] = t.Ra[a];
    h->kc.Raf[a] = (float)t.Ra[a];
  }
  build_reference(h->d, t, h->kc);
  for (int k = 0; k < MAXM * (MAXM - 1) / 2; ++k) {
    h->kc.invDp[k] = t.invDp[k];
    h->kc.invDpf[k] = t.invDpf[k];
  }
  e = hipMemcpy(ws + L.tables, &t, sizeof(Tables), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(ws + L.consts, &h->kc, sizeof(CollideConsts), hipMemcpyHostToDevice);
  if (e == hipSuccess && h->g.nseg > 1) {
    std::vector<int32_t> segs((size_t)h->d.nx + h->g.nseg + 1);
    int32_t x = 0;
    for (int s = 0; s < h->g.nseg; ++s) {
      segs[(size_t)h->d.nx + s] = x;
      for (int k = 0; k < h->seg_len[s]; ++k) segs[x++] = s;
    }
    segs[(size_t)h->d.nx + h->g.nseg] = x;
    e = hipMemcpy(ws + L.segs, segs.data(), segs.size() * 4, hipMemcpyHostToDevice);
  }
  if (e == hipSuccess) {
    uint32_t zero[16] = {0};
    e = hipMemcpy(ws + L.status, zero, sizeof(zero), hipMemcpyHostToDevice);
  }
  if (e == hipSuccess && h->d.adjoint) {   // node list 0..N-1 of the population export
    std::vector<int64_t> ids((size_t)h->g.N);
    for (int64_t k = 0; k < h->g.N; ++k) ids[(size_t)k] = k;
    e = hipMemcpy(h->adj_nodes, ids.data(), ids.size() * 8, hipMemcpyHostToDevice);
  }
  if (e != hipSuccess) {
    lbm_status s = hip_fail(nullptr, e, "uploading tables");
    delete h;
    return s;
  }
  // the device address of the scratch array of lbm_flame_speeds_static, once per device
  e = flame_scratch_resolve(h->device);
  if (e != hipSuccess) {
    lbm_status s = hip_fail(nullptr, e, "resolving the scratch array of lbm_flame_speeds_static");
    delete h;
    return s;
  }
  e = tune_corr_tile(h, ws);
  if (e != hipSuccess) {
    lbm_status s = hip_fail(nullptr, e, "timing the correction tiles");
    delete h;
    return s;
  }
  *out = h;
  return LBM_OK;
}

lbm_status lbm_destroy(lbm_handle h) {
  if (h) {
    for (GraphEntry &ge : h->graphs) {
      (void)hipGraphExecDestroy(ge.exec);
      (void)hipGraphDestroy(ge.graph);
    }
    if (h->capture) (void)hipStreamDestroy(h->capture);
  }
  delete h;
  return LBM_OK;
}

lbm_status lbm_init_fields(lbm_handle h, const double *d_rho, const double *d_u, const double *d_T,
                           const double *d_Y, void *stream) {
  if (!h) return arg_fail(nullptr, "handle is NULL");
  if (!d_rho || !d_u || !d_T || !d_Y) return arg_fail(h, "init fields must not be NULL");
  hipStream_t st = static_cast<hipStream_t>(stream);
  h->cur = 0;
  hipError_t e = launch_zero(h->b.corr, (int64_t)(h->L.corr_bytes / 4), st);
  if (e == hipSuccess) e = launch_zero(h->b.status, 16, st);
  if (e == hipSuccess) e = launch_init(h->g, h->b, h->kc, h->d.storage, d_rho, d_u, d_T, d_Y, h->cur, st);
  if (e != hipSuccess) return hip_fail(h, e, "init");
  return LBM_OK;
}

static lbm_status run_steps(lbm_handle h, int32_t n_steps, hipStream_t st, float *ms) {
  hipEvent_t ev[2] = {nullptr, nullptr};
  if (ms) {
    for (int k = 0; k < LBM_NUM_KERNELS; ++k) ms[k] = 0.f;
    if (hipEventCreate(&ev[0]) != hipSuccess || hipEventCreate(&ev[1]) != hipSuccess)
      return hip_fail(h, hipErrorOutOfMemory, "hipEventCreate");
  }
  auto timed = [&](int which, auto &&launch) -> hipError_t {
    if (!ms) return launch();
    hipError_t e = hipEventRecord(ev[0], st);
    if (e != hipSuccess) return e;
    e = launch();
    if (e != hipSuccess) return e;
    e = hipEventRecord(ev[1], st);
    if (e != hipSuccess) return e;
    e = hipEventSynchronize(ev[1]);
    if (e != hipSuccess) return e;
    float t = 0.f;
    e = hipEventElapsedTime(&t, ev[0], ev[1]);
    ms[which] += t;
    return e;
  };
  const int store = h->d.storage;
  hipError_t e = hipSuccess;
  for (int s = 0; s < n_steps && e == hipSuccess; ++s) {
    const int cur = h->cur;
    e = timed(0, [&] { return launch_step(h->g, h->b, h->kc, store, cur, st); });
    if (e == hipSuccess) e = timed(3, [&] { return launch_ghost(h->g, h->b, h->kc, store, cur, st); });
    if (e == hipSuccess && !corr_forms_psi(h->g.corr_tile))
      e = timed(1, [&] { return launch_psi(h->g, h->b, store, st); });
    if (e == hipSuccess) e = timed(2, [&] { return launch_corr(h->g, h->b, store, st); });
    if (e == hipSuccess) h->cur ^= 1;
  }
  if (ms) {
    (void)hipEventDestroy(ev[0]);
    (void)hipEventDestroy(ev[1]);
  }
  if (e != hipSuccess) return hip_fail(h, e, "step");
  return LBM_OK;
}

lbm_status lbm_step(lbm_handle h, int32_t n_steps, void *stream) {
  if (!h) return arg_fail(nullptr, "handle is NULL");
  if (n_steps < 0) return arg_fail(h, "n_steps must be >= 0");
  return run_steps(h, n_steps, static_cast<hipStream_t>(stream), nullptr);
}

lbm_status lbm_step_timed(lbm_handle h, int32_t n_steps, void *stream, float *ms_out) {
  if (!h) return arg_fail(nullptr, "handle is NULL");
  if (n_steps < 0) return arg_fail(h, "n_steps must be >= 0");
  if (!ms_out) return arg_fail(h, "ms_out is NULL");
  return run_steps(h, n_steps, static_cast<hipStream_t>(stream), ms_out);
}

lbm_status lbm_step_graph(lbm_handle h, int32_t n_steps, void *stream) {
  if (!h) return arg_fail(nullptr, "handle is NULL");
  if (n_steps < 0) return arg_fail(h, "n_steps must be >= 0");
  if (n_steps == 0) return LBM_OK;
  const int parity = h->cur;
  GraphEntry *ge = nullptr;
  for (GraphEntry &g : h->graphs)
    if (g.n_steps == n_steps && g.parity == parity) ge = &g;
  if (!ge) {
    hipError_t e = hipSuccess;
    if (!h->capture) e = hipStreamCreateWithFlags(&h->capture, hipStreamNonBlocking);
    if (e != hipSuccess) return hip_fail(h, e, "hipStreamCreateWithFlags");
    e = hipStreamBeginCapture(h->capture, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return hip_fail(h, e, "hipStreamBeginCapture");
    // recording launches nothing: the ping-pong parity is restored after it
    const lbm_status st = run_steps(h, n_steps, h->capture, nullptr);
    h->cur = parity;
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(h->capture, &graph);
    if (st != LBM_OK) {
      if (graph) (void)hipGraphDestroy(graph);
      return st;
    }
    if (e != hipSuccess) return hip_fail(h, e, "hipStreamEndCapture");
    hipGraphExec_t exec = nullptr;
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
      (void)hipGraphDestroy(graph);
      return hip_fail(h, e, "hipGraphInstantiate");
    }
    if (h->graphs.size() >= 8) {   // keep the 8 most recent recordings
      (void)hipGraphExecDestroy(h->graphs.front().exec);
      (void)hipGraphDestroy(h->graphs.front().graph);
      h->graphs.erase(h->graphs.begin());
    }
    h->graphs.push_back(GraphEntry{n_steps, parity, graph, exec});
    ge = &h->graphs.back();
  }
  const hipError_t e = hipGraphLaunch(ge->exec, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(h, e, "hipGraphLaunch");
  h->cur = parity ^ (n_steps & 1);
  return LBM_OK;
}

lbm_status lbm_macros(lbm_handle h, double *d_rho, double *d_u, double *d_T, double *d_P, double *d_Y,
                      void *stream) {
  if (!h) return arg_fail(nullptr, "handle is NULL");
  hipError_t e = launch_macros(h->g, h->b, h->kc, h->d.storage, h->cur, d_rho, d_u, d_T, d_P, d_Y,
                               static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(h, e, "macros");
  return LBM_OK;
}

lbm_status lbm_populations(lbm_handle h, const int64_t *d_nodes, int64_t n_nodes, double *d_out,
                           double *d_T_out, void *stream) {
  if (!h) return arg_fail(nullptr, "handle is NULL");
  if (n_nodes < 0) return arg_fail(h, "n_nodes must be >= 0");
  if (n_nodes > 0 && (!d_nodes || !d_out)) return arg_fail(h, "node list and output must not be NULL");
  hipError_t e = launch_export(h->g, h->b, h->kc, h->d.storage, h->cur, d_nodes, n_nodes, d_out, d_T_out,
                               static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(h, e, "populations");
  return LBM_OK;
}

lbm_status lbm_diagnostics(lbm_handle h, double T_iso, double *d_hrr, double *d_totals, void *stream) {
  if (!h) return arg_fail(nullptr, "handle is NULL");
  if (!std::isfinite(T_iso)) return arg_fail(h, "T_iso must be finite");
  if (!d_hrr && !d_totals) return LBM_OK;
  hipError_t e = launch_diag(h->g, h->b, h->kc, h->d.storage, h->cur, T_iso, d_hrr, d_totals,
                             static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(h, e, "diagnostics");
  return LBM_OK;
}

lbm_status lbm_flame_speeds(lbm_handle h, double T_iso, const double *centre, double *d_work, double *d_out,
                            double *d_totals, void *stream) {
  if (!h) return arg_fail(nullptr, "handle is NULL");
  if (!std::isfinite(T_iso)) return arg_fail(h, "T_iso must be finite");
  if (!d_work) return arg_fail(h, "d_work must not be NULL");
  if (!d_out && !d_totals) return LBM_OK;
  double c[3] = {0.0, 0.0, 0.0};
  if (centre)
    for (int k = 0; k < 3; ++k) {
      if (!std::isfinite(centre[k])) return arg_fail(h, "centre must be finite");
      c[k] = centre[k];
    }
  hipError_t e = launch_flame(h->g, h->b, h->kc, h->d.storage, h->cur, T_iso, c, d_work, d_out, d_totals,
                              static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(h, e, "flame speeds");
  return LBM_OK;
}

lbm_status lbm_flame_speeds_static(lbm_handle h, double T_iso, const double *centre, double *d_out,
                                   double *d_totals, void *stream) {
  if (!h) return arg_fail(nullptr, "handle is NULL");
  if (!std::isfinite(T_iso)) return arg_fail(h, "T_iso must be finite");
  if (h->g.N > LBM_FLAME_STATIC_MAX_NODES) {
    char buf[160];
    snprintf(buf, sizeof(buf), "lattice has %lld nodes; lbm_flame_speeds_static takes at most %d",
             (long long)h->g.N, LBM_FLAME_STATIC_MAX_NODES);
    return arg_fail(h, buf);
  }
  if (!d_out && !d_totals) return LBM_OK;
  double c[3] = {0.0, 0.0, 0.0};
  if (centre)
    for (int k = 0; k < 3; ++k) {
      if (!std::isfinite(centre[k])) return arg_fail(h, "centre must be finite");
      c[k] = centre[k];
    }
  hipError_t e = launch_flame_static(h->g, h->b, h->kc, h->d.storage, h->cur, h->device, T_iso, c, d_out,
                                     d_totals, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(h, e, "flame speeds (static scratch)");
  return LBM_OK;
}

lbm_status lbm_state_size(lbm_handle h, size_t *bytes) {
  if (!h) return arg_fail(nullptr, "handle is NULL");
  if (!bytes) return arg_fail(h, "bytes is NULL");
  *bytes = make_state_layout(h->L, h->g).total;
  return LBM_OK;
}

lbm_status lbm_state_save(lbm_handle h, void *d_state, void *stream) {
  if (!h) return arg_fail(nullptr, "handle is NULL");
  if (!d_state) return arg_fail(h, "state buffer is NULL");
  if (reinterpret_cast<uintptr_t>(d_state) % ALIGN != 0) return arg_fail(h, "state buffer must be 256-byte aligned");
  const StateLayout S = make_state_layout(h->L, h->g);
  char *dst = static_cast<char *>(d_state);
  hipStream_t st = static_cast<hipStream_t>(stream);
  hipError_t e = hipMemcpyAsync(dst + S.pop, h->b.pop[h->cur], h->L.pop_bytes, hipMemcpyDeviceToDevice, st);
  if (e == hipSuccess) e = hipMemcpyAsync(dst + S.corr, h->b.corr, h->L.corr_bytes, hipMemcpyDeviceToDevice, st);
  if (e == hipSuccess) e = hipMemcpyAsync(dst + S.T, h->b.T, (size_t)h->g.N * 8, hipMemcpyDeviceToDevice, st);
  if (e != hipSuccess) return hip_fail(h, e, "state save");
  return LBM_OK;
}

lbm_status lbm_state_load(lbm_handle h, const void *d_state, void *stream) {
  if (!h) return arg_fail(nullptr, "handle is NULL");
  if (!d_state) return arg_fail(h, "state buffer is NULL");
  if (reinterpret_cast<uintptr_t>(d_state) % ALIGN != 0) return arg_fail(h, "state buffer must be 256-byte aligned");
  const StateLayout S = make_state_layout(h->L, h->g);
  const char *src = static_cast<const char *>(d_state);
  hipStream_t st = static_cast<hipStream_t>(stream);
  hipError_t e = hipMemcpyAsync(h->b.pop[h->cur], src + S.pop, h->L.pop_bytes, hipMemcpyDeviceToDevice, st);
  if (e == hipSuccess) e = hipMemcpyAsync(h->b.corr, src + S.corr, h->L.corr_bytes, hipMemcpyDeviceToDevice, st);
  if (e == hipSuccess) e = hipMemcpyAsync(h->b.T, src + S.T, (size_t)h->g.N * 8, hipMemcpyDeviceToDevice, st);
  if (e != hipSuccess) return hip_fail(h, e, "state load");
  return LBM_OK;
}

lbm_status lbm_set_arrhenius(lbm_handle h, const double *arrhenius, void *stream) {
  if (!h) return arg_fail(nullptr, "handle is NULL");
  const int R = h->d.n_reactions;
  if (R == 0) return LBM_OK;
  if (!arrhenius) return arg_fail(h, "arrhenius is NULL");
  for (int k = 0; k < R; ++k) {
    const double A = arrhenius[3 * k], b = arrhenius[3 * k + 1], Ta = arrhenius[3 * k + 2];
    if (!(A >= 0.0) || !std::isfinite(A) || !std::isfinite(b) || !std::isfinite(Ta))
      return arg_fail(h, "Arrhenius parameters must be finite with A >= 0");
  }
  hipStream_t st = static_cast<hipStream_t>(stream);
  // the host tables are the source of the copy: no copy of the previous call may be pending
  hipError_t e = hipStreamSynchronize(st);
  if (e != hipSuccess) return hip_fail(h, e, "set_arrhenius");
  h->arrh.assign(arrhenius, arrhenius + 3 * R);
  h->d.arrhenius = h->arrh.data();
  build_tables(h->d, h->tab_host);
  e = hipMemcpyAsync(const_cast<Tables *>(h->b.tab), &h->tab_host, sizeof(Tables), hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return hip_fail(h, e, "set_arrhenius");
  return LBM_OK;
}

namespace {

// export the pulled populations (FP64, node order) of a snapshot, or of the current
// state when d_state is NULL, into the adjoint work buffer; the Newton start is returned
hipError_t adjoint_forward_state(lbm_handle h, const void *d_state, hipStream_t st, const double **T0) {
  Buffers b = h->b;
  if (d_state) {
    const StateLayout S = make_state_layout(h->L, h->g);
    char *src = const_cast<char *>(static_cast<const char *>(d_state));
    b.pop[h->cur] = src + S.pop;
    b.corr = src + S.corr;
    b.T = reinterpret_cast<double *>(src + S.T);
  }
  *T0 = b.T;
  return launch_export(h->g, b, h->kc, h->d.storage, h->cur, h->adj_nodes, h->g.N, h->adj.P, nullptr, st);
}

lbm_status adjoint_ready(lbm_handle h) {
  if (!h) return arg_fail(nullptr, "handle is NULL");
  if (!h->d.adjoint) {
    h->err = "the handle was created without the adjoint work buffers (lbm_desc.adjoint = 0)";
    return LBM_ERR_UNSUPPORTED;
  }
  return LBM_OK;
}

}  // namespace

lbm_status lbm_adjoint_step(lbm_handle h, const void *d_state, void *d_adj, double *d_grad_params, void *stream) {
  lbm_status s = adjoint_ready(h);
  if (s != LBM_OK) return s;
  if (!d_adj) return arg_fail(h, "d_adj must not be NULL");
  hipStream_t st = static_cast<hipStream_t>(stream);
  const double *T0 = nullptr;
  hipError_t e = adjoint_forward_state(h, d_state, st, &T0);
  // the incoming adjoint is copied to the work buffer Ln by the first kernel of the step
  if (e == hipSuccess) {
    AdjBufHost a = h->adj;
    a.T0 = T0;
    e = launch_adjoint_step(h->g, h->b.tab, a, h->d.omega, h->d.omega1, h->d.n_reactions, static_cast<double *>(d_adj),
                            d_grad_params, st);
  }
  if (e != hipSuccess) return hip_fail(h, e, "adjoint step");
  return LBM_OK;
}

lbm_status lbm_adjoint_macros(lbm_handle h, const void *d_state, const double *d_w_rho, const double *d_w_u,
                              const double *d_w_T, const double *d_w_P, const double *d_w_Y, double *d_adj,
                              void *stream) {
  lbm_status s = adjoint_ready(h);
  if (s != LBM_OK) return s;
  if (!d_adj) return arg_fail(h, "d_adj must not be NULL");
  hipStream_t st = static_cast<hipStream_t>(stream);
  const double *T0 = nullptr;
  hipError_t e = adjoint_forward_state(h, d_state, st, &T0);
  if (e == hipSuccess)
    e = launch_adjoint_macros(h->g, h->b.tab, h->adj.P, T0, d_w_rho, d_w_u, d_w_T, d_w_P, d_w_Y, d_adj, st);
  if (e != hipSuccess) return hip_fail(h, e, "adjoint of the macroscopic fields");
  return LBM_OK;
}

lbm_status lbm_adjoint_init(lbm_handle h, const double *d_rho, const double *d_u, const double *d_T,
                            const double *d_Y, const double *d_adj, double *d_g_rho, double *d_g_u, double *d_g_T,
                            double *d_g_Y, void *stream) {
  lbm_status s = adjoint_ready(h);
  if (s != LBM_OK) return s;
  if (!d_rho || !d_u || !d_T || !d_Y || !d_adj) return arg_fail(h, "fields and d_adj must not be NULL");
  hipError_t e = launch_adjoint_init(h->g, h->b.tab, d_rho, d_u, d_T, d_Y, d_adj, d_g_rho, d_g_u, d_g_T, d_g_Y,
                                     static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(h, e, "adjoint of the initial state");
  return LBM_OK;
}

lbm_status lbm_status_sync(lbm_handle h, void *stream, uint32_t *anomaly_bits) {
  if (!h) return arg_fail(nullptr, "handle is NULL");
  hipStream_t st = static_cast<hipStream_t>(stream);
  uint32_t bits = 0;
  hipError_t e = hipMemcpyAsync(&bits, h->b.status, sizeof(bits), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e == hipSuccess) e = launch_zero(h->b.status, 1, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return hip_fail(h, e, "status");
  if (anomaly_bits) *anomaly_bits = bits;
  if (bits) {
    h->err = "device anomaly bits set";
    return LBM_ERR_DEVICE_ANOMALY;
  }
  return LBM_OK;
}

lbm_status lbm_stream_copy(const void *d_src, void *d_dst, size_t bytes, void *stream) {
  if (!d_src || !d_dst) return arg_fail(nullptr, "buffers must not be NULL");
  if (bytes % 16 != 0 || reinterpret_cast<uintptr_t>(d_src) % 16 != 0 || reinterpret_cast<uintptr_t>(d_dst) % 16 != 0)
    return arg_fail(nullptr, "buffers and size must be multiples of 16 bytes");
  const hipError_t e = launch_stream_copy(d_src, d_dst, (int64_t)bytes, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(nullptr, e, "stream copy");
  return LBM_OK;
}

lbm_status lbm_growth_fit(const double *t, const double *R, int64_t n, double *a, double *alpha) {
  if (!t || !R || !a || !alpha) return arg_fail(nullptr, "pointers must not be NULL");
  if (n < 2) return arg_fail(nullptr, "the fit needs at least two samples");
  // centred sums: slope = sum (x - mx)(y - my) / sum (x - mx)^2, x = ln t, y = ln R
  double mx = 0.0, my = 0.0;
  for (int64_t k = 0; k < n; ++k) {
    if (!(t[k] > 0.0) || !(R[k] > 0.0) || !std::isfinite(t[k]) || !std::isfinite(R[k]))
      return arg_fail(nullptr, "times and radii must be positive and finite");
    mx += std::log(t[k]);
    my += std::log(R[k]);
  }
  mx /= (double)n;
  my /= (double)n;
  double sxx = 0.0, sxy = 0.0;
  for (int64_t k = 0; k < n; ++k) {
    const double dx = std::log(t[k]) - mx, dy = std::log(R[k]) - my;
    sxx += dx * dx;
    sxy += dx * dy;
  }
  if (!(sxx > 0.0)) return arg_fail(nullptr, "the sample times must not all be equal");
  *alpha = sxy / sxx;
  *a = std::exp(my - *alpha * mx);
  return LBM_OK;
}

const char *lbm_last_error(lbm_handle h) { return h ? h->err.c_str() : g_last_error.c_str(); }

}  // extern "C"
