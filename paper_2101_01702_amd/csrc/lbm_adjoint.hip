// Discrete adjoint of the reactive-mixture lattice Boltzmann step (gfx950).
//
// One forward step maps the pre-collision populations F_n (pulled, with the deferred
// corrections) to F_{n+1}:
//   moments (eqs. Pa, sumfDotc, g0momTotalEnergy, strongest), temperature by Newton on
//   the energy (eq. temperature), thermo (eqs. specHa, Umix), mass-action rates (Sec. 4),
//   Stefan-Maxwell relaxation and diffusion velocities (eqs. tauab, transform1, fStar),
//   the non-local fields phi -> psi -> X and grad Y (eqs. Xalpha, corrFourier), the
//   collisions of the species (eq. finalNumericalEquations), of f (eq. f) and of g
//   (eq. g with eqs. gieq, geq1mom, geq2mom, gstareq1mom, qdiff, corrFourier), the
//   equilibrium ghosts of the open faces (Sec. 5.1) and pull streaming.
// The kernels here apply the transpose of its Jacobian at F_n to an adjoint lambda_{n+1}
// and give lambda_n and the step's contribution to the gradient with respect to the
// Arrhenius parameters (ln A_k, b_k, Ta_k).  Everything is FP64.  Each derivative is
// written by hand from the forward expression it reverses; the temperature enters
// through the implicit function of the Newton equation, dT = (de - sum_a U_a dY_a) / C_v.
//
// Layout of the work: a node's 27 directions sit on 27 lanes of a 32-lane group (8 nodes
// per 256-thread workgroup).  Each lane reverses its direction's part of the collision
// (the equilibria, the inter-species term and the energy population of that direction)
// and the per-node sums over directions are group sums.  The node-level chain
// (temperature, thermo, rates, the Stefan-Maxwell solve) works on a record of the node in
// LDS, spread over the group: species on lanes 0..M-1, reactions on lanes 0..R-1, the
// scalar parts on the first lane.  The stencils of X and grad Y are reversed as gathers
// with the transposed stencil.
#include "lbm_internal.h"

namespace lbm {

namespace {

constexpr int NPB = 8;              // nodes per workgroup of the per-direction kernels
constexpr int GL = 32;              // lanes per node
constexpr int ADJ_BLOCK = NPB * GL;

__host__ __device__ constexpr int acx(int i) { return i % 3 - 1; }
__host__ __device__ constexpr int acy(int i) { return (i / 3) % 3 - 1; }
__host__ __device__ constexpr int acz(int i) { return i / 9 - 1; }
__host__ __device__ constexpr double aw1(int c) { return c == 0 ? 2.0 / 3.0 : 1.0 / 6.0; }
__host__ __device__ constexpr double awgt(int i) { return aw1(acx(i)) * aw1(acy(i)) * aw1(acz(i)); }

// ---- product form Psi_c(u, zeta) (eq. phis) and its derivatives ----------------------
__device__ __forceinline__ void psi1(int c, double u, double z, double &v, double &du, double &dz) {
  if (c == 0) {
    v = 1.0 - u * u - z;
    du = -2.0 * u;
    dz = -1.0;
  } else {
    v = 0.5 * (c * u + u * u + z);
    du = 0.5 * (c + 2.0 * u);
    dz = 0.5;
  }
}

// Phi_i(u, zeta) = prod_alpha Psi_{c_alpha}(u_alpha, zeta) with d/du and d/dzeta
struct PhiD {
  double v, du[3], dz;
};
__device__ __forceinline__ PhiD phi_d(int i, const double u[3], double z) {
  double px, pxu, pxz, py, pyu, pyz, pz, pzu, pzz;
  psi1(acx(i), u[0], z, px, pxu, pxz);
  psi1(acy(i), u[1], z, py, pyu, pyz);
  psi1(acz(i), u[2], z, pz, pzu, pzz);
  PhiD r;
  r.v = px * py * pz;
  r.du[0] = pxu * py * pz;
  r.du[1] = px * pyu * pz;
  r.du[2] = px * py * pzu;
  r.dz = pxz * py * pz + px * pyz * pz + px * py * pzz;
  return r;
}

// ---- NASA-7 (eq. specHa): h/RT, s/R, cp/R ------------------------------------------------
template <class P>
__device__ __forceinline__ double a_hRT(P a, double T) {
  return a[0] + T * (a[1] * 0.5 + T * (a[2] * (1.0 / 3.0) + T * (a[3] * 0.25 + T * (a[4] * 0.2)))) + a[5] / T;
}
template <class P>
__device__ __forceinline__ double a_sR(P a, double T, double lnT) {
  return a[0] * lnT + T * (a[1] + T * (a[2] * 0.5 + T * (a[3] * (1.0 / 3.0) + T * (a[4] * 0.25)))) + a[6];
}
template <class P>
__device__ __forceinline__ double a_cpR(P a, double T) {
  return a[0] + T * (a[1] + T * (a[2] + T * (a[3] + T * a[4])));
}

template <class TB>
__device__ __forceinline__ double invD(TB &tb, int M, int a, int b) {
  const int lo = a < b ? a : b, hi = a < b ? b : a;
  return tb.invDp[lo * M - lo * (lo + 1) / 2 + (hi - lo - 1)];
}

// Sum over the 32 lanes of a node group; every lane gets the same total, bit for bit.
// Within each row of 16 lanes by DPP moves that pair lanes symmetrically (swap
// neighbours, swap pairs, mirror each half row, mirror the row: each lane adds the value
// of a partner that adds its value back, so both form the same sum), then across the two
// rows by a swizzle that exchanges lanes l and l ^ 16.  The moves act on the two 32-bit
// halves of the double.
template <int CTRL>
__device__ __forceinline__ double dpp_mov(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(__double_as_longlong(v) & 0xffffffff), CTRL, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(__double_as_longlong(v) >> 32), CTRL, 0xf, 0xf, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
__device__ __forceinline__ double swz_xor16(double v) {
  const int lo = __builtin_amdgcn_ds_swizzle((int)(__double_as_longlong(v) & 0xffffffff), 0x401f);
  const int hi = __builtin_amdgcn_ds_swizzle((int)(__double_as_longlong(v) >> 32), 0x401f);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
__device__ __forceinline__ double gsum(double v) {
  v += dpp_mov<0xb1>(v);    // quad_perm [1, 0, 3, 2]
  v += dpp_mov<0x4e>(v);    // quad_perm [2, 3, 0, 1]
  v += dpp_mov<0x141>(v);   // row_half_mirror
  v += dpp_mov<0x140>(v);   // row_mirror
  v += swz_xor16(v);        // bit-mask swizzle: and 0x1f, xor 0x10
  return v;
}

// LDS-qualified types for the node-level chains.  Those are out-of-line functions, where a
// plain pointer argument has no known address space and every access through it would
// take the flat path; the record and the workgroup's copy of the tables are passed as
// LDS pointers instead.
typedef __attribute__((address_space(3))) double lds_double;
typedef const __attribute__((address_space(3))) Tables lds_tables;

// the workgroup's copy of the tables (sizeof(Tables) is a multiple of 8)
__device__ __forceinline__ void tables_to_lds(const Tables *src, Tables *dst) {
  const double *s = reinterpret_cast<const double *>(src);
  double *d = reinterpret_cast<double *>(dst);
  for (int k = threadIdx.x; k < (int)(sizeof(Tables) / 8); k += blockDim.x) d[k] = s[k];
}

// ---- record of one node in LDS ---------------------------------------------------------
// Forward quantities of the node (written by the group's first lane), then the reduced
// adjoints of the per-direction terms, the adjoints of the moments, and the working
// arrays of the node-level chains (held in LDS rather than registers: that chain runs on
// one lane of the group).
template <int M>
struct Rec {
  // forward scalars
  static constexpr int RHO = 0, U = 1, RHOE = 4, QM = 5, PT = 8 /* 3x3 */, T = 17, LNT = 18, ZETA = 19, PP = 20,
                       H = 21, CV = 22, ANOM = 23;
  // forward per species, SPW words each
  enum { S_RS, S_Y, S_ZA, S_HA, S_UA, S_HRT, S_CPR, S_C, S_GIB, S_RDOT, S_BETA, S_T, S_CA, S_SA, S_JA,
         S_RA = S_JA + 3, S_DU = S_RA + 3, S_TINY = S_DU + 3, S_GY, SPW = S_GY + 3 };
  static constexpr int SP = 24;
  static constexpr int sp(int a, int f) { return SP + a * SPW + f; }
  static constexpr int K = SP + M * SPW;       // K_ab, full M x M
  static constexpr int LU = K + M * M;         // elimination factors of the Stefan-Maxwell matrix
  static constexpr int RX = LU + M * M;        // per reaction: forward and reverse rate
  // reduced adjoints of the per-direction terms
  static constexpr int L0 = RX + 2 * MAXR;
  static constexpr int L_RHOF = L0, L_U = L0 + 1, L_ZETA = L0 + 4, L_A0 = L0 + 5, L_A1 = L0 + 6, L_B = L0 + 9 /* 3x3 */,
                       L_CG = L0 + 18, L_A0G = L0 + 21 /* [2] */, L_A1G = L0 + 23 /* [2][3] */, L_BG = L0 + 29 /* [2][9] */,
                       L_END = L0 + 47;
  enum { A_RHOB, A_ZETAB, A_DU, A_C = A_DU + 3, A_S, A_BETA, APW };
  static constexpr int AS = L_END;
  static constexpr int asp(int a, int f) { return AS + a * APW + f; }
  static constexpr int LK = AS + M * APW;      // adjoint of K_ab (both orders), full M x M
  // adjoints of the moments (output of the node-level chain)
  static constexpr int MO = LK + M * M;
  static constexpr int M_RHO = MO, M_J = MO + 1, M_P = MO + 4 /* 3x3 */, M_RHOE = MO + 13, M_Q = MO + 14,
                       M_RA = MO + 17 /* [M] */, M_JA = MO + 17 + M /* [M][3] */;
  // working arrays of the node-level reverse chain
  enum { W_LY, W_LZA, W_LHA, W_LRS, W_LC, W_LT, W_LRDOT, W_LJA, W_MU = W_LJA + 3, WPW = W_MU + 3 };
  static constexpr int WK = M_JA + 3 * M;
  static constexpr int wk(int a, int f) { return WK + a * WPW + f; }
  // scalar adjoints carried from the first part of the reverse chain to the last
  enum { C_LRHO, C_LU, C_LZETA = C_LU + 3, C_LH, C_LPT, C_LRHOE, C_LQ, C_LPM = C_LQ + 3, C_LUMIX = C_LPM + 9, C_LT,
         C_LA1, CPW = C_LA1 + 3 };
  static constexpr int SC = WK + M * WPW;
  static constexpr int WORDS = SC + CPW;
};

// ---- moments of the pulled populations on a lane's direction ---------------------------
// lane i holds F[s][i]; the moments are summed over the group
template <int M>
struct Mom {
  double rho, j[3], P[3][3], rhoE, q[3], ra[M - 1], ja[M - 1][3];
};

template <int M>
__device__ __forceinline__ void group_moments(int i, bool valid, const double *f, Mom<M> &m) {
  const double c[3] = {double(acx(i)), double(acy(i)), double(acz(i))};
  const double ff = valid ? f[M - 1] : 0.0, gg = valid ? f[M] : 0.0;
  m.rho = gsum(ff);
  m.rhoE = gsum(gg);
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    m.j[d] = gsum(c[d] * ff);
    m.q[d] = gsum(c[d] * gg);
  }
#pragma unroll
  for (int d = 0; d < 3; ++d)
#pragma unroll
    for (int e = d; e < 3; ++e) {
      m.P[d][e] = gsum(c[d] * c[e] * ff);
      m.P[e][d] = m.P[d][e];
    }
#pragma unroll
  for (int a = 0; a < M - 1; ++a) {
    const double fa = valid ? f[a] : 0.0;
    m.ra[a] = gsum(fa);
#pragma unroll
    for (int d = 0; d < 3; ++d) m.ja[a][d] = gsum(c[d] * fa);
  }
}

// ---- node-level forward ---------------------------------------------------------------------
// Called by every lane of a node's group (ok: the group holds a node), which all hold the
// node's moments: lane a < M takes species a, sums over species are group sums, and the
// Newton iteration for the temperature runs on every lane alike.  Macros (O1),
// temperature (O2) and thermo into the record (node_forward); the production rates (O3)
// one reaction per lane (fwd_rate) and one species per lane (fwd_rdot); Stefan-Maxwell
// (O4) and the collision coefficients (fwd_sm).
template <int M>
__device__ __noinline__ void node_forward(lds_tables &tb, const Mom<M> &m, double T0, lds_double *r, int lane,
                                         bool ok, bool rates_and_sm) {
  using RC = Rec<M>;
  const double rho = m.rho, inv_rho = 1.0 / rho;
  double u[3];
  for (int d = 0; d < 3; ++d) u[d] = m.j[d] * inv_rho;
  if (ok && lane == 0) {
    r[RC::RHO] = rho;
    r[RC::RHOE] = m.rhoE;
    for (int d = 0; d < 3; ++d) {
      r[RC::U + d] = u[d];
      r[RC::QM + d] = m.q[d];
      for (int e = 0; e < 3; ++e) r[RC::PT + 3 * d + e] = m.P[d][e];
    }
  }
  // species densities and momenta; the last species is slaved (eq. strongest)
  double rsum = 0.0, jsum[3] = {0.0, 0.0, 0.0};
  for (int a = 0; a < M - 1; ++a) {
    rsum += m.ra[a];
    for (int d = 0; d < 3; ++d) jsum[d] += m.ja[a][d];
  }
  const int a = lane;
  const bool sp = a < M;
  double Y = 0.0;
  if (sp) {
    const double rs = a < M - 1 ? m.ra[a] : rho - rsum;
    double ja[3];
    for (int d = 0; d < 3; ++d) ja[d] = a < M - 1 ? m.ja[a][d] : m.j[d] - jsum[d];
    Y = rs * inv_rho;
    const bool tiny = fabs(rs) < 1e-300;
    if (ok) {
      r[RC::sp(a, RC::S_RS)] = rs;
      r[RC::sp(a, RC::S_Y)] = Y;
      r[RC::sp(a, RC::S_TINY)] = tiny ? 1.0 : 0.0;
      for (int d = 0; d < 3; ++d) {
        r[RC::sp(a, RC::S_JA + d)] = ja[d];
        r[RC::sp(a, RC::S_RA + d)] = tiny ? 0.0 : ja[d] / rs - u[d];
      }
    }
  }
  uint32_t anom = 0;
  if (!(rho > 0.0) || !(rho - rsum > 0.0)) anom |= LBM_ANOM_NEG_DENSITY;
  // temperature: sum_a Y_a U_a(T) = rhoE / rho - u^2 / 2 (Newton from the stored value)
  const double usq = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
  const double e = m.rhoE * inv_rho - 0.5 * usq;
  double ec[6], dc[5];
  for (int k = 0; k < 6; ++k) ec[k] = gsum(sp ? Y * tb.ucoef[a][k] : 0.0);
  for (int k = 0; k < 5; ++k) dc[k] = gsum(sp ? Y * tb.cvcoef[a][k] : 0.0);
  double T = T0;
  int conv = 0;
  for (int it = 0; it < 50; ++it) {
    const double ev = ec[0] + T * (ec[1] + T * (ec[2] + T * (ec[3] + T * (ec[4] + T * ec[5])))) - e;
    const double dv = dc[0] + T * (dc[1] + T * (dc[2] + T * (dc[3] + T * dc[4])));
    const double dT = -ev / dv;
    T += dT;
    if (fabs(dT) <= 1e-12 * fabs(T)) {
      conv = 1;
      break;
    }
  }
  if (!conv) anom |= LBM_ANOM_NEWTON;
  if (!isfinite(T) || !isfinite(rho)) anom |= LBM_ANOM_NONFINITE;
  const double lnT = log(T);
  double pz = 0.0, pH = 0.0, pC = 0.0;
  if (sp) {
    const double za = tb.Ra[a] * T, h = a_hRT(tb.nasa[a], T), cp = a_cpR(tb.nasa[a], T);
    if (ok) {
      r[RC::sp(a, RC::S_ZA)] = za;
      r[RC::sp(a, RC::S_HRT)] = h;
      r[RC::sp(a, RC::S_CPR)] = cp;
      r[RC::sp(a, RC::S_HA)] = za * h;
      r[RC::sp(a, RC::S_UA)] = za * (h - 1.0);
      // concentrations and Gibbs functions for the production rates (Sec. 4)
      if (rates_and_sm) {
        r[RC::sp(a, RC::S_C)] = r[RC::sp(a, RC::S_RS)] * tb.conc_scale[a];
        r[RC::sp(a, RC::S_GIB)] = h - a_sR(tb.nasa[a], T, lnT);
      }
    }
    pz = Y * za;
    pH = Y * za * h;
    pC = Y * tb.Ra[a] * (cp - 1.0);
  }
  const double zeta = gsum(pz), H = gsum(pH), Cv = gsum(pC);
  if (ok && lane == 0) {
    r[RC::T] = T;
    r[RC::LNT] = lnT;
    r[RC::ZETA] = zeta;
    r[RC::PP] = rho * zeta;
    r[RC::H] = H;
    r[RC::CV] = Cv;
    r[RC::ANOM] = double(anom);
  }
}

// one reaction's forward and reverse rates (mass action, Sec. 4) into the record
template <int M>
__device__ __forceinline__ void fwd_rate(lds_tables &tb, lds_double *r, int k) {
  using RC = Rec<M>;
  const double lnT = r[RC::LNT], invT = 1.0 / r[RC::T];
  // species index M of a padded reaction side stands for a factor 1
  auto conc = [&](int idx) -> double { return idx < M ? r[RC::sp(idx, RC::S_C)] : 1.0; };
  const double lnkf = tb.lnA[k] + tb.bexp[k] * lnT - tb.Ta[k] * invT;
  double fwd = exp(lnkf);
  for (int q = 0; q < tb.nreac[k]; ++q) fwd *= conc(tb.reac_idx[k][q]);
  double rev = 0.0;
  if (tb.rev[k]) {
    double dG = 0.0;
    for (int a = 0; a < M; ++a) dG += tb.dnu_a[k][a] * r[RC::sp(a, RC::S_GIB)];
    rev = exp(lnkf + dG - tb.dnu[k] * (tb.ln_c0_const - lnT));
    for (int q = 0; q < tb.nprod[k]; ++q) rev *= conc(tb.prod_idx[k][q]);
  }
  r[RC::RX + 2 * k] = fwd;
  r[RC::RX + 2 * k + 1] = rev;
}

// one species' production rate from the reactions' rates in the record
template <int M>
__device__ __forceinline__ void fwd_rdot(lds_tables &tb, lds_double *r, int a) {
  using RC = Rec<M>;
  double s = 0.0;
  for (int k = 0; k < tb.R; ++k) s += tb.dnu_a[k][a] * (r[RC::RX + 2 * k] - r[RC::RX + 2 * k + 1]);
  r[RC::sp(a, RC::S_RDOT)] = s * tb.rdot_scale[a];
}

// Stefan-Maxwell relaxation (eqs. tauab, transform1) and the collision coefficients of
// the species, by all lanes of the group (workgroup barriers between the stages):
// K_ab = zeta_a zeta_b / (zeta D_ab), t_a = sum_b Y_b K_ab, beta_a = t_a / (2 + t_a),
// A_aa = 1 + t_a / 2, A_ab = -K_ab Y_b / 2 (row a on lane a); the elimination one pivot
// at a time (row q on lane q); the three right-hand sides on lanes 0..2.
template <int M>
__device__ __noinline__ void fwd_sm(lds_tables &tb, lds_double *r, int lane, bool ok) {
  using RC = Rec<M>;
  const int a = lane;
  if (ok && a < M) {
    const double inv_zeta = 1.0 / r[RC::ZETA], za = r[RC::sp(a, RC::S_ZA)];
    double t = 0.0;
    for (int b = 0; b < M; ++b) {
      const double K = b == a ? 0.0 : za * r[RC::sp(b, RC::S_ZA)] * invD(tb, M, a, b) * inv_zeta;
      r[RC::K + a * M + b] = K;
      if (b != a) t += r[RC::sp(b, RC::S_Y)] * K;
    }
    r[RC::sp(a, RC::S_T)] = t;
    r[RC::sp(a, RC::S_BETA)] = t / (2.0 + t);
    for (int b = 0; b < M; ++b)
      r[RC::LU + a * M + b] = (a == b) ? 1.0 + 0.5 * t : -0.5 * r[RC::K + a * M + b] * r[RC::sp(b, RC::S_Y)];
  }
  __syncthreads();
  // Gaussian elimination without pivoting (strictly row-diagonally dominant): the
  // multipliers below the diagonal, U on and above it
  for (int k = 0; k < M; ++k) {
    if (ok && a > k && a < M) {
      const double l = r[RC::LU + a * M + k] / r[RC::LU + k * M + k];
      r[RC::LU + a * M + k] = l;
      for (int cc = k + 1; cc < M; ++cc) r[RC::LU + a * M + cc] -= l * r[RC::LU + k * M + cc];
    }
    __syncthreads();
  }
  // du: L z = r_a - u (z in the du slots), then U du = z in place
  if (ok && lane < 3) {
    const int d = lane;
    for (int q = 0; q < M; ++q) {
      double v = r[RC::sp(q, RC::S_RA + d)];
      for (int b = 0; b < q; ++b) v -= r[RC::LU + q * M + b] * r[RC::sp(b, RC::S_DU + d)];
      r[RC::sp(q, RC::S_DU + d)] = v;
    }
    for (int q = M - 1; q >= 0; --q) {
      double v = r[RC::sp(q, RC::S_DU + d)];
      for (int b = q + 1; b < M; ++b) v -= r[RC::LU + q * M + b] * r[RC::sp(b, RC::S_DU + d)];
      r[RC::sp(q, RC::S_DU + d)] = v / r[RC::LU + q * M + q];
    }
  }
  // collision coefficients of the stored species: c_a = 2 beta_a rho_a + rho_dot_a (the
  // equilibrium and source share Phi(u, zeta_a)), s_a = (beta_a - 1) Y_a (eq. fStar)
  if (ok && a < M - 1) {
    const double beta = r[RC::sp(a, RC::S_BETA)];
    r[RC::sp(a, RC::S_CA)] = 2.0 * beta * r[RC::sp(a, RC::S_RS)] + r[RC::sp(a, RC::S_RDOT)];
    r[RC::sp(a, RC::S_SA)] = (beta - 1.0) * r[RC::sp(a, RC::S_Y)];
  }
}

// ---- the node-level adjoint chain ------------------------------------------------------------
// Inputs in the record: the reduced adjoints of the per-direction terms, plus direct
// adjoints of node quantities given by the caller (lT, lY, lP, lrho, lu, lphi).
// Output: the adjoints of the moments in the record; the Arrhenius gradient in pg[3R].
// Called by every lane of the node's group (ok: the group holds a node).  rev_a: the
// node's scalar adjoints (the Grad forms of g and of its ghosts) on the first lane,
// then the per-species terms with lane a on species a (the collision's coefficients,
// the enthalpy flux, the Stefan-Maxwell solve); the production rates one reaction per
// lane (rev_rate); rev_b on the first lane (thermo, temperature, the moments).  The
// scalar adjoints are carried in the record; the lanes' parts of them are group sums.

// the scalar part of rev_a (first lane)
template <int M>
__device__ __noinline__ void rev_scalars(lds_tables &tb, double omega, double omega1, lds_double *r, bool collision,
                                         double lT, double lP, double lrho_in, const double *lu_in) {
  using RC = Rec<M>;
  const double rho = r[RC::RHO], P = r[RC::PP];
  double u[3];
  for (int d = 0; d < 3; ++d) u[d] = r[RC::U + d];
  double lrho = lrho_in, lu[3], lzeta = 0.0, lH = 0.0, lPt = lP, lrhoE = 0.0, lq[3] = {0.0, 0.0, 0.0};
  double lPm[3][3], lU = 0.0, lA1[3] = {0.0, 0.0, 0.0};
  for (int d = 0; d < 3; ++d) {
    lu[d] = lu_in ? lu_in[d] : 0.0;
    for (int e = 0; e < 3; ++e) lPm[d][e] = 0.0;
  }
  auto Y = [&](int a) -> double { return r[RC::sp(a, RC::S_Y)]; };

  // The Grad forms: R = h2 P^eq + P v v, P^eq = P I + rho v v, q^eq = h2 rho v, h2 = H + v^2/2
  // at the velocity v (u, or 0 for a zero-velocity ghost, which has no u part).  Adds the
  // adjoints of (rho, u, P, H) from those of (q^eq, R).
  auto grad_eq_vjp = [&](const double *v, bool v_is_u, const double *lqe, const double (*lR)[3]) {
    const double vsq = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
    const double h2 = r[RC::H] + 0.5 * vsq;
    double lh2 = 0.0;
    for (int d = 0; d < 3; ++d) {
      lh2 += lqe[d] * rho * v[d];
      lrho += lqe[d] * h2 * v[d];
      if (v_is_u) lu[d] += lqe[d] * h2 * rho;
    }
    for (int d = 0; d < 3; ++d)
      for (int e = 0; e < 3; ++e) {
        const double Peq = (d == e ? P : 0.0) + rho * v[d] * v[e];
        lh2 += lR[d][e] * Peq;
        lrho += lR[d][e] * h2 * v[d] * v[e];
        lPt += lR[d][e] * ((d == e ? h2 : 0.0) + v[d] * v[e]);
        if (v_is_u) {
          const double f = lR[d][e] * (h2 * rho + P);
          lu[d] += f * v[e];
          lu[e] += f * v[d];
        }
      }
    lH += lh2;
    if (v_is_u)
      for (int d = 0; d < 3; ++d) lu[d] += lh2 * v[d];
  };

  // --- per-direction terms (reduced) ---
  lrho += r[RC::L_RHOF];
  for (int d = 0; d < 3; ++d) lu[d] += r[RC::L_U + d];
  lzeta += r[RC::L_ZETA];
  if (collision) {
    const double om = omega, om1 = omega1;
    // g: A0 = om (2.5 rhoE - 1.5 tr R), B_dd = om (4.5 R_dd - 1.5 rhoE), B_de = 4.5 om R_de,
    //    A1 = 3 om q^eq + 3 (om - om1)(q - u.(P - P^eq) - q^eq) + 3 om1 rho sum_a H_a Y_a du_a
    const double lA0 = r[RC::L_A0];
    double lR[3][3], lqe[3];
    lrhoE += om * 2.5 * lA0;
    for (int d = 0; d < 3; ++d)
      for (int e = 0; e < 3; ++e) {
        const double lB = r[RC::L_B + 3 * d + e];
        lR[d][e] = 4.5 * om * lB + (d == e ? -1.5 * om * lA0 : 0.0);
        if (d == e) lrhoE -= 1.5 * om * lB;
      }
    const double kap = 3.0 * (om - om1);
    for (int d = 0; d < 3; ++d) {
      lA1[d] = r[RC::L_A1 + d];
      lqe[d] = 3.0 * om1 * lA1[d];
      lq[d] += kap * lA1[d];
    }
    // -kap u_c (P_cd - P^eq_cd) with P^eq_cd = P delta_cd + rho u_c u_d
    for (int d = 0; d < 3; ++d)
      for (int cc = 0; cc < 3; ++cc) {
        const double w = -kap * lA1[d];
        const double Peq = (cc == d ? P : 0.0) + rho * u[cc] * u[d];
        lu[cc] += w * (r[RC::PT + 3 * cc + d] - Peq);
        lPm[cc][d] += w * u[cc];
        if (cc == d) lPt -= w * u[cc];
        lrho -= w * u[cc] * u[cc] * u[d];
        lu[cc] -= w * u[cc] * rho * u[d];
        lu[d] -= w * u[cc] * rho * u[cc];
      }
    grad_eq_vjp(u, true, lqe, lR);
  }
  // ghost equilibria of g (Grad form at rhoE_g = rho (U + v^2/2), no relaxation factor)
  for (int z = 0; z < 2; ++z) {
    const double lA0 = r[RC::L_A0G + z];
    double lR[3][3], lqe[3];
    double lrhoEg = 2.5 * lA0;
    for (int d = 0; d < 3; ++d) {
      lqe[d] = 3.0 * r[RC::L_A1G + 3 * z + d];
      for (int e = 0; e < 3; ++e) {
        const double lB = r[RC::L_BG + 9 * z + 3 * d + e];
        lR[d][e] = 4.5 * lB + (d == e ? -1.5 * lA0 : 0.0);
        if (d == e) lrhoEg -= 1.5 * lB;
      }
    }
    const double zero[3] = {0.0, 0.0, 0.0};
    const double *v = z ? zero : u;
    const double vsq = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
    double Umix = 0.0;
    for (int a = 0; a < M; ++a) Umix += Y(a) * r[RC::sp(a, RC::S_UA)];
    lrho += lrhoEg * (Umix + 0.5 * vsq);
    lU += lrhoEg * rho;
    if (!z)
      for (int d = 0; d < 3; ++d) lu[d] += lrhoEg * rho * v[d];
    grad_eq_vjp(v, z == 0, lqe, lR);
  }

  r[RC::SC + RC::C_LRHO] = lrho;
  r[RC::SC + RC::C_LZETA] = lzeta;
  r[RC::SC + RC::C_LH] = lH;
  r[RC::SC + RC::C_LPT] = lPt;
  r[RC::SC + RC::C_LRHOE] = lrhoE;
  r[RC::SC + RC::C_LUMIX] = lU;
  r[RC::SC + RC::C_LT] = lT;
  for (int d = 0; d < 3; ++d) {
    r[RC::SC + RC::C_LU + d] = lu[d];
    r[RC::SC + RC::C_LQ + d] = lq[d];
    r[RC::SC + RC::C_LA1 + d] = lA1[d];
    for (int e = 0; e < 3; ++e) r[RC::SC + RC::C_LPM + 3 * d + e] = lPm[d][e];
  }
}

template <int M>
__device__ __noinline__ void rev_a(lds_tables &tb, double omega, double omega1, lds_double *r, bool collision,
                                   double lT, const double *lY_in, int64_t lY_stride, double lP, double lrho_in,
                                   const double *lu_in, int lane, bool ok) {
  using RC = Rec<M>;
  const int a = lane;
  const bool sp = ok && a < M;
  // per-species working arrays
  if (sp) {
    r[RC::wk(a, RC::W_LY)] = lY_in ? lY_in[a * lY_stride] : 0.0;
    r[RC::wk(a, RC::W_LZA)] = r[RC::asp(a, RC::A_ZETAB)];
    r[RC::wk(a, RC::W_LHA)] = 0.0;
    r[RC::wk(a, RC::W_LRS)] = r[RC::asp(a, RC::A_RHOB)];
    r[RC::wk(a, RC::W_LC)] = 0.0;
    r[RC::wk(a, RC::W_LT)] = 0.0;
    r[RC::wk(a, RC::W_LRDOT)] = 0.0;
    for (int d = 0; d < 3; ++d) r[RC::wk(a, RC::W_LJA + d)] = 0.0;
  }
  if (ok && lane == 0) rev_scalars<M>(tb, omega, omega1, r, collision, lT, lP, lrho_in, lu_in);
  __syncthreads();
  if (!collision) return;   // uniform over the workgroup
  const double rho = r[RC::RHO], P = r[RC::PP], zeta = r[RC::ZETA], om1 = omega1;
  auto Y = [&](int q) -> double { return r[RC::sp(q, RC::S_Y)]; };
  auto rs = [&](int q) -> double { return r[RC::sp(q, RC::S_RS)]; };
  // enthalpy flux hyd = 3 om1 rho sum_a H_a Y_a du_a, the Cg weights
  // w_a = (2 - om1)/2 P H_a, and the species coefficients c_a = 2 beta_a rho_a + rho_dot_a,
  // s_a = (beta_a - 1) Y_a
  double lrho_p = 0.0, lPt_p = 0.0;
  if (sp) {
    const double Ha = r[RC::sp(a, RC::S_HA)];
    double s = 0.0;
    for (int d = 0; d < 3; ++d) {
      const double lA1 = r[RC::SC + RC::C_LA1 + d];
      s += lA1 * r[RC::sp(a, RC::S_DU + d)];
      r[RC::asp(a, RC::A_DU + d)] += 3.0 * om1 * rho * Ha * Y(a) * lA1;
    }
    lrho_p = 3.0 * om1 * Ha * Y(a) * s;
    r[RC::wk(a, RC::W_LHA)] += 3.0 * om1 * rho * Y(a) * s;
    r[RC::wk(a, RC::W_LY)] += 3.0 * om1 * rho * Ha * s;
    double cg = 0.0;
    for (int d = 0; d < 3; ++d) cg += r[RC::L_CG + d] * r[RC::sp(a, RC::S_GY + d)];
    lPt_p = 0.5 * (2.0 - om1) * Ha * cg;
    r[RC::wk(a, RC::W_LHA)] += 0.5 * (2.0 - om1) * P * cg;
    if (a < M - 1) {
      const double beta = r[RC::sp(a, RC::S_BETA)];
      const double lc = r[RC::asp(a, RC::A_C)], ls = r[RC::asp(a, RC::A_S)];
      const double lbeta = r[RC::asp(a, RC::A_BETA)] + 2.0 * rs(a) * lc + Y(a) * ls;
      r[RC::wk(a, RC::W_LRS)] += 2.0 * beta * lc;
      r[RC::wk(a, RC::W_LRDOT)] += lc;
      r[RC::wk(a, RC::W_LY)] += (beta - 1.0) * ls;
      const double ta = r[RC::sp(a, RC::S_T)];
      r[RC::wk(a, RC::W_LT)] += 2.0 * lbeta / ((2.0 + ta) * (2.0 + ta));
    }
  }
  lrho_p = gsum(lrho_p);
  lPt_p = gsum(lPt_p);
  if (ok && lane == 0) {
    r[RC::SC + RC::C_LRHO] += lrho_p;
    r[RC::SC + RC::C_LPT] += lPt_p;
  }
  __syncthreads();
  // Stefan-Maxwell solve A du = r (three right-hand sides): A^T mu = lambda_du by the
  // same factors (U^T then L^T), one right-hand side per lane
  if (ok && lane < 3) {
    const int d = lane;
    for (int q = 0; q < M; ++q) {   // U^T w = lambda
      double v = r[RC::asp(q, RC::A_DU + d)];
      for (int b = 0; b < q; ++b) v -= r[RC::LU + b * M + q] * r[RC::wk(b, RC::W_MU + d)];
      r[RC::wk(q, RC::W_MU + d)] = v / r[RC::LU + q * M + q];
    }
    for (int q = M - 1; q >= 0; --q) {   // L^T mu = w (unit diagonal)
      double v = r[RC::wk(q, RC::W_MU + d)];
      for (int b = q + 1; b < M; ++b) v -= r[RC::LU + b * M + q] * r[RC::wk(b, RC::W_MU + d)];
      r[RC::wk(q, RC::W_MU + d)] = v;
    }
  }
  __syncthreads();
  // lambda_r = mu with r_a = j_a / rho_a - u (0 when rho_a is negligible), on lane a;
  // lambda_A = -mu du^T, column b of A on lane b
  double lu_p[3] = {0.0, 0.0, 0.0};
  if (sp) {
    if (r[RC::sp(a, RC::S_TINY)] == 0.0) {
      double mj = 0.0;
      for (int d = 0; d < 3; ++d) {
        const double mu = r[RC::wk(a, RC::W_MU + d)];
        r[RC::wk(a, RC::W_LJA + d)] += mu / rs(a);
        mj += mu * r[RC::sp(a, RC::S_JA + d)];
        lu_p[d] = -mu;
      }
      r[RC::wk(a, RC::W_LRS)] -= mj / (rs(a) * rs(a));
    }
    const int b = a;
    for (int q = 0; q < M; ++q) {
      double lA = 0.0;
      for (int d = 0; d < 3; ++d) lA -= r[RC::wk(q, RC::W_MU + d)] * r[RC::sp(b, RC::S_DU + d)];
      if (q == b) {
        r[RC::wk(b, RC::W_LT)] += 0.5 * lA;
      } else {
        // A_qb = -K_qb Y_b / 2
        r[RC::LK + q * M + b] += -0.5 * Y(b) * lA;
        r[RC::wk(b, RC::W_LY)] += -0.5 * r[RC::K + q * M + b] * lA;
      }
    }
  }
  for (int d = 0; d < 3; ++d) lu_p[d] = gsum(lu_p[d]);
  if (ok && lane == 0)
    for (int d = 0; d < 3; ++d) r[RC::SC + RC::C_LU + d] += lu_p[d];
  __syncthreads();
  // t_q = sum_b Y_b K_qb: column b on lane b
  if (sp) {
    const int b = a;
    for (int q = 0; q < M; ++q)
      if (q != b) {
        r[RC::wk(b, RC::W_LY)] += r[RC::wk(q, RC::W_LT)] * r[RC::K + q * M + b];
        r[RC::LK + q * M + b] += r[RC::wk(q, RC::W_LT)] * Y(b);
      }
  }
  __syncthreads();
  // K_ab = zeta_a zeta_b / (zeta D_ab), symmetric: row a on lane a; each pair's zeta term
  // on the lane of its first species
  double lz_p = 0.0;
  if (sp) {
    const double za = r[RC::sp(a, RC::S_ZA)];
    for (int b = 0; b < M; ++b) {
      if (b == a) continue;
      const double lK = r[RC::LK + a * M + b] + r[RC::LK + b * M + a];
      const double K = r[RC::K + a * M + b];
      r[RC::wk(a, RC::W_LZA)] += lK * K / za;
      if (b > a) lz_p += lK * K / zeta;
    }
  }
  lz_p = gsum(lz_p);
  if (ok && lane == 0) r[RC::SC + RC::C_LZETA] -= lz_p;
}

// The adjoint of reaction k's rates (Sec. 4): its Arrhenius gradient into pg[3k..3k+2],
// the adjoints of the concentrations it touches added into lc[M]; returns its part of the
// temperature adjoint.
template <int M>
__device__ __forceinline__ double rev_rate(lds_tables &tb, lds_double *r, int k, lds_double *lc, lds_double *pg) {
  using RC = Rec<M>;
  const double T = r[RC::T], lnT = r[RC::LNT], invT = 1.0 / T;
  double lT = 0.0;
  // production rates: rho_dot_a = m_a dt / rho_ref sum_k nu_ka q_k, q_k = fwd_k - rev_k,
  // fwd = exp(ln k_f) prod c^nu', rev = exp(ln k_f - ln K_c) prod c^nu'',
  // ln k_f = ln A + b ln T - Ta / T, d ln K_c / dT = (sum_a nu_ka h_a - nu_k) / T
  auto conc = [&](int idx) -> double { return idx < M ? r[RC::sp(idx, RC::S_C)] : 1.0; };
  double lq_k = 0.0;
  for (int a = 0; a < M - 1; ++a) lq_k += tb.rdot_scale[a] * tb.dnu_a[k][a] * r[RC::wk(a, RC::W_LRDOT)];
  const double fwd = r[RC::RX + 2 * k], rev = r[RC::RX + 2 * k + 1], qk = fwd - rev;
  const double g = lq_k * qk;   // adjoint of ln k_f
  if (pg) {
    pg[3 * k] = g;
    pg[3 * k + 1] = g * lnT;
    pg[3 * k + 2] = -g * invT;
  }
  lT += g * (tb.bexp[k] * invT + tb.Ta[k] * invT * invT);
  const double lnkf = tb.lnA[k] + tb.bexp[k] * lnT - tb.Ta[k] * invT;
  // d (prod c) / d c_a: the product with one factor removed, per factor
  const double kf = exp(lnkf);
  for (int q = 0; q < tb.nreac[k]; ++q) {
    double p = kf;
    for (int q2 = 0; q2 < tb.nreac[k]; ++q2)
      if (q2 != q) p *= conc(tb.reac_idx[k][q2]);
    const int a = tb.reac_idx[k][q];
    if (a < M) lc[a] += lq_k * p;
  }
  if (tb.rev[k]) {
    double dh = -tb.dnu[k], dG = 0.0;
    for (int a = 0; a < M; ++a) {
      dh += tb.dnu_a[k][a] * r[RC::sp(a, RC::S_HRT)];
      dG += tb.dnu_a[k][a] * r[RC::sp(a, RC::S_GIB)];
    }
    lT += lq_k * rev * dh * invT;   // d q / d ln K_c = rev
    const double kr = exp(lnkf + dG - tb.dnu[k] * (tb.ln_c0_const - lnT));
    for (int q = 0; q < tb.nprod[k]; ++q) {
      double p = kr;
      for (int q2 = 0; q2 < tb.nprod[k]; ++q2)
        if (q2 != q) p *= conc(tb.prod_idx[k][q2]);
      const int a = tb.prod_idx[k][q];
      if (a < M) lc[a] -= lq_k * p;
    }
  }
  return lT;
}

template <int M>
__device__ __noinline__ void rev_b(lds_tables &tb, lds_double *r, bool collision, const double *lphi) {
  using RC = Rec<M>;
  const double rho = r[RC::RHO], inv_rho = 1.0 / rho, T = r[RC::T], invT = 1.0 / T;
  const double zeta = r[RC::ZETA], Cv = r[RC::CV];
  double u[3];
  for (int d = 0; d < 3; ++d) u[d] = r[RC::U + d];
  double lrho = r[RC::SC + RC::C_LRHO], lzeta = r[RC::SC + RC::C_LZETA], lH = r[RC::SC + RC::C_LH];
  double lPt = r[RC::SC + RC::C_LPT], lrhoE = r[RC::SC + RC::C_LRHOE], lU = r[RC::SC + RC::C_LUMIX];
  double lT = r[RC::SC + RC::C_LT];
  double lu[3], lq[3], lPm[3][3];
  for (int d = 0; d < 3; ++d) {
    lu[d] = r[RC::SC + RC::C_LU + d];
    lq[d] = r[RC::SC + RC::C_LQ + d];
    for (int e = 0; e < 3; ++e) lPm[d][e] = r[RC::SC + RC::C_LPM + 3 * d + e];
  }
  auto Y = [&](int a) -> double { return r[RC::sp(a, RC::S_Y)]; };
  if (collision)
    for (int a = 0; a < M; ++a) r[RC::wk(a, RC::W_LRS)] += r[RC::wk(a, RC::W_LC)] * tb.conc_scale[a];
  // non-local arguments: phi_d = rho u_d (1 - 3 zeta) - rho u_d^3 (eq. Xalpha)
  if (lphi)
    for (int d = 0; d < 3; ++d) {
      lrho += lphi[d] * (u[d] * (1.0 - 3.0 * zeta) - u[d] * u[d] * u[d]);
      lu[d] += lphi[d] * rho * (1.0 - 3.0 * zeta - 3.0 * u[d] * u[d]);
      lzeta -= 3.0 * rho * lphi[d] * u[d];
    }
  // thermo: H = sum Y_a H_a, P = rho zeta, zeta = T sum Y_a R_a, zeta_a = R_a T,
  // H_a = R_a T h_a(T) (d H_a / dT = R_a cp_a), U = sum Y_a U_a (d U / dT = C_v)
  for (int a = 0; a < M; ++a) {
    r[RC::wk(a, RC::W_LY)] += lH * r[RC::sp(a, RC::S_HA)] + lU * r[RC::sp(a, RC::S_UA)];
    r[RC::wk(a, RC::W_LHA)] += lH * Y(a);
  }
  lT += lU * Cv;
  lrho += lPt * zeta;
  lzeta += lPt * rho;
  lT += lzeta * zeta * invT;
  for (int a = 0; a < M; ++a) {
    r[RC::wk(a, RC::W_LY)] += lzeta * T * tb.Ra[a];
    lT += r[RC::wk(a, RC::W_LZA)] * tb.Ra[a] + r[RC::wk(a, RC::W_LHA)] * tb.Ra[a] * r[RC::sp(a, RC::S_CPR)];
  }
  // temperature (eq. temperature): sum Y_a U_a(T) = rhoE / rho - u^2 / 2
  const double le = lT / Cv;
  for (int a = 0; a < M; ++a) r[RC::wk(a, RC::W_LY)] -= lT * r[RC::sp(a, RC::S_UA)] / Cv;
  lrhoE += le * inv_rho;
  lrho -= le * r[RC::RHOE] * inv_rho * inv_rho;
  for (int d = 0; d < 3; ++d) lu[d] -= le * u[d];
  // Y_a = rho_a / rho
  for (int a = 0; a < M; ++a) {
    const double ly = r[RC::wk(a, RC::W_LY)];
    r[RC::wk(a, RC::W_LRS)] += ly * inv_rho;
    lrho -= ly * Y(a) * inv_rho;
  }
  // u = j / rho
  double lj[3];
  for (int d = 0; d < 3; ++d) {
    lj[d] = lu[d] * inv_rho;
    lrho -= lu[d] * u[d] * inv_rho;
  }
  // slaved species: rho_M = rho - sum rho_a, j_M = j - sum j_a
  const double lrM = r[RC::wk(M - 1, RC::W_LRS)];
  lrho += lrM;
  for (int d = 0; d < 3; ++d) lj[d] += r[RC::wk(M - 1, RC::W_LJA + d)];
  r[RC::M_RHO] = lrho;
  r[RC::M_RHOE] = lrhoE;
  for (int d = 0; d < 3; ++d) {
    r[RC::M_J + d] = lj[d];
    r[RC::M_Q + d] = lq[d];
    for (int e = 0; e < 3; ++e) r[RC::M_P + 3 * d + e] = lPm[d][e];
  }
  for (int a = 0; a < M - 1; ++a) {
    r[RC::M_RA + a] = r[RC::wk(a, RC::W_LRS)] - lrM;
    for (int d = 0; d < 3; ++d)
      r[RC::M_JA + 3 * a + d] = r[RC::wk(a, RC::W_LJA + d)] - r[RC::wk(M - 1, RC::W_LJA + d)];
  }
}


// adjoint of the pulled population of direction i from the adjoints of the moments
template <int M>
__device__ __forceinline__ void moment_adjoint(int i, const double *r, double *out) {
  using RC = Rec<M>;
  const double c[3] = {double(acx(i)), double(acy(i)), double(acz(i))};
  double f = r[RC::M_RHO], g = r[RC::M_RHOE];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    f += c[d] * r[RC::M_J + d];
    g += c[d] * r[RC::M_Q + d];
#pragma unroll
    for (int e = 0; e < 3; ++e) f += c[d] * c[e] * r[RC::M_P + 3 * d + e];
  }
  out[M - 1] = f;
  out[M] = g;
#pragma unroll
  for (int a = 0; a < M - 1; ++a) {
    double v = r[RC::M_RA + a];
#pragma unroll
    for (int d = 0; d < 3; ++d) v += c[d] * r[RC::M_JA + 3 * a + d];
    out[a] = v;
  }
}

// ---- lattice neighbourhood of the adjoint (periodic and open faces) --------------------
struct ALat {
  int nx, ny, nz;
  int per[3];
  int bc[6];
  int64_t N;
};
__device__ __forceinline__ int wrapc(int v, int L) { return v < 0 ? v + L : (v >= L ? v - L : v); }

// push source of the adjoint: the node that pulls population (s, i) of node y after
// streaming, y + c_i (wrapped on periodic axes); -1 when it lies beyond an open face
__device__ __forceinline__ int64_t push_node(const ALat &L, int x, int y, int z, int i) {
  const int n3[3] = {L.nx, L.ny, L.nz};
  int v[3] = {x + acx(i), y + acy(i), z + acz(i)};
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    if (L.per[a]) v[a] = wrapc(v[a], n3[a]);
    else if (v[a] < 0 || v[a] >= n3[a]) return -1;
  }
  return ((int64_t)v[2] * L.ny + v[1]) * L.nx + v[0];
}

// Adjoint of the ghost equilibria of node (x, y, z) along direction i: every ghost cell
// whose adjacent node it is (the one-cell layer beyond open faces: the node's position
// with one or more coordinates moved across an open face) is pulled by the node g + c_i
// when that lies in the lattice.  Summed per velocity kind of the ghost: zero_u = 1 when a
// crossed face is a zero-velocity face.
template <int S>
__device__ __forceinline__ bool ghost_adjoint(const ALat &L, int x, int y, int z, int i, const double *Ln,
                                              double (&lg)[2][S]) {
  const int n3[3] = {L.nx, L.ny, L.nz}, p3[3] = {x, y, z}, c3[3] = {acx(i), acy(i), acz(i)};
  // per axis: options 0 = in place, 1 = the ghost before the first node, 2 = after the last
  bool opt[3][3];
  bool any = false;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    opt[a][0] = true;
    opt[a][1] = !L.per[a] && p3[a] == 0;
    opt[a][2] = !L.per[a] && p3[a] == n3[a] - 1;
    any = any || opt[a][1] || opt[a][2];
  }
#pragma unroll
  for (int z2 = 0; z2 < 2; ++z2)
#pragma unroll
    for (int s = 0; s < S; ++s) lg[z2][s] = 0.0;
  if (!any) return false;
  bool hit = false;
  for (int ox = 0; ox < 3; ++ox) {
    if (!opt[0][ox]) continue;
    for (int oy = 0; oy < 3; ++oy) {
      if (!opt[1][oy]) continue;
      for (int oz = 0; oz < 3; ++oz) {
        if (!opt[2][oz]) continue;
        const int o[3] = {ox, oy, oz};
        if (ox == 0 && oy == 0 && oz == 0) continue;
        int rcv[3];
        bool ok = true, zero_u = false;
        for (int a = 0; a < 3 && ok; ++a) {
          if (o[a] == 0) {
            int v = p3[a] + c3[a];
            if (L.per[a]) v = wrapc(v, n3[a]);
            ok = v >= 0 && v < n3[a];
            rcv[a] = v;
          } else {
            // ghost at -1 (o = 1) or n (o = 2): pulled by node 0 along c = +1, n - 1 along -1
            const int need = o[a] == 1 ? 1 : -1;
            ok = c3[a] == need;
            rcv[a] = o[a] == 1 ? 0 : n3[a] - 1;
            zero_u = zero_u || L.bc[2 * a + (o[a] == 1 ? 0 : 1)] == LBM_BC_OPEN_EQ_U0;
          }
        }
        if (!ok) continue;
        hit = true;
        const int64_t rn = ((int64_t)rcv[2] * L.ny + rcv[1]) * L.nx + rcv[0];
        for (int s = 0; s < S; ++s) lg[zero_u ? 1 : 0][s] += Ln[((int64_t)s * Q + i) * L.N + rn];
      }
    }
  }
  return hit;
}

// The three (node, c) pairs per axis whose gradient neighbour is z: wrap(y + c) on a
// periodic axis, clamp(y + c) on an open one.  Inside an open axis they are (z, 0),
// (z - 1, +1) and (z + 1, -1); the first node has (0, -1) in place of (z - 1, +1), the
// last (L - 1, +1) in place of (z + 1, -1) (both, on an axis of one node).
struct APairs {
  int y[3], c[3];
};
__device__ __forceinline__ APairs axis_pairs(int zc, int Lax, bool periodic) {
  APairs p;
  p.y[0] = zc;
  p.c[0] = 0;
  if (periodic) {
    p.y[1] = wrapc(zc - 1, Lax);
    p.c[1] = 1;
    p.y[2] = wrapc(zc + 1, Lax);
    p.c[2] = -1;
  } else {
    const bool lo = zc >= 1, hi = zc <= Lax - 2;
    p.y[1] = lo ? zc - 1 : 0;
    p.c[1] = lo ? 1 : -1;
    p.y[2] = hi ? zc + 1 : zc;
    p.c[2] = hi ? -1 : 1;
  }
  return p;
}

// ---- kernels -------------------------------------------------------------------------------
struct AdjBuf {
  const double *P;     // [S][27][N] pulled populations of the forward state
  const double *Ln;    // [S][27][N] incoming adjoint (lambda_{n+1})
  const double *T0;    // [N] stored temperature of the forward state (Newton start)
  double *fY, *fw;     // [M][N] forward mass fractions and Cg weights
  double *lX, *lgY;    // [3][N], [M][3][N]
  double *lpsi, *lphi; // [3][N]
  double *lYs;         // [M][N]
  double *part;        // [3R][nblocks] Arrhenius gradient partials
};

// forward side fields: Y_a and the weights w_a = (2 - omega1)/2 P H_a of Cg.  A node's
// directions on the lanes of a 32-lane group (moments by group sums), its species on
// lanes 0..M-1.
template <int M>
// It also copies the incoming adjoint of its node into the work buffer Ln (lam_in is
// overwritten with lambda_n by k_adj_step, while Ln is read at the neighbours).
__global__ __launch_bounds__(ADJ_BLOCK) void k_adj_fwd(ALat L, const Tables *tbp, AdjBuf ab, double omega1,
                                                       const double *lam_in, double *Ln) {
  constexpr int S = M + 1;
  const Tables &tb = *tbp;
  const int slot = threadIdx.x / GL, lane = threadIdx.x % GL;
  const int64_t n = (int64_t)blockIdx.x * NPB + slot;
  const bool node_ok = n < L.N;
  const int64_t nn = node_ok ? n : 0;
  const bool valid = node_ok && lane < Q;
  const int i = lane < Q ? lane : 13;
  const int64_t N = L.N;
  double f[S], lam[S];
#pragma unroll
  for (int s = 0; s < S; ++s) {
    f[s] = valid ? ab.P[((int64_t)s * Q + i) * N + nn] : 0.0;
    lam[s] = valid ? lam_in[((int64_t)s * Q + i) * N + nn] : 0.0;
  }
  if (valid)
#pragma unroll
    for (int s = 0; s < S; ++s) Ln[((int64_t)s * Q + i) * N + nn] = lam[s];
  Mom<M> m;
  group_moments<M>(i, valid, f, m);
  // species on lanes a < M; the Newton iteration on every lane alike, on the group sums
  // of the internal-energy and heat-capacity polynomials
  double rsum = 0.0;
  for (int a = 0; a < M - 1; ++a) rsum += m.ra[a];
  const int a = lane;
  const bool sp = a < M;
  const double Y = sp ? (a < M - 1 ? m.ra[a] : m.rho - rsum) / m.rho : 0.0;
  const double usq = (m.j[0] * m.j[0] + m.j[1] * m.j[1] + m.j[2] * m.j[2]) / (m.rho * m.rho);
  const double e = m.rhoE / m.rho - 0.5 * usq;
  double ec[6], dc[5];
  for (int k = 0; k < 6; ++k) ec[k] = gsum(sp ? Y * tb.ucoef[a][k] : 0.0);
  for (int k = 0; k < 5; ++k) dc[k] = gsum(sp ? Y * tb.cvcoef[a][k] : 0.0);
  double T = ab.T0[nn];
  for (int it = 0; it < 50; ++it) {
    const double ev = ec[0] + T * (ec[1] + T * (ec[2] + T * (ec[3] + T * (ec[4] + T * ec[5])))) - e;
    const double dv = dc[0] + T * (dc[1] + T * (dc[2] + T * (dc[3] + T * dc[4])));
    const double dT = -ev / dv;
    T += dT;
    if (fabs(dT) <= 1e-12 * fabs(T)) break;
  }
  const double zeta = gsum(sp ? Y * tb.Ra[a] * T : 0.0);
  const double Pp = m.rho * zeta;
  if (node_ok && sp) {
    ab.fY[a * N + nn] = Y;
    ab.fw[a * N + nn] = 0.5 * (2.0 - omega1) * Pp * tb.Ra[a] * T * a_hRT(tb.nasa[a], T);
  }
}

// adjoints of the stencil outputs at each node: X (from the axis directions of f) and
// Cg (from g), the latter spread over the species as lambda_gY_a = w_a lambda_Cg.  A
// node's directions on the lanes of a 32-lane group, summed over the group.
template <int M>
__global__ __launch_bounds__(ADJ_BLOCK) void k_adj_x(ALat L, AdjBuf ab) {
  const int slot = threadIdx.x / GL, lane = threadIdx.x % GL;
  const int64_t n = (int64_t)blockIdx.x * NPB + slot;
  const bool node_ok = n < L.N;
  const int64_t nn = node_ok ? n : 0;
  const bool valid = node_ok && lane < Q;
  const int i = lane < Q ? lane : 13;
  const int64_t N = L.N;
  const int x = (int)(nn % L.nx), y = (int)((nn / L.nx) % L.ny), z = (int)(nn / ((int64_t)L.nx * L.ny));
  const int64_t pn = valid ? push_node(L, x, y, z, i) : -1;
  const double Lf = pn >= 0 ? ab.Ln[((int64_t)(M - 1) * Q + i) * N + pn] : 0.0;
  const double Lg = pn >= 0 ? ab.Ln[((int64_t)M * Q + i) * N + pn] : 0.0;
  const int c[3] = {acx(i), acy(i), acz(i)};
  const bool axis = c[0] * c[0] + c[1] * c[1] + c[2] * c[2] == 1;
  double lX[3], lC[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    lX[d] = gsum(axis ? 0.5 * c[d] * Lf : 0.0);
    lC[d] = gsum(3.0 * awgt(i) * c[d] * Lg);
  }
  if (!node_ok) return;
  if (lane < 3) {
    const int d = lane;
    ab.lX[d * N + nn] = d == 0 ? lX[0] : (d == 1 ? lX[1] : lX[2]);
  }
  if (lane < M) {
    const int a = lane;
    const double w = ab.fw[a * N + nn];
#pragma unroll
    for (int d = 0; d < 3; ++d) ab.lgY[(a * 3 + d) * N + nn] = w * lC[d];
  }
}

// transposed isotropic gradient: out(z) = sum over (y, i) with nb(y, i) = z of
// 3 w_i c_i,alpha in(y).  DIAG: a vector input, out_alpha from in_alpha (out[3]); else
// one species' vector input, out = sum_alpha of the components (out[1]).  The 27 source
// nodes are fixed, so their loads are independent of each other.
template <bool DIAG>
__device__ __forceinline__ void transposed_grad(const ALat &L, int64_t n, const double *in, int64_t comp_stride,
                                                double *out) {
  const int x = (int)(n % L.nx), y = (int)((n / L.nx) % L.ny), z = (int)(n / ((int64_t)L.nx * L.ny));
  const APairs px = axis_pairs(x, L.nx, L.per[0]), py = axis_pairs(y, L.ny, L.per[1]),
               pz = axis_pairs(z, L.nz, L.per[2]);
  double o[3] = {0.0, 0.0, 0.0};
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b)
#pragma unroll
      for (int cc = 0; cc < 3; ++cc) {
        const int cv[3] = {px.c[a], py.c[b], pz.c[cc]};
        const double w3 = 3.0 * aw1(cv[0]) * aw1(cv[1]) * aw1(cv[2]);
        const int64_t src = ((int64_t)pz.y[cc] * L.ny + py.y[b]) * L.nx + px.y[a];
#pragma unroll
        for (int d = 0; d < 3; ++d) o[DIAG ? d : 0] += w3 * double(cv[d]) * in[d * comp_stride + src];
      }
#pragma unroll
  for (int d = 0; d < (DIAG ? 3 : 1); ++d) out[d] = o[d];
}

// lambda_psi = -G^T lambda_X (X_alpha = -grad_alpha psi_alpha)
__global__ __launch_bounds__(128) void k_adj_psi(ALat L, AdjBuf ab) {
  const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= L.N) return;
  double o[3];
  transposed_grad<true>(L, n, ab.lX, L.N, o);
  for (int d = 0; d < 3; ++d) ab.lpsi[d * L.N + n] = -o[d];
}

// lambda_phi = (1/omega - 1/2) G^T lambda_psi; lambda_Y_a = G^T lambda_gY_a.  One thread
// per (node, output): output a < M is species a, output M the three components of phi.
template <int M>
__global__ __launch_bounds__(128) void k_adj_phi(ALat L, AdjBuf ab, double coef) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= L.N * (M + 1)) return;
  const int comp = (int)(t / L.N);
  const int64_t n = t - (int64_t)comp * L.N;
  double o[3];
  if (comp == M) {
    transposed_grad<true>(L, n, ab.lpsi, L.N, o);
    for (int d = 0; d < 3; ++d) ab.lphi[d * L.N + n] = coef * o[d];
  } else {
    transposed_grad<false>(L, n, ab.lgY + (int64_t)comp * 3 * L.N, L.N, o);
    ab.lYs[comp * L.N + n] = o[0];
  }
}

// The reverse of the collision, ghosts and streaming of one step at each node (see the
// file header).  Writes lambda_n into out and the Arrhenius partials of the workgroup.
template <int M>
__global__ __launch_bounds__(ADJ_BLOCK) void k_adj_step(ALat L, const Tables *tbp, AdjBuf ab, double omega,
                                                        double omega1, double *out) {
  constexpr int S = M + 1;
  using RC = Rec<M>;
  __shared__ double recs[NPB][RC::WORDS];
  __shared__ double pgs[NPB][3 * MAXR];
  __shared__ double lcs[NPB][GL][M];   // per lane: its reactions' concentration adjoints
  __shared__ Tables tbs;
  const Tables &tb = *tbp;
  tables_to_lds(tbp, &tbs);
  lds_tables &tl = *(lds_tables *)&tbs;
  const int slot = threadIdx.x / GL, lane = threadIdx.x % GL;
  const int64_t n = (int64_t)blockIdx.x * NPB + slot;
  const bool node_ok = n < L.N;
  const int64_t nn = node_ok ? n : 0;
  const bool valid = node_ok && lane < Q;
  const int i = lane < Q ? lane : 13;
  const int64_t N = L.N;
  double *r = recs[slot];
  lds_double *rl = (lds_double *)recs[slot];
  const int x = (int)(nn % L.nx), y = (int)((nn / L.nx) % L.ny), z = (int)(nn / ((int64_t)L.nx * L.ny));
  // clear the reduced-adjoint part of the record
  for (int k = RC::L0 + lane; k < RC::MO; k += GL) r[k] = 0.0;
  for (int k = lane; k < 3 * MAXR; k += GL) pgs[slot][k] = 0.0;
  for (int a = 0; a < M; ++a) lcs[slot][lane][a] = 0.0;
  __syncthreads();

  // adjoints arriving at this node's post-collision populations (push)
  double Lp[S];
  {
    const int64_t pn = valid ? push_node(L, x, y, z, i) : -1;
#pragma unroll
    for (int s = 0; s < S; ++s) Lp[s] = pn >= 0 ? ab.Ln[((int64_t)s * Q + i) * N + pn] : 0.0;
  }
  // the lane's pulled populations, the node's moments and its forward chain; the direct
  // term -2 f_a of d f_a' / d beta_a is taken here, while f is at hand
  {
    double f[S];
#pragma unroll
    for (int s = 0; s < S; ++s) f[s] = valid ? ab.P[((int64_t)s * Q + i) * N + nn] : 0.0;
#pragma unroll
    for (int a = 0; a < M - 1; ++a) {
      const double lb = gsum(-2.0 * f[a] * Lp[a]);
      if (lane == 0) r[RC::asp(a, RC::A_BETA)] = lb;
    }
    Mom<M> m;
    group_moments<M>(i, valid, f, m);
    node_forward<M>(tl, m, ab.T0[nn], rl, lane, node_ok, true);
  }
  // grad Y_a at the node from the neighbours' mass fractions (forward O6 stencil)
  {
    const int c[3] = {acx(i), acy(i), acz(i)};
    int v[3] = {x + c[0], y + c[1], z + c[2]};
    const int n3[3] = {L.nx, L.ny, L.nz};
#pragma unroll
    for (int a = 0; a < 3; ++a) v[a] = L.per[a] ? wrapc(v[a], n3[a]) : (v[a] < 0 ? 0 : (v[a] >= n3[a] ? n3[a] - 1 : v[a]));
    const int64_t nb = ((int64_t)v[2] * L.ny + v[1]) * L.nx + v[0];
    const double w3 = valid ? 3.0 * awgt(i) : 0.0;
#pragma unroll
    for (int a = 0; a < M; ++a) {
      const double ya = node_ok ? ab.fY[a * N + nb] : 0.0;
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        const double gy = gsum(w3 * c[d] * ya);
        if (lane == 0) r[RC::sp(a, RC::S_GY + d)] = gy;
      }
    }
  }
  __syncthreads();
  // production rates: one reaction per lane, then one species per lane; then the
  // Stefan-Maxwell step on the first lane
  if (node_ok)
    for (int k = lane; k < tl.R; k += GL) fwd_rate<M>(tl, rl, k);
  __syncthreads();
  if (node_ok && lane < M) fwd_rdot<M>(tl, rl, lane);
  __syncthreads();
  fwd_sm<M>(tl, rl, lane, node_ok);
  __syncthreads();

  // adjoints arriving at the ghost equilibria of this node
  double lg[2][S];
  const bool has_ghost = valid ? ghost_adjoint<S>(L, x, y, z, i, ab.Ln, lg) : false;
  if (!has_ghost)
#pragma unroll
    for (int s = 0; s < S; ++s) lg[0][s] = lg[1][s] = 0.0;

  // per-direction forward values
  const double rho = r[RC::RHO], zeta = r[RC::ZETA];
  double u[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) u[d] = r[RC::U + d];
  const double c[3] = {double(acx(i)), double(acy(i)), double(acz(i))};
  const double wi = awgt(i);

  // f: omega rho Phi_i(u, zeta); the ghost f: rho Phi_i(v, zeta)
  double lrhof = 0.0, lu[3] = {0.0, 0.0, 0.0}, lzeta = 0.0;
  {
    const PhiD p = phi_d(i, u, zeta);
    const double a = omega * Lp[M - 1];
    lrhof += a * p.v;
    lzeta += a * rho * p.dz;
#pragma unroll
    for (int d = 0; d < 3; ++d) lu[d] += a * rho * p.du[d];
    lrhof += lg[0][M - 1] * p.v;
    lzeta += lg[0][M - 1] * rho * p.dz;
#pragma unroll
    for (int d = 0; d < 3; ++d) lu[d] += lg[0][M - 1] * rho * p.du[d];
    const double zero[3] = {0.0, 0.0, 0.0};
    const PhiD p0 = phi_d(i, zero, zeta);
    lrhof += lg[1][M - 1] * p0.v;
    lzeta += lg[1][M - 1] * rho * p0.dz;
  }
  // g: bracket adjoints, collision (w_i Lg) and ghosts (w_i lg)
  {
    const double a = wi * Lp[M];
    double* dummy = nullptr;
    (void)dummy;
    const double vals[2] = {wi * lg[0][M], wi * lg[1][M]};
    double s;
    s = gsum(a);
    if (lane == 0) r[RC::L_A0] = s;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      s = gsum(a * c[d]);
      if (lane == 0) r[RC::L_A1 + d] = s;
      s = gsum(3.0 * a * c[d]);
      if (lane == 0) r[RC::L_CG + d] = s;
#pragma unroll
      for (int e = 0; e < 3; ++e) {
        s = gsum(a * c[d] * c[e]);
        if (lane == 0) r[RC::L_B + 3 * d + e] = s;
      }
    }
#pragma unroll
    for (int zz = 0; zz < 2; ++zz) {
      s = gsum(vals[zz]);
      if (lane == 0) r[RC::L_A0G + zz] = s;
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        s = gsum(vals[zz] * c[d]);
        if (lane == 0) r[RC::L_A1G + 3 * zz + d] = s;
#pragma unroll
        for (int e = 0; e < 3; ++e) {
          s = gsum(vals[zz] * c[d] * c[e]);
          if (lane == 0) r[RC::L_BG + 9 * zz + 3 * d + e] = s;
        }
      }
    }
  }
  // species: f_a' = (1 - 2 beta_a) f_a + c_a Phi_i(u, zeta_a) + s_a sum_{b != a} K_ab G_b,
  // G_b = rho_b (Phi_i(u, zeta_b) - Phi_i(u + du_b, zeta_b))
  double G[M];
#pragma unroll
  for (int b = 0; b < M; ++b) {
    const double zb = r[RC::sp(b, RC::S_ZA)], rb = r[RC::sp(b, RC::S_RS)];
    double us[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) us[d] = u[d] + r[RC::sp(b, RC::S_DU + d)];
    const PhiD pe = phi_d(i, u, zb);
    const PhiD ps = phi_d(i, us, zb);
    G[b] = rb * (pe.v - ps.v);
    // Gamma_b = sum_{a != b} L_a s_a K_ab
    double gam = 0.0;
#pragma unroll
    for (int a = 0; a < M - 1; ++a)
      if (a != b) gam += Lp[a] * r[RC::sp(a, RC::S_SA)] * r[RC::K + a * M + b];
    const double lrb = gsum(gam * (pe.v - ps.v));
    const double lzb = gsum(gam * rb * (pe.dz - ps.dz));
    double ldu[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      lu[d] += gam * rb * (pe.du[d] - ps.du[d]);
      ldu[d] = gsum(-gam * rb * ps.du[d]);
    }
    if (lane == 0) {
      r[RC::asp(b, RC::A_RHOB)] += lrb;
      r[RC::asp(b, RC::A_ZETAB)] += lzb;
#pragma unroll
      for (int d = 0; d < 3; ++d) r[RC::asp(b, RC::A_DU + d)] += ldu[d];
    }
  }
#pragma unroll
  for (int a = 0; a < M - 1; ++a) {
    const double ca = r[RC::sp(a, RC::S_CA)], sa = r[RC::sp(a, RC::S_SA)], ra = r[RC::sp(a, RC::S_RS)];
    double FK = 0.0;
#pragma unroll
    for (int b = 0; b < M; ++b)
      if (b != a) FK += r[RC::K + a * M + b] * G[b];
    const double La = Lp[a];
    // equilibrium and source (coefficient c_a), and the ghosts rho_a Phi_i(v, zeta_a)
    const double zero[3] = {0.0, 0.0, 0.0};
    const PhiD pa = phi_d(i, u, r[RC::sp(a, RC::S_ZA)]);
    const PhiD p0 = phi_d(i, zero, r[RC::sp(a, RC::S_ZA)]);
    const double lc = gsum(La * pa.v);
    const double ls = gsum(La * FK);
    const double lrg = gsum(lg[0][a] * pa.v + lg[1][a] * p0.v);
    const double lzg = gsum(ca * La * pa.dz + lg[0][a] * ra * pa.dz + lg[1][a] * ra * p0.dz);
#pragma unroll
    for (int d = 0; d < 3; ++d) lu[d] += ca * La * pa.du[d] + lg[0][a] * ra * pa.du[d];
    // K_ab: L_a s_a G_b
    double lk[M];
#pragma unroll
    for (int b = 0; b < M; ++b) lk[b] = (b != a) ? gsum(La * sa * G[b]) : 0.0;
    if (lane == 0) {
      r[RC::asp(a, RC::A_C)] += lc;
      r[RC::asp(a, RC::A_S)] += ls;
      r[RC::asp(a, RC::A_RHOB)] += lrg;
      r[RC::asp(a, RC::A_ZETAB)] += lzg;
#pragma unroll
      for (int b = 0; b < M; ++b)
        if (b != a) r[RC::LK + a * M + b] += lk[b];
    }
  }
  {
    const double s0 = gsum(lrhof), s1 = gsum(lzeta);
    double su[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) su[d] = gsum(lu[d]);
    if (lane == 0) {
      r[RC::L_RHOF] = s0;
      r[RC::L_ZETA] = s1;
#pragma unroll
      for (int d = 0; d < 3; ++d) r[RC::L_U + d] = su[d];
    }
  }
  __syncthreads();
  rev_a<M>(tl, omega, omega1, rl, true, 0.0, ab.lYs + nn, N, 0.0, 0.0, nullptr, lane, node_ok);
  __syncthreads();
  // the rates' adjoints, one reaction per lane; the concentration adjoints summed per
  // species over the lanes' rows, the temperature adjoint over the group
  {
    double lTr = 0.0;
    if (node_ok)
      for (int k = lane; k < tl.R; k += GL)
        lTr += rev_rate<M>(tl, rl, k, (lds_double *)lcs[slot][lane], (lds_double *)pgs[slot]);
    lTr = gsum(lTr);
    __syncthreads();
    if (node_ok && lane < M) {
      double sc = 0.0;
      for (int q = 0; q < GL; ++q) sc += lcs[slot][q][lane];
      r[RC::wk(lane, RC::W_LC)] = sc;
    }
    if (node_ok && lane == 0) r[RC::SC + RC::C_LT] += lTr;
  }
  __syncthreads();
  if (lane == 0 && node_ok) {
    double lphi[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) lphi[d] = ab.lphi[d * N + nn];
    rev_b<M>(tl, rl, true, lphi);
  }
  __syncthreads();
  if (valid) {
    // lambda_n: the direct part (the relaxation factors of each population) plus the
    // part through the moments
    double mo[S];
    moment_adjoint<M>(i, r, mo);
    out[((int64_t)(M - 1) * Q + i) * N + nn] = (1.0 - omega) * Lp[M - 1] + mo[M - 1];
    out[((int64_t)M * Q + i) * N + nn] = (1.0 - omega) * Lp[M] + mo[M];
#pragma unroll
    for (int a = 0; a < M - 1; ++a)
      out[((int64_t)a * Q + i) * N + nn] = (1.0 - 2.0 * r[RC::sp(a, RC::S_BETA)]) * Lp[a] + mo[a];
  }
  // Arrhenius partials of the workgroup: fixed order over its nodes
  for (int k = threadIdx.x; k < 3 * tb.R; k += ADJ_BLOCK) {
    double s = 0.0;
    for (int q = 0; q < NPB; ++q) s += pgs[q][k];
    ab.part[(int64_t)k * gridDim.x + blockIdx.x] = s;
  }
}

// sum of the workgroup partials into the caller's gradient (+=): one workgroup per
// entry, strided partial sums per thread, then a tree over the workgroup (a fixed order)
constexpr int PSUM_BLOCK = 256;
__global__ __launch_bounds__(PSUM_BLOCK) void k_adj_param_sum(const double *part, int64_t nparts, double *grad) {
  __shared__ double red[PSUM_BLOCK];
  const int k = blockIdx.x;
  double s = 0.0;
  for (int64_t j = threadIdx.x; j < nparts; j += PSUM_BLOCK) s += part[(int64_t)k * nparts + j];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int h = PSUM_BLOCK / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) grad[k] += red[0];
}

// Adjoint of the macroscopic fields (lbm_macros) of a state: lambda = sum over nodes of
// w_rho rho + w_u . u + w_T T + w_P P + w_Y . Y differentiated with respect to the pulled
// populations.
template <int M>
__global__ __launch_bounds__(ADJ_BLOCK) void k_adj_macros(ALat L, const Tables *tbp, const double *P, const double *T0,
                                                          const double *w_rho, const double *w_u, const double *w_T,
                                                          const double *w_P, const double *w_Y, double *out) {
  constexpr int S = M + 1;
  using RC = Rec<M>;
  __shared__ double recs[NPB][RC::WORDS];
  __shared__ Tables tbs;
  tables_to_lds(tbp, &tbs);
  lds_tables &tl = *(lds_tables *)&tbs;
  const int slot = threadIdx.x / GL, lane = threadIdx.x % GL;
  const int64_t n = (int64_t)blockIdx.x * NPB + slot;
  const bool node_ok = n < L.N;
  const int64_t nn = node_ok ? n : 0;
  const bool valid = node_ok && lane < Q;
  const int i = lane < Q ? lane : 13;
  const int64_t N = L.N;
  double *r = recs[slot];
  lds_double *rl = (lds_double *)recs[slot];
  for (int k = RC::L0 + lane; k < RC::MO; k += GL) r[k] = 0.0;
  __syncthreads();
  double f[S];
#pragma unroll
  for (int s = 0; s < S; ++s) f[s] = valid ? P[((int64_t)s * Q + i) * N + nn] : 0.0;
  Mom<M> m;
  group_moments<M>(i, valid, f, m);
  node_forward<M>(tl, m, T0[nn], rl, lane, node_ok, false);
  __syncthreads();
  {
    double lu[3];
    for (int d = 0; d < 3; ++d) lu[d] = w_u ? w_u[d * N + nn] : 0.0;
    rev_a<M>(tl, 0.0, 0.0, rl, false, w_T ? w_T[nn] : 0.0, w_Y ? w_Y + nn : nullptr, N, w_P ? w_P[nn] : 0.0,
             w_rho ? w_rho[nn] : 0.0, lu, lane, node_ok);
    if (lane == 0 && node_ok) rev_b<M>(tl, rl, false, nullptr);
  }
  __syncthreads();
  if (valid) {
    double mo[S];
    moment_adjoint<M>(i, r, mo);
#pragma unroll
    for (int s = 0; s < S; ++s) out[((int64_t)s * Q + i) * N + nn] = mo[s];
  }
}

// Adjoint of the equilibrium initial state (lbm_init_fields): from lambda_0 on the pulled
// populations, the gradients with respect to the fields rho, u, T, Y of each node.
// f = rho Phi(u, zeta), f_a = rho Y_a Phi(u, zeta_a), g = Grad(rho E, q^eq, R^eq) with
// E = U(T, Y) + u^2/2 (eqs. feq, gieq; reading R10).
template <int M>
__global__ __launch_bounds__(ADJ_BLOCK) void k_adj_init(ALat L, const Tables *tbp, const double *rho0,
                                                        const double *u0, const double *Tf, const double *Y0,
                                                        const double *lam, double *g_rho, double *g_u, double *g_T,
                                                        double *g_Y) {
  const Tables &tb = *tbp;
  const int slot = threadIdx.x / GL, lane = threadIdx.x % GL;
  const int64_t n = (int64_t)blockIdx.x * NPB + slot;
  const bool node_ok = n < L.N;
  const int64_t nn = node_ok ? n : 0;
  const bool valid = node_ok && lane < Q;
  const int i = lane < Q ? lane : 13;
  const int64_t N = L.N;
  const double rho = rho0[nn], T = Tf[nn];
  double u[3], Y[M], za[M], h[M];
  for (int d = 0; d < 3; ++d) u[d] = u0[d * N + nn];
  double zeta = 0.0, H = 0.0, U = 0.0;
  for (int a = 0; a < M; ++a) {
    Y[a] = Y0[a * N + nn];
    za[a] = tb.Ra[a] * T;
    h[a] = a_hRT(tb.nasa[a], T);
    zeta += Y[a] * za[a];
    H += Y[a] * za[a] * h[a];
    U += Y[a] * za[a] * (h[a] - 1.0);
  }
  const double c[3] = {double(acx(i)), double(acy(i)), double(acz(i))};
  const double Lf = valid ? lam[((int64_t)(M - 1) * Q + i) * N + nn] : 0.0;
  const double Lg = valid ? lam[((int64_t)M * Q + i) * N + nn] : 0.0;
  // f and species
  double lrho = 0.0, lu[3] = {0.0, 0.0, 0.0}, lzeta = 0.0, lza[M], lY[M];
  const PhiD pf = phi_d(i, u, zeta);
  lrho += Lf * pf.v;
  lzeta += Lf * rho * pf.dz;
  for (int d = 0; d < 3; ++d) lu[d] += Lf * rho * pf.du[d];
  for (int a = 0; a < M; ++a) {
    lza[a] = 0.0;
    lY[a] = 0.0;
  }
  for (int a = 0; a < M - 1; ++a) {
    const double La = valid ? lam[((int64_t)a * Q + i) * N + nn] : 0.0;
    const PhiD p = phi_d(i, u, za[a]);
    lrho += La * Y[a] * p.v;
    lY[a] += La * rho * p.v;
    lza[a] += La * rho * Y[a] * p.dz;
    for (int d = 0; d < 3; ++d) lu[d] += La * rho * Y[a] * p.du[d];
  }
  // g bracket adjoints
  const double wl = awgt(i) * Lg;
  double lA0 = gsum(wl), lA1[3], lB[3][3];
  for (int d = 0; d < 3; ++d) {
    lA1[d] = gsum(wl * c[d]);
    for (int e = 0; e < 3; ++e) lB[d][e] = gsum(wl * c[d] * c[e]);
  }
  lrho = gsum(lrho);
  lzeta = gsum(lzeta);
  for (int d = 0; d < 3; ++d) lu[d] = gsum(lu[d]);
  for (int a = 0; a < M; ++a) {
    lza[a] = gsum(lza[a]);
    lY[a] = gsum(lY[a]);
  }
  if (lane != 0 || !node_ok) return;
  // Grad form: A0 = 2.5 rhoE - 1.5 tr R, A1 = 3 q^eq, B_dd = 4.5 R_dd - 1.5 rhoE, B_de = 4.5 R_de
  const double usq = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
  const double h2 = H + 0.5 * usq, P = rho * zeta;
  double lrhoE = 2.5 * lA0, lR[3][3], lqe[3];
  for (int d = 0; d < 3; ++d) {
    lqe[d] = 3.0 * lA1[d];
    for (int e = 0; e < 3; ++e) {
      lR[d][e] = 4.5 * lB[d][e] + (d == e ? -1.5 * lA0 : 0.0);
      if (d == e) lrhoE -= 1.5 * lB[d][e];
    }
  }
  double lh2 = 0.0, lP = 0.0, lH = 0.0, lU = 0.0;
  for (int d = 0; d < 3; ++d) {
    lh2 += lqe[d] * rho * u[d];
    lrho += lqe[d] * h2 * u[d];
    lu[d] += lqe[d] * h2 * rho;
  }
  for (int d = 0; d < 3; ++d)
    for (int e = 0; e < 3; ++e) {
      const double Peq = (d == e ? P : 0.0) + rho * u[d] * u[e];
      lh2 += lR[d][e] * Peq;
      lrho += lR[d][e] * h2 * u[d] * u[e];
      lP += lR[d][e] * ((d == e ? h2 : 0.0) + u[d] * u[e]);
      const double fct = lR[d][e] * (h2 * rho + P);
      lu[d] += fct * u[e];
      lu[e] += fct * u[d];
    }
  lH += lh2;
  for (int d = 0; d < 3; ++d) lu[d] += lh2 * u[d];
  // rhoE = rho (U + u^2/2)
  lrho += lrhoE * (U + 0.5 * usq);
  lU += lrhoE * rho;
  for (int d = 0; d < 3; ++d) lu[d] += lrhoE * rho * u[d];
  // P = rho zeta
  lrho += lP * zeta;
  lzeta += lP * rho;
  // zeta = sum Y_a zeta_a, H = sum Y_a zeta_a h_a, U = sum Y_a zeta_a (h_a - 1), zeta_a = R_a T
  double lT = 0.0;
  for (int a = 0; a < M; ++a) {
    lY[a] += lzeta * za[a] + lH * za[a] * h[a] + lU * za[a] * (h[a] - 1.0);
    // d (zeta_a h_a) / dT = R_a cp_a; d (zeta_a (h_a - 1)) / dT = R_a (cp_a - 1)
    const double cp = a_cpR(tb.nasa[a], T);
    lT += (lza[a] + lzeta * Y[a]) * tb.Ra[a] + lH * Y[a] * tb.Ra[a] * cp + lU * Y[a] * tb.Ra[a] * (cp - 1.0);
  }
  if (g_rho) g_rho[nn] = lrho;
  if (g_T) g_T[nn] = lT;
  if (g_u)
    for (int d = 0; d < 3; ++d) g_u[d * N + nn] = lu[d];
  if (g_Y)
    for (int a = 0; a < M; ++a) g_Y[a * N + nn] = lY[a];
}

inline unsigned ablocks(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

ALat make_alat(const Geom &g) {
  ALat L;
  L.nx = g.nx;
  L.ny = g.ny;
  L.nz = g.nz;
  for (int a = 0; a < 3; ++a) L.per[a] = g.per[a];
  for (int k = 0; k < 6; ++k) L.bc[k] = g.bc[k];
  L.N = g.N;
  return L;
}

template <int M>
hipError_t adj_step_m(const Geom &g, const Tables *tb, const AdjBufHost &h, double omega, double omega1, int R,
                      double *adj, double *grad, hipStream_t st) {
  const ALat L = make_alat(g);
  AdjBuf ab{h.P, h.Ln, h.T0, h.fY, h.fw, h.lX, h.lgY, h.lpsi, h.lphi, h.lYs, h.part};
  hipLaunchKernelGGL((k_adj_fwd<M>), dim3(ablocks(g.N, NPB)), dim3(ADJ_BLOCK), 0, st, L, tb, ab, omega1,
                     (const double *)adj, h.Ln);
  hipLaunchKernelGGL((k_adj_x<M>), dim3(ablocks(g.N, NPB)), dim3(ADJ_BLOCK), 0, st, L, ab);
  hipLaunchKernelGGL(k_adj_psi, dim3(ablocks(g.N, 64)), dim3(64), 0, st, L, ab);
  hipLaunchKernelGGL((k_adj_phi<M>), dim3(ablocks(g.N * (M + 1), 128)), dim3(128), 0, st, L, ab, 1.0 / omega - 0.5);
  const unsigned nb = ablocks(g.N, NPB);
  hipLaunchKernelGGL((k_adj_step<M>), dim3(nb), dim3(ADJ_BLOCK), 0, st, L, tb, ab, omega, omega1, adj);
  if (grad && R > 0)
    hipLaunchKernelGGL(k_adj_param_sum, dim3(3 * R), dim3(PSUM_BLOCK), 0, st, (const double *)h.part, (int64_t)nb,
                       grad);
  return hipGetLastError();
}

template <int M>
hipError_t adj_macros_m(const Geom &g, const Tables *tb, const double *P, const double *T0, const double *w_rho,
                        const double *w_u, const double *w_T, const double *w_P, const double *w_Y, double *adj,
                        hipStream_t st) {
  const ALat L = make_alat(g);
  hipLaunchKernelGGL((k_adj_macros<M>), dim3(ablocks(g.N, NPB)), dim3(ADJ_BLOCK), 0, st, L, tb, P, T0, w_rho, w_u,
                     w_T, w_P, w_Y, adj);
  return hipGetLastError();
}

template <int M>
hipError_t adj_init_m(const Geom &g, const Tables *tb, const double *rho, const double *u, const double *T,
                      const double *Y, const double *lam, double *g_rho, double *g_u, double *g_T, double *g_Y,
                      hipStream_t st) {
  const ALat L = make_alat(g);
  hipLaunchKernelGGL((k_adj_init<M>), dim3(ablocks(g.N, NPB)), dim3(ADJ_BLOCK), 0, st, L, tb, rho, u, T, Y, lam,
                     g_rho, g_u, g_T, g_Y);
  return hipGetLastError();
}

}  // namespace

#define LBM_ADJ_DISPATCH(CALL)                                                                            \
  switch (g.M) {                                                                                          \
    case 2: return CALL(2); case 3: return CALL(3); case 4: return CALL(4); case 5: return CALL(5);        \
    case 6: return CALL(6); case 7: return CALL(7); case 8: return CALL(8); case 9: return CALL(9);        \
    case 10: return CALL(10);                                                                              \
    default: return hipErrorInvalidValue;                                                                  \
  }

hipError_t launch_adjoint_step(const Geom &g, const Tables *tb, const AdjBufHost &h, double omega, double omega1,
                               int R, double *adj, double *grad, hipStream_t st) {
#define LBM_CALL(MM) adj_step_m<MM>(g, tb, h, omega, omega1, R, adj, grad, st)
  LBM_ADJ_DISPATCH(LBM_CALL)
#undef LBM_CALL
}

hipError_t launch_adjoint_macros(const Geom &g, const Tables *tb, const double *P, const double *T0,
                                 const double *w_rho, const double *w_u, const double *w_T, const double *w_P,
                                 const double *w_Y, double *adj, hipStream_t st) {
#define LBM_CALL(MM) adj_macros_m<MM>(g, tb, P, T0, w_rho, w_u, w_T, w_P, w_Y, adj, st)
  LBM_ADJ_DISPATCH(LBM_CALL)
#undef LBM_CALL
}

hipError_t launch_adjoint_init(const Geom &g, const Tables *tb, const double *rho, const double *u, const double *T,
                               const double *Y, const double *lam, double *g_rho, double *g_u, double *g_T,
                               double *g_Y, hipStream_t st) {
#define LBM_CALL(MM) adj_init_m<MM>(g, tb, rho, u, T, Y, lam, g_rho, g_u, g_T, g_Y, st)
  LBM_ADJ_DISPATCH(LBM_CALL)
#undef LBM_CALL
}

}  // namespace lbm
