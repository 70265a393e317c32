/*
 * FP64 CPU oracle of the reactive-mixture lattice Boltzmann step.
 *
 * TEST INFRASTRUCTURE ONLY: the reference the HIP path is checked against.  Only
 * the tests, the smoke check and the benchmark's CPU-baseline leg may load it.
 *
 * Written from the paper (Sawant, Dorschner & Karlin, "Reactive mixtures with the
 * lattice Boltzmann model"): Sec. 2 (species LBM), Sec. 3 (mixture f and energy g),
 * Sec. 4 (coupling loop), Sec. 5.1 (boundary treatment of the 1D flame).  Each
 * function names the equation it follows.  Plain loops in double precision, in the
 * paper's order; nothing is fused or reordered beyond the written definitions.
 *
 * Readings of points the paper leaves open (listed with reasons in the design
 * notes of the repository):
 *   - lattice units dx = dt = 1; specific energies scaled by kappa = (dt/dx)^2,
 *     so that R_a T in lattice units is kappa R_U T / m_a;
 *   - thermo data: single-range NASA-7 polynomials (formation enthalpy included),
 *     standard state T0 = 298.15 K, P0 (Sec. 4);
 *   - production rates: mass action with integer orders equal to the
 *     stoichiometric coefficients, reverse rate from the equilibrium constant of
 *     the NASA-7 Gibbs function, CGS units (the paper delegates this to Cantera);
 *   - the reaction source carries weight dt as printed in eq. (finalNumerical-
 *     Equations), evaluated at the pre-collision state;
 *   - derivatives in X and q^corr: isotropic lattice gradient
 *     (1/theta) sum_i w_i c_i phi(x + c_i) (Thampi et al.), applied twice for X,
 *     no summation over alpha in X_alpha;
 *   - P^eq = rho R T I + rho u u (second moment of the product-form f^eq);
 *   - open faces: ghost populations are the equilibria at the adjacent boundary
 *     node's (rho_a, u, T), with u = 0 on a zero-velocity face; gradients use the
 *     boundary node's value outside the lattice (zero gradient);
 *   - u_a := u when |rho_a| < 1e-300;
 *   - temperature by Newton from the stored temperature, |dT| <= 1e-12 T, at
 *     most 50 iterations.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#define Q ORC_Q
#define MAXM ORC_MAXM

/* Arithmetic type of every quantity that depends on the state or on the Arrhenius
 * parameters.  Plain double here.  The reverse sweep (oracle_ad.cpp) compiles this
 * same file with a type that records each operation on a tape in its place, so that
 * its derivatives come from exactly these steps.  ORC_VAL gives the double value. */
#ifndef ORC_REAL
typedef double real;
#define ORC_VAL(x) (x)
#endif

static const double R_UNIV = 8.314462618;   /* J/(mol K) */
static const double THETA = 1.0 / 3.0;      /* lattice reference temperature (Sec. 3) */

/* ---- D3Q27 lattice (Sec. 2, after eq. sumfDotc) ---------------------------------- */
static int CX(int i) { return i % 3 - 1; }
static int CY(int i) { return (i / 3) % 3 - 1; }
static int CZ(int i) { return i / 9 - 1; }
static int CI(int i, int a) { return a == 0 ? CX(i) : (a == 1 ? CY(i) : CZ(i)); }

/* one-dimensional weights w_0 = 1 - theta, w_{+-1} = theta/2 (Sec. 3, after eq. giqeq) */
static double w1d(int c) { return c == 0 ? 1.0 - THETA : 0.5 * THETA; }
static double weight(int i) { return w1d(CX(i)) * w1d(CY(i)) * w1d(CZ(i)); }

typedef struct {
  /* O1: moments */
  real rho, j[3], u[3], Pt[3][3], rhoE, q[3];
  real rho_a[MAXM], j_a[MAXM][3], u_a[MAXM][3], Y[MAXM];
  /* O2: temperature and thermodynamics */
  real T, m, zeta, zeta_a[MAXM], P, H, H_a[MAXM];
  int newton_iters;
  /* O3: chemistry */
  real rdot[MAXM];
  /* O4: Stefan-Maxwell */
  real K[MAXM][MAXM], inv_tau[MAXM], beta[MAXM], du[MAXM][3];
  /* O5/O6: non-local fields */
  real phi[3], psi[3], X[3], gradY[MAXM][3];
} node_t;

struct orc_sim {
  orc_problem p;
  double molar_mass[MAXM], nasa7[MAXM][7], diff[MAXM][MAXM];
  int32_t nu_reac[ORC_MAXR][MAXM], nu_prod[ORC_MAXR][MAXM];
  real arrh[ORC_MAXR][3];
  uint8_t reversible[ORC_MAXR];
  int64_t N;
  int S;
  real *pop;      /* [S][Q][N] pre-collision, current time */
  real *post;     /* [S][Q][N] post-collision of the last step */
  double *Tstore; /* [N] temperature, Newton start value */
  node_t *nd;     /* [N] per-node quantities of the last step */
  real *scratch;  /* [N] */
};

/* ---- thermodynamics (Sec. 3 eq. specHa, Umix; NASA-7 form) ------------------------- */
static real cp_R(const double *a, real T) {
  return a[0] + a[1] * T + a[2] * T * T + a[3] * T * T * T + a[4] * T * T * T * T;
}
static real h_RT(const double *a, real T) {
  return a[0] + a[1] * T / 2.0 + a[2] * T * T / 3.0 + a[3] * T * T * T / 4.0 +
         a[4] * T * T * T * T / 5.0 + a[5] / T;
}
static real s_R(const double *a, real T) {
  return a[0] * log(T) + a[1] * T + a[2] * T * T / 2.0 + a[3] * T * T * T / 3.0 +
         a[4] * T * T * T * T / 4.0 + a[6];
}
/* lattice specific gas constant R_a = kappa R_U / m_a (per K), m_a in kg/mol */
static double gas_const(const orc_sim *s, int a) {
  return s->p.kappa * R_UNIV / (s->molar_mass[a] * 1e-3);
}
/* U_a = U_a^0 + int C_v: the NASA-7 enthalpy already contains the formation part */
static real spec_U(const orc_sim *s, int a, real T) {
  return gas_const(s, a) * T * (h_RT(s->nasa7[a], T) - 1.0);
}
static real spec_H(const orc_sim *s, int a, real T) {
  return gas_const(s, a) * T * h_RT(s->nasa7[a], T);
}
static real spec_Cv(const orc_sim *s, int a, real T) {
  return gas_const(s, a) * (cp_R(s->nasa7[a], T) - 1.0);
}

/* ---- product-form functions (eq. phis) and populations (eqs. feq, fstar, fsource) -- */
static real psi1d(int c, real xi, real zeta) {
  const real s = xi * xi + zeta;
  if (c == 0) return 1.0 - s;
  if (c == 1) return 0.5 * (xi + s);
  return 0.5 * (-xi + s);
}
static real product_form(int i, real dens, const real v[3], real zeta) {
  return dens * psi1d(CX(i), v[0], zeta) * psi1d(CY(i), v[1], zeta) * psi1d(CZ(i), v[2], zeta);
}

/* ---- Grad approximation for g (eqs. gieq, giqeq) ---------------------------------- */
static real grad_form(int i, real rhoE, const real q[3], const real Rt[3][3]) {
  real qc = 0.0, contr = 0.0;
  for (int a = 0; a < 3; ++a) qc += q[a] * CI(i, a);
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) {
      const real lhs = Rt[a][b] - (a == b ? rhoE * THETA : (real)0.0);
      const double rhs = CI(i, a) * CI(i, b) - (a == b ? THETA : 0.0);
      contr += lhs * rhs;
    }
  return weight(i) * (rhoE + qc / THETA + contr / (2.0 * THETA * THETA));
}

/* equilibrium energy flux and second moment (eqs. geq1mom, geq2mom) with
 * P^eq = rho R T I + rho u u */
static void energy_eq_moments(real rho, const real u[3], real zeta, real H,
                              real qeq[3], real Peq[3][3], real Req[3][3]) {
  const real usq = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
  const real P = rho * zeta;
  for (int a = 0; a < 3; ++a) {
    qeq[a] = (H + usq / 2.0) * rho * u[a];
    for (int b = 0; b < 3; ++b) {
      Peq[a][b] = (a == b ? rho * zeta : (real)0.0) + rho * u[a] * u[b];
      Req[a][b] = (H + usq / 2.0) * Peq[a][b] + P * u[a] * u[b];
    }
  }
}

/* ---- temperature from energy (eq. temperature), Newton ----------------------------- */
static int temperature(const orc_sim *s, const real *Y, real e_target, double T_start,
                       real *T_out) {
  real T = T_start;
  for (int it = 1; it <= 50; ++it) {
    real e = -e_target, de = 0.0;
    for (int a = 0; a < s->p.M; ++a) {
      e += Y[a] * spec_U(s, a, T);
      de += Y[a] * spec_Cv(s, a, T);
    }
    const real dT = -e / de;
    T += dT;
    if (fabs(dT) <= 1e-12 * fabs(T)) {
      *T_out = T;
      return it;
    }
  }
  *T_out = T;
  return -1;
}

/* ---- production rates (Sec. 4 item 3; mass action with K_c from NASA-7 Gibbs) ----- */
static void production_rates(const orc_sim *s, const real *rho_a, real T, real *rdot) {
  const int M = s->p.M;
  real c[MAXM], g[MAXM], wdot[MAXM];
  for (int a = 0; a < M; ++a) {
    c[a] = rho_a[a] * s->p.rho_ref / s->molar_mass[a];           /* mol/cm^3 */
    g[a] = h_RT(s->nasa7[a], T) - s_R(s->nasa7[a], T);           /* G_a/(R_U T) */
    wdot[a] = 0.0;
  }
  for (int k = 0; k < s->p.R; ++k) {
    const real A = s->arrh[k][0], b = s->arrh[k][1], Ta = s->arrh[k][2];
    const real kf = A * pow(T, b) * exp(-Ta / T);
    real fwd = kf;
    for (int a = 0; a < M; ++a)
      for (int n = 0; n < s->nu_reac[k][a]; ++n) fwd *= c[a];
    real rev = 0.0;
    if (s->reversible[k]) {
      double dnu = 0.0;
      real dG = 0.0;
      for (int a = 0; a < M; ++a) {
        const double nu = (double)(s->nu_prod[k][a] - s->nu_reac[k][a]);
        dnu += nu;
        dG += nu * g[a];
      }
      const real c0 = s->p.p0 / (R_UNIV * T) * 1e-6;              /* mol/cm^3 */
      const real Kc = exp(-dG) * pow(c0, dnu);
      const real kr = kf / Kc;
      rev = kr;
      for (int a = 0; a < M; ++a)
        for (int n = 0; n < s->nu_prod[k][a]; ++n) rev *= c[a];
    }
    const real qk = fwd - rev;
    for (int a = 0; a < M; ++a) wdot[a] += (double)(s->nu_prod[k][a] - s->nu_reac[k][a]) * qk;
  }
  /* g/(cm^3 s) -> lattice density per step */
  for (int a = 0; a < M; ++a) rdot[a] = s->molar_mass[a] * wdot[a] * s->p.dt_phys / s->p.rho_ref;
}

/* ---- Stefan-Maxwell relaxation (eqs. fStar, tauab, transform1) ---------------------- */
/* binary diffusivity at temperature T: the given constant, or with a temperature
 * exponent the power law D_ab (T / T_ref)^n (a stand-in for the temperature-dependent
 * transport data of Sec. 3) */
static real diffusivity(const orc_sim *s, int a, int b, real T) {
  if (s->p.diff_T_exp == 0.0) return s->diff[a][b];
  return s->diff[a][b] * pow(T / s->p.diff_T_ref, s->p.diff_T_exp);
}

/* relaxation rates at temperature T: the given omega, omega1, or with a temperature
 * exponent the rates whose viscosity and conductivity factors 1/omega - 1/2 and
 * 1/omega1 - 1/2 (eqs. mu, lambda) scale as (T / T_ref)^n (a stand-in for the
 * temperature-dependent transport data of Sec. 3) */
static void relaxation_rates(const orc_sim *s, real T, real *om, real *om1) {
  if (s->p.visc_T_exp == 0.0) {
    *om = s->p.omega;
    *om1 = s->p.omega1;
    return;
  }
  const real sc = pow(T / s->p.visc_T_ref, s->p.visc_T_exp);
  *om = 1.0 / (0.5 + (1.0 / s->p.omega - 0.5) * sc);
  *om1 = 1.0 / (0.5 + (1.0 / s->p.omega1 - 0.5) * sc);
}

/* K_ab = 1/tau_ab with tau_ab = (m_a m_b / (m R_U T)) D_ab, written with lattice
 * R_a T: 1/tau_ab = (R_a T)(R_b T) / ((R T) D_ab). */
static void relaxation(const orc_sim *s, const real *Y, const real *zeta_a, real zeta, real T,
                       real K[MAXM][MAXM], real *inv_tau, real *beta) {
  const int M = s->p.M;
  for (int a = 0; a < M; ++a)
    for (int b = 0; b < M; ++b)
      K[a][b] = (a == b) ? (real)0.0 : zeta_a[a] * zeta_a[b] / (zeta * diffusivity(s, a, b, T));
  for (int a = 0; a < M; ++a) {
    inv_tau[a] = 0.0;
    for (int b = 0; b < M; ++b)
      if (b != a) inv_tau[a] += Y[b] * K[a][b];
    const real tau = 1.0 / inv_tau[a];
    beta[a] = 1.0 / (2.0 * tau + 1.0);
  }
}

/* (1 + 1/(2 tau_a)) du_a - 1/2 sum_{b!=a} (1/tau_ab) Y_b du_b = u_a - u, for each
 * spatial component; Gaussian elimination (the matrix is strictly diagonally
 * dominant by rows, so no pivoting). */
static void diffusion_velocities(int M, real K[MAXM][MAXM], const real *inv_tau,
                                 const real *Y, const real rhs[MAXM][3], real du[MAXM][3]) {
  real A[MAXM][MAXM], B[MAXM][3];
  for (int a = 0; a < M; ++a) {
    for (int b = 0; b < M; ++b) A[a][b] = (a == b) ? 1.0 + 0.5 * inv_tau[a] : -0.5 * K[a][b] * Y[b];
    for (int d = 0; d < 3; ++d) B[a][d] = rhs[a][d];
  }
  for (int k = 0; k < M; ++k) {
    for (int r = k + 1; r < M; ++r) {
      const real l = A[r][k] / A[k][k];
      for (int c = k; c < M; ++c) A[r][c] -= l * A[k][c];
      for (int d = 0; d < 3; ++d) B[r][d] -= l * B[k][d];
    }
  }
  for (int r = M - 1; r >= 0; --r)
    for (int d = 0; d < 3; ++d) {
      real v = B[r][d];
      for (int c = r + 1; c < M; ++c) v -= A[r][c] * du[c][d];
      du[r][d] = v / A[r][r];
    }
}

/* ---- lattice neighbourhood ---------------------------------------------------------- */
static int64_t node_index(const orc_sim *s, int x, int y, int z) {
  return (int64_t)x + (int64_t)s->p.nx * ((int64_t)y + (int64_t)s->p.ny * z);
}
static void node_coords(const orc_sim *s, int64_t n, int *x, int *y, int *z) {
  *x = (int)(n % s->p.nx);
  *y = (int)((n / s->p.nx) % s->p.ny);
  *z = (int)(n / ((int64_t)s->p.nx * s->p.ny));
}
static int dim(const orc_sim *s, int a) { return a == 0 ? s->p.nx : (a == 1 ? s->p.ny : s->p.nz); }

/* neighbour for gradients: periodic wrap, or the boundary node outside an open face
 * (zero gradient), or its mirror image outside a symmetry face.  *mirror gets a bit
 * per axis whose symmetry face the neighbour lies beyond. */
static int64_t grad_neighbour(const orc_sim *s, int64_t n, int i, int *mirror) {
  int xyz[3];
  node_coords(s, n, &xyz[0], &xyz[1], &xyz[2]);
  *mirror = 0;
  for (int a = 0; a < 3; ++a) {
    const int L = dim(s, a);
    int v = xyz[a] + CI(i, a);
    if (s->p.bc[2 * a] == ORC_BC_PERIODIC) {
      v = ((v % L) + L) % L;
    } else if (v < 0) {
      if (s->p.bc[2 * a] == ORC_BC_SYMMETRY) *mirror |= 1 << a;
      v = -1 - v;
    } else if (v >= L) {
      if (s->p.bc[2 * a + 1] == ORC_BC_SYMMETRY) *mirror |= 1 << a;
      v = 2 * L - 1 - v;
    }
    xyz[a] = v;
  }
  return node_index(s, xyz[0], xyz[1], xyz[2]);
}

/* isotropic lattice gradient, component alpha, of a nodal field that is a scalar
 * (vec_axis < 0) or the vec_axis component of a vector: that component changes sign
 * in the mirror image beyond a symmetry face normal to its axis */
static real iso_grad_v(const orc_sim *s, const real *field, int64_t n, int alpha, int vec_axis) {
  real acc = 0.0;
  for (int i = 0; i < Q; ++i) {
    int mirror;
    real v = field[grad_neighbour(s, n, i, &mirror)];
    if (vec_axis >= 0 && (mirror >> vec_axis & 1)) v = -v;
    acc += weight(i) * CI(i, alpha) * v;
  }
  return acc / THETA;
}
static real iso_grad(const orc_sim *s, const real *field, int64_t n, int alpha) {
  return iso_grad_v(s, field, n, alpha, -1);
}

/* ---- O1-O5: local part of the step at one node ---------------------------------------- */
static uint32_t node_local(const orc_sim *s, int64_t n, double T_start, node_t *d, int with_source) {
  const int M = s->p.M, S = s->S;
  const int64_t N = s->N;
  const real *pf = s->pop + (int64_t)(M - 1) * Q * N;   /* mixture f */
  const real *pg = s->pop + (int64_t)M * Q * N;         /* energy g */
  uint32_t anom = 0;
  (void)S;
  memset(d, 0, sizeof(*d));

  /* mixture moments (Sec. 3): rho, rho u, pressure tensor, rho E, q */
  for (int i = 0; i < Q; ++i) {
    const real f = pf[(int64_t)i * N + n];
    const real g = pg[(int64_t)i * N + n];
    d->rho += f;
    d->rhoE += g;
    for (int a = 0; a < 3; ++a) {
      d->j[a] += f * CI(i, a);
      d->q[a] += g * CI(i, a);
      for (int b = 0; b < 3; ++b) d->Pt[a][b] += f * CI(i, a) * CI(i, b);
    }
  }
  for (int a = 0; a < 3; ++a) d->u[a] = d->j[a] / d->rho;

  /* species moments (eq. Pa); the last species is slaved (eq. strongest) */
  real rho_sum = 0.0, j_sum[3] = {0.0, 0.0, 0.0};
  for (int sp = 0; sp < M - 1; ++sp) {
    const real *pa = s->pop + (int64_t)sp * Q * N;
    for (int i = 0; i < Q; ++i) {
      const real f = pa[(int64_t)i * N + n];
      d->rho_a[sp] += f;
      for (int a = 0; a < 3; ++a) d->j_a[sp][a] += f * CI(i, a);
    }
    rho_sum += d->rho_a[sp];
    for (int a = 0; a < 3; ++a) j_sum[a] += d->j_a[sp][a];
  }
  d->rho_a[M - 1] = d->rho - rho_sum;
  for (int a = 0; a < 3; ++a) d->j_a[M - 1][a] = d->j[a] - j_sum[a];
  for (int sp = 0; sp < M; ++sp) {
    d->Y[sp] = d->rho_a[sp] / d->rho;
    for (int a = 0; a < 3; ++a)
      d->u_a[sp][a] = fabs(d->rho_a[sp]) < 1e-300 ? d->u[a] : d->j_a[sp][a] / d->rho_a[sp];
  }
  if (!(d->rho > 0.0) || !(d->rho_a[M - 1] > 0.0)) anom |= ORC_ANOM_NEG_DENSITY;

  /* O2: temperature from E - u^2/2 (eq. temperature), then EOS (eq. eosIdealGas) */
  const real usq = d->u[0] * d->u[0] + d->u[1] * d->u[1] + d->u[2] * d->u[2];
  const real E = d->rhoE / d->rho;
  d->newton_iters = temperature(s, d->Y, E - usq / 2.0, T_start, &d->T);
  if (d->newton_iters < 0) anom |= ORC_ANOM_NEWTON;
  real inv_m = 0.0;
  for (int sp = 0; sp < M; ++sp) inv_m += d->Y[sp] / s->molar_mass[sp];
  d->m = 1.0 / inv_m;
  d->zeta = s->p.kappa * R_UNIV * d->T / (d->m * 1e-3);
  d->P = d->rho * d->zeta;
  d->H = 0.0;
  for (int sp = 0; sp < M; ++sp) {
    d->zeta_a[sp] = gas_const(s, sp) * d->T;
    d->H_a[sp] = spec_H(s, sp, d->T);
    d->H += d->Y[sp] * d->H_a[sp];
  }
  if (!with_source) return anom;

  /* O3: chemistry */
  production_rates(s, d->rho_a, d->T, d->rdot);

  /* O4: relaxation times and diffusion velocities */
  relaxation(s, d->Y, d->zeta_a, d->zeta, d->T, d->K, d->inv_tau, d->beta);
  real rhs[MAXM][3];
  for (int sp = 0; sp < M; ++sp)
    for (int a = 0; a < 3; ++a) rhs[sp][a] = d->u_a[sp][a] - d->u[a];
  diffusion_velocities(M, d->K, d->inv_tau, d->Y, rhs, d->du);

  /* O5: argument of the isotropy correction (eq. Xalpha) */
  for (int a = 0; a < 3; ++a)
    d->phi[a] = d->rho * d->u[a] * (1.0 - 3.0 * d->zeta) - d->rho * d->u[a] * d->u[a] * d->u[a];

  if (!isfinite(d->T) || !isfinite(d->rho) || !isfinite(d->rhoE)) anom |= ORC_ANOM_NONFINITE;
  return anom;
}

/* ---- O7: collision at one node (eqs. finalNumericalEquations, f, g) -------------------- */
static void collide(orc_sim *s, int64_t n) {
  const int M = s->p.M;
  const int64_t N = s->N;
  const node_t *d = &s->nd[n];
  real om, om1;
  relaxation_rates(s, d->T, &om, &om1);

  /* mixture f (eq. f) with the isotropy correction A_i . X (eq. Ai) */
  {
    const real *pf = s->pop + (int64_t)(M - 1) * Q * N;
    real *of = s->post + (int64_t)(M - 1) * Q * N;
    for (int i = 0; i < Q; ++i) {
      const real f = pf[(int64_t)i * N + n];
      const real feq = product_form(i, d->rho, d->u, d->zeta);
      const int c2 = CX(i) * CX(i) + CY(i) * CY(i) + CZ(i) * CZ(i);
      real AX = 0.0;
      if (c2 == 1)
        for (int a = 0; a < 3; ++a) AX += 0.5 * CI(i, a) * d->X[a];
      of[(int64_t)i * N + n] = f + om * (feq - f) + AX;
    }
  }

  /* species a < M (eq. finalNumericalEquations with F_ai of eq. fStar) */
  for (int sp = 0; sp < M - 1; ++sp) {
    const real *pa = s->pop + (int64_t)sp * Q * N;
    real *oa = s->post + (int64_t)sp * Q * N;
    for (int i = 0; i < Q; ++i) {
      const real f = pa[(int64_t)i * N + n];
      const real feq = product_form(i, d->rho_a[sp], d->u, d->zeta_a[sp]);
      real F = 0.0;
      for (int b = 0; b < M; ++b) {
        if (b == sp) continue;
        real ub[3];
        for (int a = 0; a < 3; ++a) ub[a] = d->u[a] + d->du[b][a];
        const real feq_b = product_form(i, d->rho_a[b], d->u, d->zeta_a[b]);
        const real fst_b = product_form(i, d->rho_a[b], ub, d->zeta_a[b]);
        F += d->K[sp][b] * (feq_b - fst_b);
      }
      F *= d->Y[sp];
      const real src = product_form(i, d->rdot[sp], d->u, d->zeta_a[sp]);   /* eq. fsource */
      oa[(int64_t)i * N + n] = f + 2.0 * d->beta[sp] * (feq - f) + (d->beta[sp] - 1.0) * F + src;
    }
  }

  /* energy g (eq. g) */
  {
    const real *pg = s->pop + (int64_t)M * Q * N;
    real *og = s->post + (int64_t)M * Q * N;
    real qeq[3], Peq[3][3], Req[3][3];
    energy_eq_moments(d->rho, d->u, d->zeta, d->H, qeq, Peq, Req);
    real hyd[3] = {0.0, 0.0, 0.0}, hgrad[3] = {0.0, 0.0, 0.0};
    for (int sp = 0; sp < M; ++sp)
      for (int a = 0; a < 3; ++a) {
        hyd[a] += d->H_a[sp] * d->Y[sp] * d->du[sp][a];
        hgrad[a] += d->H_a[sp] * d->gradY[sp][a];
      }
    real qstar[3];
    for (int a = 0; a < 3; ++a) {
      real uPdiff = 0.0;   /* (u . (P - P^eq))_a */
      for (int b = 0; b < 3; ++b) uPdiff += d->u[b] * (d->Pt[b][a] - Peq[b][a]);
      const real qdiff = (om1 / (om - om1)) * d->rho * hyd[a];                 /* eq. qdiff */
      const real qcorr = 0.5 * ((om1 - 2.0) / (om1 - om)) * d->P * hgrad[a];  /* eq. corrFourier */
      qstar[a] = d->q[a] - uPdiff + qdiff + qcorr;                               /* eq. gstareq1mom */
    }
    for (int i = 0; i < Q; ++i) {
      const real g = pg[(int64_t)i * N + n];
      const real geq = grad_form(i, d->rhoE, qeq, Req);
      const real gst = grad_form(i, d->rhoE, qstar, Req);
      og[(int64_t)i * N + n] = g + om1 * (geq - g) + (om - om1) * (gst - g);
    }
  }
}

/* ---- O8: ghost equilibrium at an open face (Sec. 5.1) -------------------------------- */
static real ghost_value(const orc_sim *s, int set, int i, const node_t *d, int zero_u) {
  const int M = s->p.M;
  real ug[3];
  for (int a = 0; a < 3; ++a) ug[a] = zero_u ? (real)0.0 : d->u[a];
  if (set < M - 1) return product_form(i, d->rho_a[set], ug, d->zeta_a[set]);
  if (set == M - 1) return product_form(i, d->rho, ug, d->zeta);
  const real usq = ug[0] * ug[0] + ug[1] * ug[1] + ug[2] * ug[2];
  real U = 0.0;
  for (int sp = 0; sp < M; ++sp) U += d->Y[sp] * spec_U(s, sp, d->T);
  const real rhoE = d->rho * (U + usq / 2.0);
  real qeq[3], Peq[3][3], Req[3][3];
  energy_eq_moments(d->rho, ug, d->zeta, d->H, qeq, Peq, Req);
  return grad_form(i, rhoE, qeq, Req);
}

/* direction i with the components along the axes in mask reversed */
static int mirror_dir(int i, int mask) {
  int c[3] = {CX(i), CY(i), CZ(i)};
  for (int a = 0; a < 3; ++a)
    if (mask >> a & 1) c[a] = -c[a];
  return (c[0] + 1) + 3 * (c[1] + 1) + 9 * (c[2] + 1);
}

/* O8: pull streaming.  A source beyond an open face is the equilibrium at the boundary
 * node (Sec. 5.1).  Beyond a symmetry face the source is the mirror image: the
 * population of the mirrored direction at the mirrored node, post-collision with its
 * corrections; beyond a symmetry and an open face, the equilibrium of the mirrored
 * direction at the mirrored boundary node. */
static void stream_node(orc_sim *s, int64_t n) {
  const int S = s->S;
  const int64_t N = s->N;
  int xyz[3];
  node_coords(s, n, &xyz[0], &xyz[1], &xyz[2]);
  for (int i = 0; i < Q; ++i) {
    int src[3], open_out = 0, zero_u = 0, mirror = 0;
    for (int a = 0; a < 3; ++a) {
      const int L = dim(s, a);
      int v = xyz[a] - CI(i, a);
      if (s->p.bc[2 * a] == ORC_BC_PERIODIC) {
        v = ((v % L) + L) % L;
      } else if (v < 0) {
        if (s->p.bc[2 * a] == ORC_BC_SYMMETRY) {
          mirror |= 1 << a;
        } else {
          open_out = 1;
          if (s->p.bc[2 * a] == ORC_BC_OPEN_U0) zero_u = 1;
        }
        v = -1 - v;
      } else if (v >= L) {
        if (s->p.bc[2 * a + 1] == ORC_BC_SYMMETRY) {
          mirror |= 1 << a;
        } else {
          open_out = 1;
          if (s->p.bc[2 * a + 1] == ORC_BC_OPEN_U0) zero_u = 1;
        }
        v = 2 * L - 1 - v;
      }
      src[a] = v;
    }
    const int64_t m = node_index(s, src[0], src[1], src[2]);
    const int im = mirror_dir(i, mirror);
    for (int set = 0; set < S; ++set) {
      real v;
      if (open_out)
        v = ghost_value(s, set, im, &s->nd[m], zero_u);
      else
        v = s->post[((int64_t)set * Q + im) * N + m];
      s->pop[((int64_t)set * Q + i) * N + n] = v;
    }
  }
}

/* ---- public driver -------------------------------------------------------------------- */
orc_sim *orc_create(const orc_problem *p) {
  if (p->M < 2 || p->M > MAXM || p->R < 0 || p->R > ORC_MAXR) return NULL;
  if (p->nx < 1 || p->ny < 1 || p->nz < 1) return NULL;
  for (int a = 0; a < 3; ++a) {
    const int lo = p->bc[2 * a], hi = p->bc[2 * a + 1];
    if ((lo == ORC_BC_PERIODIC) != (hi == ORC_BC_PERIODIC)) return NULL;
  }
  if (p->omega == p->omega1) return NULL;   /* the printed q^diff and q^corr prefactors are singular */
  if (p->diff_T_exp != 0.0 && !(p->diff_T_ref > 0.0)) return NULL;
  if (p->visc_T_exp != 0.0 && !(p->visc_T_ref > 0.0)) return NULL;
  orc_sim *s = (orc_sim *)calloc(1, sizeof(orc_sim));
  s->p = *p;
  const int M = p->M;
  for (int a = 0; a < M; ++a) {
    s->molar_mass[a] = p->molar_mass[a];
    for (int k = 0; k < 7; ++k) s->nasa7[a][k] = p->nasa7[a * 7 + k];
    for (int b = 0; b < M; ++b) s->diff[a][b] = p->diff[a * M + b];
  }
  for (int k = 0; k < p->R; ++k) {
    for (int a = 0; a < M; ++a) {
      s->nu_reac[k][a] = p->nu_reac[k * M + a];
      s->nu_prod[k][a] = p->nu_prod[k * M + a];
    }
    for (int c = 0; c < 3; ++c) s->arrh[k][c] = p->arrhenius[k * 3 + c];
    s->reversible[k] = p->reversible[k];
  }
  s->p.molar_mass = NULL;
  s->p.nasa7 = s->p.diff = s->p.arrhenius = NULL;
  s->p.nu_reac = s->p.nu_prod = NULL;
  s->p.reversible = NULL;
  s->N = (int64_t)p->nx * p->ny * p->nz;
  s->S = M + 1;
  s->pop = (real *)calloc((size_t)s->S * Q * s->N, sizeof(real));
  s->post = (real *)calloc((size_t)s->S * Q * s->N, sizeof(real));
  s->Tstore = (double *)calloc((size_t)s->N, sizeof(double));
  s->nd = (node_t *)calloc((size_t)s->N, sizeof(node_t));
  s->scratch = (real *)calloc((size_t)s->N, sizeof(real));
  if (!s->pop || !s->post || !s->Tstore || !s->nd || !s->scratch) {
    orc_destroy(s);
    return NULL;
  }
  return s;
}

void orc_destroy(orc_sim *s) {
  if (!s) return;
  free(s->pop);
  free(s->post);
  free(s->Tstore);
  free(s->nd);
  free(s->scratch);
  free(s);
}

/* initial state: equilibrium populations at the given fields (no non-equilibrium part) */
static void init_fields(orc_sim *s, const real *rho, const real *u, const real *T, const real *Y) {
  const int M = s->p.M;
  const int64_t N = s->N;
  for (int64_t n = 0; n < N; ++n) {
    node_t d;
    memset(&d, 0, sizeof(d));
    d.rho = rho[n];
    for (int a = 0; a < 3; ++a) d.u[a] = u[a * N + n];
    d.T = T[n];
    real inv_m = 0.0;
    for (int sp = 0; sp < M; ++sp) {
      d.Y[sp] = Y[sp * N + n];
      d.rho_a[sp] = d.rho * d.Y[sp];
      inv_m += d.Y[sp] / s->molar_mass[sp];
      d.zeta_a[sp] = gas_const(s, sp) * d.T;
      d.H_a[sp] = spec_H(s, sp, d.T);
      d.H += d.Y[sp] * d.H_a[sp];
    }
    d.m = 1.0 / inv_m;
    d.zeta = s->p.kappa * R_UNIV * d.T / (d.m * 1e-3);
    d.P = d.rho * d.zeta;
    for (int set = 0; set < s->S; ++set)
      for (int i = 0; i < Q; ++i)
        s->pop[((int64_t)set * Q + i) * N + n] = ghost_value(s, set, i, &d, 0);
    s->Tstore[n] = ORC_VAL(T[n]);
  }
}

#ifndef ORC_REAL
void orc_init(orc_sim *s, const double *rho, const double *u, const double *T, const double *Y) {
  init_fields(s, rho, u, T, Y);
}
#endif

static void nonlocal_fields(orc_sim *s, int nthreads) {
  const int M = s->p.M;
  const int64_t N = s->N;
  real *fld = s->scratch;
  (void)nthreads;
  /* psi_alpha = (1/omega - 1/2) d_alpha phi_alpha ; X_alpha = -d_alpha psi_alpha (eq. Xalpha).
   * phi_alpha is odd under a mirror normal to alpha (it is odd in u_alpha), psi_alpha even */
  for (int a = 0; a < 3; ++a) {
    for (int64_t n = 0; n < N; ++n) fld[n] = s->nd[n].phi[a];
#pragma omp parallel for schedule(static) num_threads(nthreads)
    for (int64_t n = 0; n < N; ++n) {
      real om, om1;
      relaxation_rates(s, s->nd[n].T, &om, &om1);
      s->nd[n].psi[a] = (1.0 / om - 0.5) * iso_grad_v(s, fld, n, a, a);
    }
  }
  for (int a = 0; a < 3; ++a) {
    for (int64_t n = 0; n < N; ++n) fld[n] = s->nd[n].psi[a];
#pragma omp parallel for schedule(static) num_threads(nthreads)
    for (int64_t n = 0; n < N; ++n) s->nd[n].X[a] = -iso_grad(s, fld, n, a);   /* psi is even under mirrors */
  }
  /* gradients of the mass fractions (eq. corrFourier) */
  for (int sp = 0; sp < M; ++sp) {
    for (int64_t n = 0; n < N; ++n) fld[n] = s->nd[n].Y[sp];
#pragma omp parallel for schedule(static) num_threads(nthreads)
    for (int64_t n = 0; n < N; ++n)
      for (int a = 0; a < 3; ++a) s->nd[n].gradY[sp][a] = iso_grad(s, fld, n, a);
  }
}

uint32_t orc_step(orc_sim *s, int32_t nsteps, int32_t nthreads) {
  const int64_t N = s->N;
  uint32_t anom_all = 0;
  if (nthreads < 1) nthreads = 1;
  for (int step = 0; step < nsteps; ++step) {
    uint32_t anom = 0;
#pragma omp parallel for schedule(static) num_threads(nthreads) reduction(| : anom)
    for (int64_t n = 0; n < N; ++n) anom |= node_local(s, n, s->Tstore[n], &s->nd[n], 1);
    nonlocal_fields(s, nthreads);
#pragma omp parallel for schedule(static) num_threads(nthreads)
    for (int64_t n = 0; n < N; ++n) collide(s, n);
#pragma omp parallel for schedule(static) num_threads(nthreads)
    for (int64_t n = 0; n < N; ++n) stream_node(s, n);
    for (int64_t n = 0; n < N; ++n) s->Tstore[n] = ORC_VAL(s->nd[n].T);
    anom_all |= anom;
  }
  return anom_all;
}

/* O9: the macroscopic fields of the current state (O1-O2 at every node) */
static uint32_t macros_fields(orc_sim *s, real *rho, real *u, real *T, real *P, real *Y) {
  const int M = s->p.M;
  const int64_t N = s->N;
  uint32_t anom = 0;
  for (int64_t n = 0; n < N; ++n) {
    node_t d;
    anom |= node_local(s, n, s->Tstore[n], &d, 0);
    if (rho) rho[n] = d.rho;
    if (u)
      for (int a = 0; a < 3; ++a) u[a * N + n] = d.u[a];
    if (T) T[n] = d.T;
    if (P) P[n] = d.P;
    if (Y)
      for (int sp = 0; sp < M; ++sp) Y[sp * N + n] = d.Y[sp];
  }
  return anom;
}

#ifndef ORC_REAL
uint32_t orc_macros(orc_sim *s, double *rho, double *u, double *T, double *P, double *Y) {
  return macros_fields(s, rho, u, T, P, Y);
}

/* Flame-front diagnostics of the current state (Sec. 5.2).  Displacement speed (eq. sd):
 *   S_d = [ -sum_a H_a rho_dot_a + div(lambda grad T) - rho (sum_a C_p,a Y_a du_a) . grad T ]
 *         / (rho C_p |grad T|),
 * with the conductivity of eq. lambda, lambda = (1/omega1 - 1/2) P C_p (dt = 1), the
 * mixture C_p = sum_a Y_a C_p,a, the diffusion velocities du_a of the Stefan-Maxwell
 * solve (eq. transform1), and the isotropic lattice gradient for grad and for each term
 * of div (reading R3; lambda dT/dx_alpha is odd under a mirror normal to alpha).  The
 * absolute speed is S_a = S_d + u . n with n = -grad T / |grad T|.  Where grad T = 0
 * both are set to 0.  w is the weight of a node in a mean over the surface T = T_iso:
 * max(0, 1 - |T - T_iso| / |grad T|), a hat one cell wide across the surface, which
 * turns the surface integral of eq. rmean into a sum over nodes.
 * out[3][N]: S_d, S_a, w.  totals[5]: sum w, sum w S_d, sum w S_a, sum w rho S_d,
 * sum w |x - centre| (the last over sum w is the mean radius of eq. rmean). */
uint32_t orc_flame_speeds(orc_sim *s, double T_iso, const double *centre, double *out, double *totals) {
  const int M = s->p.M;
  const int64_t N = s->N;
  uint32_t anom = 0;
  node_t *d = (node_t *)calloc((size_t)N, sizeof(node_t));
  double *T = (double *)malloc(sizeof(double) * (size_t)N);
  double *gT = (double *)malloc(sizeof(double) * 3 * (size_t)N);
  double *G = (double *)malloc(sizeof(double) * 3 * (size_t)N);
  double *lam = (double *)malloc(sizeof(double) * (size_t)N);
  double *cp = (double *)malloc(sizeof(double) * (size_t)N);
  for (int64_t n = 0; n < N; ++n) {
    anom |= node_local(s, n, s->Tstore[n], &d[n], 1);
    T[n] = d[n].T;
    cp[n] = 0.0;
    for (int sp = 0; sp < M; ++sp) cp[n] += d[n].Y[sp] * (spec_Cv(s, sp, T[n]) + gas_const(s, sp));
    double om, om1;
    relaxation_rates(s, T[n], &om, &om1);
    lam[n] = (1.0 / om1 - 0.5) * d[n].P * cp[n];
  }
  for (int64_t n = 0; n < N; ++n)
    for (int a = 0; a < 3; ++a) gT[a * N + n] = iso_grad(s, T, n, a);
  for (int a = 0; a < 3; ++a)
    for (int64_t n = 0; n < N; ++n) G[a * N + n] = lam[n] * gT[a * N + n];
  for (int k = 0; k < 5; ++k) totals[k] = 0.0;
  for (int64_t n = 0; n < N; ++n) {
    double div = 0.0;
    for (int a = 0; a < 3; ++a) div += iso_grad_v(s, G + a * N, n, a, a);
    double hrr = 0.0;
    for (int sp = 0; sp < M; ++sp) hrr -= d[n].H_a[sp] * d[n].rdot[sp];
    double flux = 0.0;   /* (sum_a C_p,a Y_a du_a) . grad T */
    for (int sp = 0; sp < M; ++sp) {
      const double c = (spec_Cv(s, sp, T[n]) + gas_const(s, sp)) * d[n].Y[sp];
      for (int a = 0; a < 3; ++a) flux += c * d[n].du[sp][a] * gT[a * N + n];
    }
    const double g2 = gT[n] * gT[n] + gT[N + n] * gT[N + n] + gT[2 * N + n] * gT[2 * N + n];
    const double mag = sqrt(g2);
    double Sd = 0.0, Sa = 0.0, w = 0.0;
    if (mag > 0.0) {
      Sd = (hrr + div - d[n].rho * flux) / (d[n].rho * cp[n] * mag);
      double un = 0.0;
      for (int a = 0; a < 3; ++a) un -= d[n].u[a] * gT[a * N + n] / mag;
      Sa = Sd + un;
      w = 1.0 - fabs(T[n] - T_iso) / mag;
      if (w < 0.0) w = 0.0;
    }
    out[n] = Sd;
    out[N + n] = Sa;
    out[2 * N + n] = w;
    int xyz[3];
    node_coords(s, n, &xyz[0], &xyz[1], &xyz[2]);
    double r2 = 0.0;
    for (int a = 0; a < 3; ++a) r2 += (xyz[a] - centre[a]) * (xyz[a] - centre[a]);
    totals[0] += w;
    totals[1] += w * Sd;
    totals[2] += w * Sa;
    totals[3] += w * d[n].rho * Sd;
    totals[4] += w * sqrt(r2);
  }
  free(d);
  free(T);
  free(gT);
  free(G);
  free(lam);
  free(cp);
  return anom;
}

#endif /* ORC_REAL */

void orc_get_state(const orc_sim *s, double *pop, double *T) {
  const int64_t n = (int64_t)s->S * Q * s->N;
  if (pop)
    for (int64_t k = 0; k < n; ++k) pop[k] = ORC_VAL(s->pop[k]);
  if (T) memcpy(T, s->Tstore, sizeof(double) * (size_t)s->N);
}

void orc_set_state(orc_sim *s, const double *pop, const double *T) {
  const int64_t n = (int64_t)s->S * Q * s->N;
  if (pop)
    for (int64_t k = 0; k < n; ++k) s->pop[k] = pop[k];
  if (T) memcpy(s->Tstore, T, sizeof(double) * (size_t)s->N);
}

void orc_get_post(const orc_sim *s, double *post) {
  const int64_t n = (int64_t)s->S * Q * s->N;
  for (int64_t k = 0; k < n; ++k) post[k] = ORC_VAL(s->post[k]);
}

void orc_get_field(const orc_sim *s, int32_t which, double *out) {
  const int M = s->p.M;
  const int64_t N = s->N;
  for (int64_t n = 0; n < N; ++n) {
    const node_t *d = &s->nd[n];
    switch (which) {
      case ORC_F_T: out[n] = ORC_VAL(d->T); break;
      case ORC_F_RDOT:
        for (int sp = 0; sp < M; ++sp) out[sp * N + n] = ORC_VAL(d->rdot[sp]);
        break;
      case ORC_F_DU:
        for (int sp = 0; sp < M; ++sp)
          for (int a = 0; a < 3; ++a) out[(sp * 3 + a) * N + n] = ORC_VAL(d->du[sp][a]);
        break;
      case ORC_F_BETA:
        for (int sp = 0; sp < M; ++sp) out[sp * N + n] = ORC_VAL(d->beta[sp]);
        break;
      case ORC_F_X:
        for (int a = 0; a < 3; ++a) out[a * N + n] = ORC_VAL(d->X[a]);
        break;
      case ORC_F_GRADY:
        for (int sp = 0; sp < M; ++sp)
          for (int a = 0; a < 3; ++a) out[(sp * 3 + a) * N + n] = ORC_VAL(d->gradY[sp][a]);
        break;
      case ORC_F_PHI:
        for (int a = 0; a < 3; ++a) out[a * N + n] = ORC_VAL(d->phi[a]);
        break;
      case ORC_F_PSI:
        for (int a = 0; a < 3; ++a) out[a * N + n] = ORC_VAL(d->psi[a]);
        break;
      case ORC_F_NEWTON: out[n] = (double)d->newton_iters; break;
      default: break;
    }
  }
}

/* ---- pieces exposed for unit pins ---------------------------------------------------- */
#ifndef ORC_REAL
void orc_product_form(double dens, const double *v, double zeta, double *out27) {
  for (int i = 0; i < Q; ++i) out27[i] = product_form(i, dens, v, zeta);
}

void orc_grad_form(double rhoE, const double *q, const double *R9, double *out27) {
  double Rt[3][3];
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) Rt[a][b] = R9[a * 3 + b];
  for (int i = 0; i < Q; ++i) out27[i] = grad_form(i, rhoE, q, Rt);
}

void orc_thermo(const orc_sim *s, int32_t a, double T, double *out6) {
  out6[0] = cp_R(s->nasa7[a], T);
  out6[1] = h_RT(s->nasa7[a], T);
  out6[2] = s_R(s->nasa7[a], T);
  out6[3] = spec_U(s, a, T);
  out6[4] = spec_H(s, a, T);
  out6[5] = spec_Cv(s, a, T);
}

int32_t orc_temperature(const orc_sim *s, const double *Y, double e_target, double T_start,
                        double *T_out) {
  return temperature(s, Y, e_target, T_start, T_out);
}

void orc_rates(const orc_sim *s, const double *rho_a, double T, double *rdot) {
  production_rates(s, rho_a, T, rdot);
}

void orc_diffusion(const orc_sim *s, const double *Y, double T, const double *rhs, double *du,
                   double *beta) {
  const int M = s->p.M;
  double zeta_a[MAXM] = {0}, K[MAXM][MAXM], inv_tau[MAXM], r[MAXM][3], d[MAXM][3];
  double inv_m = 0.0;
  for (int a = 0; a < M; ++a) {
    zeta_a[a] = gas_const(s, a) * T;
    inv_m += Y[a] / s->molar_mass[a];
  }
  const double zeta = s->p.kappa * R_UNIV * T * inv_m / 1e-3;
  relaxation(s, Y, zeta_a, zeta, T, K, inv_tau, beta);
  for (int a = 0; a < M; ++a)
    for (int c = 0; c < 3; ++c) r[a][c] = rhs[a * 3 + c];
  diffusion_velocities(M, K, inv_tau, Y, r, d);
  for (int a = 0; a < M; ++a)
    for (int c = 0; c < 3; ++c) du[a * 3 + c] = d[a][c];
}

void orc_iso_grad(const orc_sim *s, const double *field, double *grad3) {
  for (int64_t n = 0; n < s->N; ++n)
    for (int a = 0; a < 3; ++a) grad3[a * s->N + n] = iso_grad(s, field, n, a);
}
#endif /* ORC_REAL */
