/*
 * FP64 CPU oracle of the reactive-mixture lattice Boltzmann step
 * (Sawant, Dorschner & Karlin, "Reactive mixtures with the lattice Boltzmann
 * model").
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the correctness reference for the
 * HIP path.  Only the tests, the smoke check and the benchmark's CPU-baseline leg
 * may load it; the product path never calls it.  It shares no code with the HIP
 * library.
 *
 * Conventions
 *   - D3Q27, velocity index i = (cx+1) + 3 (cy+1) + 9 (cz+1), c in {-1,0,1}^3.
 *   - Node index n = x + nx (y + ny z).
 *   - Stored population sets S = M + 1: species 0..M-2 (the last species M-1 is
 *     slaved to the mixture, Sec. 3 "strong coupling"), then the mixture f, then
 *     the energy g.  Population arrays are [S][27][N].
 *   - The state held is the pre-collision population at the current time.
 */
#ifndef REACTLBM_ORACLE_H
#define REACTLBM_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ORC_Q 27
#define ORC_MAXM 16
#define ORC_MAXR 64

enum { ORC_BC_PERIODIC = 0, ORC_BC_OPEN = 1, ORC_BC_OPEN_U0 = 2, ORC_BC_SYMMETRY = 3 };
enum { ORC_ANOM_NONFINITE = 1u, ORC_ANOM_NEWTON = 2u, ORC_ANOM_NEG_DENSITY = 4u };

typedef struct {
  int32_t nx, ny, nz;
  int32_t bc[6];               /* -x,+x,-y,+y,-z,+z */
  int32_t M;                   /* species, 2..ORC_MAXM */
  int32_t R;                   /* reactions, 0..ORC_MAXR */
  const double *molar_mass;    /* [M] g/mol */
  const double *nasa7;         /* [M][7] */
  const double *diff;          /* [M][M] lattice units, symmetric */
  const int32_t *nu_reac;      /* [R][M] */
  const int32_t *nu_prod;      /* [R][M] */
  const double *arrhenius;     /* [R][3]: A (CGS), b, Ta (K) */
  const uint8_t *reversible;   /* [R] */
  double omega, omega1;
  double kappa;                /* s^2/m^2 */
  double dt_phys;              /* s per step */
  double rho_ref;              /* g/cm^3 per lattice density unit */
  double p0;                   /* Pa, standard pressure of the thermo data */
  double diff_T_ref;           /* K; with diff_T_exp != 0: D_ab(T) = D_ab (T / diff_T_ref)^diff_T_exp */
  double diff_T_exp;
  double visc_T_ref;           /* K; with visc_T_exp != 0: 1/omega - 1/2 and 1/omega1 - 1/2 */
  double visc_T_exp;           /* scale with (T / visc_T_ref)^visc_T_exp at each node */
} orc_problem;

typedef struct orc_sim orc_sim;

/* whole-lattice driver */
orc_sim *orc_create(const orc_problem *p);
void orc_destroy(orc_sim *s);
void orc_init(orc_sim *s, const double *rho, const double *u, const double *T, const double *Y);
uint32_t orc_step(orc_sim *s, int32_t nsteps, int32_t nthreads);
uint32_t orc_macros(orc_sim *s, double *rho, double *u, double *T, double *P, double *Y);
/* S_d, S_a (eq. sd) and isosurface weights of the current state; out[3][N], totals[5] */
uint32_t orc_flame_speeds(orc_sim *s, double T_iso, const double *centre, double *out, double *totals);
void orc_get_state(const orc_sim *s, double *pop, double *T);
void orc_set_state(orc_sim *s, const double *pop, const double *T);
void orc_get_post(const orc_sim *s, double *post);

/* per-node quantities of the last step (for the pins) */
enum {
  ORC_F_T = 0,      /* [N]      */
  ORC_F_RDOT = 1,   /* [M][N]   */
  ORC_F_DU = 2,     /* [M][3][N] */
  ORC_F_BETA = 3,   /* [M][N]   */
  ORC_F_X = 4,      /* [3][N]   */
  ORC_F_GRADY = 5,  /* [M][3][N] */
  ORC_F_PHI = 6,    /* [3][N]   */
  ORC_F_PSI = 7,    /* [3][N]   */
  ORC_F_NEWTON = 8  /* [N] iterations used */
};
void orc_get_field(const orc_sim *s, int32_t which, double *out);

/* pieces of the method, for unit pins */
void orc_product_form(double dens, const double *v, double zeta, double *out27);
void orc_grad_form(double rhoE, const double *q, const double *R9, double *out27);
void orc_thermo(const orc_sim *s, int32_t a, double T, double *out6);
int32_t orc_temperature(const orc_sim *s, const double *Y, double e_target, double T_start,
                        double *T_out);
void orc_rates(const orc_sim *s, const double *rho_a, double T, double *rdot);
void orc_diffusion(const orc_sim *s, const double *Y, double T, const double *rhs,
                   double *du, double *beta);
void orc_iso_grad(const orc_sim *s, const double *field, double *grad3);

#ifdef __cplusplus
}
#endif

#endif
