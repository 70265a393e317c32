// Internal layout shared by the kernels and the host side of the C ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "lbm.h"

namespace lbm {

constexpr int Q = 27;
constexpr int MAXM = LBM_MAX_SPECIES;
constexpr int MAXR = LBM_MAX_REACTIONS;
constexpr int MAXORD = LBM_MAX_ORDER;

// Read-only constant tables, uploaded into the workspace at create time and read
// with uniform loads by every kernel.
struct Tables {
  int32_t M, R, S, open_any;
  double Ra[MAXM];            // lattice gas constant kappa R_U / m_a  (per K)
  double nasa[MAXM][7];       // NASA-7 rows
  double ucoef[MAXM][6];      // U_a(T) = sum_k ucoef[k] T^k (k=0: Ra a6; 1: Ra (a1-1); k>=2: Ra a_k/k)
  double cvcoef[MAXM][5];     // C_v,a(T) = sum_k cvcoef[k] T^k
  double invD[MAXM][MAXM];    // 1 / D_ab, zero on the diagonal
  float invDf[MAXM][MAXM];
  double invDp[MAXM * (MAXM - 1) / 2];   // 1 / D_ab for a < b, row-major pairs
  float invDpf[MAXM * (MAXM - 1) / 2];
  double conc_scale[MAXM];    // rho_ref / m_a: lattice density -> mol/cm^3
  double rdot_scale[MAXM];    // m_a dt_phys / rho_ref: mol/(cm^3 s) -> lattice density/step
  double lnA[MAXR], bexp[MAXR], Ta[MAXR], dnu[MAXR];
  int32_t rev[MAXR];
  int32_t nu_r[MAXR][MAXM];
  int32_t nu_p[MAXR][MAXM];
  double dnu_a[MAXR][MAXM];             // nu'' - nu' per species
  int32_t nreac[MAXR], nprod[MAXR];     // molecules on each side
  int32_t reac_idx[MAXR][MAXORD];       // their species, repeated by coefficient
  int32_t prod_idx[MAXR][MAXORD];
  double ln_c0_const;         // ln(p0 * 1e-6 / R_U): ln c0(T) = ln_c0_const - ln T (mol/cm^3)
  double omega, omega1;
  double dexp, ln_dTref;      // D_ab(T) = D_ab exp(dexp (ln T - ln_dTref)); dexp = 0: constant
  double vexp, ln_vTref;      // 1/omega(T) - 1/2 = c_om exp(vexp (ln T - ln_vTref)); vexp = 0: constant
  double c_om, c_om1;         // 1/omega - 1/2 and 1/omega1 - 1/2 at the reference temperature
};

// Constants of the collision.  The init, ghost and output kernels take them as a kernel
// argument; the step kernel reads a copy in the workspace through a constant-address
// pointer.  Both are read with scalar loads, which stay valid after a kernel's first
// store to global memory.
struct CollideConsts {
  double omega;
  double Ra[MAXM];                       // lattice gas constants kappa R_U / m_a
  float Raf[MAXM];
  double invDp[MAXM * (MAXM - 1) / 2];   // 1 / D_ab for a < b, row-major pairs
  float invDpf[MAXM * (MAXM - 1) / 2];
  // deviation formats: stored value = (f - ref[s][i]) * isc[s], f = ref[s][i] + sc[s] * stored
  float ref[MAXM + 1][Q];
  float sc[MAXM + 1], isc[MAXM + 1];
  double vexp, ln_vTref, c_om;           // temperature law of omega (as in Tables)
};

// A plane of one (set, direction) holds the rows (z, y) of the lattice padded with a
// ghost layer on open y and z axes, x fastest (NX = nx), and after them, on an open x
// axis, the x ghost cells.  Row r = (z + pz) NY + (y + py); cell x of row r at r NX + x.
// The x axis may be split into nseg independent segments (a batch of lattices of the
// same cross-section side by side, each with the x faces' boundary conditions at both
// of its ends); segment s has the x ghost cells XG + 2 s NY NZ + r before its first x
// and XG + (2 s + 1) NY NZ + r after its last.  One segment: XG + r and XG + NY NZ + r.
struct Geom {
  int32_t M;                  // species
  int32_t nx, ny, nz;
  int32_t px, py, pz;         // ghost padding inside the rows (px = 0; 1 on open y, z)
  int32_t NX, NY, NZ;         // row length nx and padded row counts
  int32_t per[3];             // periodic axis flags
  int32_t bc[6];
  int32_t xg;                 // 1 when the x axis is open: x ghost cells after the rows
  int32_t nseg;               // independent segments along x (1: one lattice)
  int64_t N, NPAD;            // interior nodes, cells of one plane
  int64_t XG;                 // first x ghost cell, NX NY NZ
  const int32_t *x_seg;       // [nx] segment of each x (nseg > 1)
  const int32_t *seg_off;     // [nseg + 1] first x of each segment, then nx (nseg > 1)
  int32_t vt;                 // 1: relaxation rates from the temperature law (visc_T_exp != 0)
  int32_t corr_tile;          // tile shape of the correction stencil (chosen at create time)
};

// Device pointers into the workspace.
struct Buffers {
  uint32_t *status;           // anomaly word
  const Tables *tab;
  void *pop[2];               // [S][27][NPAD] storage type
  double *T;                  // [N] stored temperature
  void *side_Y;               // [M][N] storage type: mass fractions
  void *side_w;               // [M][N]: (2 - omega1)/2 * P * H_a
  void *side_phi;             // [3][N]: argument of the isotropy correction
  void *side_rho;             // [N]   density (ghost equilibria)
  void *side_u;               // [3][N] velocity (ghost equilibria)
  void *psi;                  // [3][N]
  void *corr;                 // [6][NPAD]: X (3), then the energy-flux correction (3); zero in ghost cells
  const CollideConsts *kc;    // device copy of the collision constants
  double *diag;               // [8][ceil(N / 128)] partial sums of the diagnostics
};

// Work buffers of the discrete adjoint (in the workspace when lbm_desc.adjoint != 0).
struct AdjBufHost {
  double *P;            // [S][27][N] pulled populations of the forward state being reversed
  double *Ln;           // [S][27][N] copy of the incoming adjoint
  const double *T0;     // [N] stored temperature of that state (Newton start)
  double *fY, *fw;      // [M][N] mass fractions and Cg weights of the forward state
  double *lX, *lgY;     // [3][N] adjoint of X; [M][3][N] adjoint of grad Y_a
  double *lpsi, *lphi;  // [3][N]
  double *lYs;          // [M][N] adjoint of Y_a from the gradient stencil
  double *part;         // [3R][ceil(N / 8)] Arrhenius gradient partials
};

// launchers (lbm_device.hip)
hipError_t launch_init(const Geom &g, const Buffers &b, const CollideConsts &kc, int store, const double *rho,
                       const double *u, const double *T, const double *Y, int cur, hipStream_t st);
hipError_t launch_step(const Geom &g, const Buffers &b, const CollideConsts &kc, int store, int cur,
                       hipStream_t st);
hipError_t launch_psi(const Geom &g, const Buffers &b, int store, hipStream_t st);
hipError_t launch_corr(const Geom &g, const Buffers &b, int store, hipStream_t st);
// the correction-stencil tile shapes valid for the lattice (their count, at most
// LBM_CORR_TILES_MAX), whether a shape forms psi itself (then k_psi is not launched
// before it), and one launch of the stencil alone with g.corr_tile (for timing them)
constexpr int LBM_CORR_TILES_MAX = 8;
int corr_tile_candidates(const Geom &g, int *out);
bool corr_forms_psi(int tile);
hipError_t launch_corr_only(const Geom &g, const Buffers &b, int store, hipStream_t st);
hipError_t launch_ghost(const Geom &g, const Buffers &b, const CollideConsts &kc, int store, int cur,
                        hipStream_t st);
hipError_t launch_macros(const Geom &g, const Buffers &b, const CollideConsts &kc, int store, int cur,
                         double *rho, double *u, double *T, double *P, double *Y, hipStream_t st);
hipError_t launch_export(const Geom &g, const Buffers &b, const CollideConsts &kc, int store, int cur,
                         const int64_t *nodes, int64_t n_nodes, double *out, double *T_out, hipStream_t st);
hipError_t launch_diag(const Geom &g, const Buffers &b, const CollideConsts &kc, int store, int cur, double T_iso,
                       double *hrr, double *totals, hipStream_t st);
hipError_t launch_flame(const Geom &g, const Buffers &b, const CollideConsts &kc, int store, int cur, double T_iso,
                        const double *centre, double *work, double *out, double *totals, hipStream_t st);
hipError_t launch_zero(void *p, int64_t n_words32, hipStream_t st);
hipError_t launch_stream_copy(const void *src, void *dst, int64_t bytes, hipStream_t st);
// the scratch array of lbm_flame_speeds_static: its address on `device` (the current
// device) is resolved once per device; then the flame speeds with their work fields and
// partial sums in it (g.N <= LBM_FLAME_STATIC_MAX_NODES)
hipError_t flame_scratch_resolve(int device);
// launchers of the discrete adjoint (lbm_adjoint.hip); tb is the device copy of the tables
hipError_t launch_adjoint_step(const Geom &g, const Tables *tb, const AdjBufHost &h, double omega, double omega1,
                               int R, double *adj, double *grad, hipStream_t st);
hipError_t launch_adjoint_macros(const Geom &g, const Tables *tb, const double *P, const double *T0,
                                 const double *w_rho, const double *w_u, const double *w_T, const double *w_P,
                                 const double *w_Y, double *adj, hipStream_t st);
hipError_t launch_adjoint_init(const Geom &g, const Tables *tb, const double *rho, const double *u, const double *T,
                               const double *Y, const double *lam, double *g_rho, double *g_u, double *g_T,
                               double *g_Y, hipStream_t st);
hipError_t launch_flame_static(const Geom &g, const Buffers &b, const CollideConsts &kc, int store, int cur,
                               int device, double T_iso, const double *centre, double *out, double *totals,
                               hipStream_t st);

}  // namespace lbm
