/*
 * C ABI of the reactive-mixture lattice Boltzmann step on one MI355X (gfx950).
 *
 * The model is the one of Sawant, Dorschner & Karlin, "Reactive mixtures with the
 * lattice Boltzmann model": M species populations (Sec. 2, eq. finalNumerical-
 * Equations) relaxing to a Stefan-Maxwell quasi-equilibrium with an Arrhenius
 * source, a mixture population f for mass and momentum (Sec. 3, eq. f) and an
 * energy population g for total energy with heat of formation (Sec. 3, eq. g),
 * temperature recovered from energy (eq. temperature), on the D3Q27 lattice.  The
 * last species is slaved to the mixture (eq. strongest), so M + 1 population sets
 * are stored.
 *
 * Conventions
 *   - Lattice units dx = dt = 1.  Node n = x + nx (y + ny z), x fastest.
 *   - Velocity index i = (cx+1) + 3 (cy+1) + 9 (cz+1), c in {-1,0,1}^3.
 *   - Population sets s = 0..M-2 species, s = M-1 mixture f, s = M energy g.
 *   - All device pointers are caller-owned; the library never allocates or frees
 *     device memory (lbm_step_graph creates a capture stream and graph objects of
 *     the HIP runtime, released by lbm_destroy).  Device work is enqueued on the
 *     given stream (a hipStream_t passed as void*, NULL = default stream) and is
 *     asynchronous; only lbm_create (table upload and tile timing),
 *     lbm_status_sync and lbm_step_timed wait for the device.
 *   - Every call returns an lbm_status; nothing aborts or throws across the ABI.
 *     On error, lbm_last_error(h) explains it (lbm_last_error(NULL) for errors of
 *     calls that have no handle).
 *   - A handle is not thread-safe; calls on one handle must not overlap.
 */
#ifndef REACTLBM_LBM_H
#define REACTLBM_LBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lbm_ctx *lbm_handle;

typedef enum {
  LBM_OK = 0,
  LBM_ERR_ARG = -1,            /* invalid argument or descriptor                 */
  LBM_ERR_UNSUPPORTED = -2,    /* valid but not provided by this library         */
  LBM_ERR_HIP = -3,            /* a HIP runtime call failed                      */
  LBM_ERR_WORKSPACE = -4,      /* workspace too small or misaligned              */
  LBM_ERR_DEVICE_ANOMALY = -5  /* lbm_status_sync found anomaly bits set         */
} lbm_status;

/* boundary types per face (Sec. 5.1: zero-gradient ends by equilibrium ghosts,
 * zero velocity imposed at the unburnt end) */
enum {
  LBM_BC_PERIODIC = 0, /* both faces of an axis must be periodic together        */
  LBM_BC_OPEN_EQ = 1,  /* ghost = equilibrium at the adjacent node's rho_a, u, T  */
  LBM_BC_OPEN_EQ_U0 = 2, /* same with ghost velocity 0                           */
  LBM_BC_SYMMETRY = 3   /* mirror plane half a cell beyond the boundary nodes (Sec. 5.2):
                           a ghost holds the mirrored population of the mirrored node, with
                           mirrored deferred corrections; beyond a symmetry and an open face,
                           the equilibrium of the mirrored direction                        */
};

/* population storage; the node-local work (temperature inversion, thermo,
 * production rates, Stefan-Maxwell solve) is double precision in all of them.
 * The deviation formats store (f_i - f_ref,i) / sc per population in 16 bits,
 * with f_ref the equilibrium of each set at the caller's quiescent reference state
 * (lbm_desc.ref_state) and sc the reference magnitude of the set; their side
 * fields and corrections are FP32. */
enum { LBM_STORE_F64 = 0, LBM_STORE_F32 = 1, LBM_STORE_F16_DEV = 2, LBM_STORE_BF16_DEV = 3 };

/* anomaly bits latched on the device, read by lbm_status_sync */
enum {
  LBM_ANOM_NONFINITE = 1u,    /* non-finite density, energy or temperature        */
  LBM_ANOM_NEWTON = 2u,       /* temperature inversion did not converge in 50 its */
  LBM_ANOM_NEG_DENSITY = 4u   /* rho <= 0 or slaved species density <= 0          */
};

#define LBM_MAX_SPECIES 10
#define LBM_MAX_REACTIONS 64
#define LBM_MAX_ORDER 8      /* molecules on one side of a reaction */

/*
 * Statement of the problem (Sec. 2-4).  Host arrays, copied by lbm_create.
 *   nx, ny, nz      lattice size, each >= 1
 *   bc[6]           faces -x,+x,-y,+y,-z,+z (LBM_BC_*)
 *   n_species       M, 2..LBM_MAX_SPECIES; species M-1 is slaved (eq. strongest)
 *   n_reactions     R, 0..LBM_MAX_REACTIONS
 *   molar_mass[M]   g/mol
 *   nasa7[M][7]     single-range NASA-7 coefficients (c_p/R polynomial a1..a5,
 *                   enthalpy constant a6 including the formation enthalpy,
 *                   entropy constant a7); eq. specHa
 *   diff_ab[M][M]   binary diffusivities D_ab in lattice units, symmetric, > 0
 *                   off the diagonal (eqs. stefanMaxwell, tauab)
 *   nu_reac[R][M], nu_prod[R][M]   stoichiometric coefficients, 0..3, at most
 *                   LBM_MAX_ORDER molecules on each side
 *   arrhenius[R][3] A (CGS mol, cm^3, s), temperature exponent b, activation
 *                   temperature Ta (K): k_f = A T^b exp(-Ta/T)
 *   reversible[R]   nonzero: reverse rate k_f / K_c, K_c from the NASA-7 Gibbs
 *                   function at p0
 *   omega, omega1   relaxation of f and of the energy flux (eqs. f, g), in (0,2)
 *   kappa           (dt/dx)^2 in s^2/m^2: lattice R_a T = kappa R_U T / m_a
 *   dt_phys         seconds per step (chemistry)
 *   rho_ref         g/cm^3 per lattice density unit (chemistry)
 *   p0              standard pressure of the thermo data, Pa (Sec. 4: 1 atm)
 *   storage         LBM_STORE_*
 *   ref_state       [2 + M] host array (rho in lattice units, T in K, Y[M] mass
 *                   fractions summing to 1) of the reference state at rest of the
 *                   deviation formats; may be NULL for LBM_STORE_F64 / _F32
 *   n_segments      0 or 1: one lattice.  >= 2: a batch of independent lattices of
 *                   the same ny x nz cross-section and transport, mechanism and
 *                   units, side by side along x (e.g. quasi-1D flames of different
 *                   lengths, Sec. 5.1).  Segment s takes segment_lengths[s] >= 1
 *                   consecutive x; the lengths sum to nx, the x faces must not be
 *                   periodic, and every segment has bc[0] at its first x and bc[1]
 *                   after its last.  Nodes of different segments never exchange
 *                   populations or stencil values.  Node indices, fields and
 *                   populations keep the one-lattice layout of nx x ny x nz.
 *   segment_lengths [n_segments] host array, read when n_segments >= 2
 *   diff_T_ref, diff_T_exp   temperature dependence of the diffusivities: with
 *                   diff_T_exp != 0 (|exp| <= 4, diff_T_ref > 0 in K) every binary
 *                   diffusivity is D_ab (T / diff_T_ref)^diff_T_exp at the node's
 *                   temperature (a power law standing in for the temperature-dependent
 *                   transport data of Sec. 3); 0: the constants diff_ab
 *   visc_T_ref, visc_T_exp   temperature dependence of the viscosity and the
 *                   conductivity: with visc_T_exp != 0 (|exp| <= 4, visc_T_ref > 0
 *                   in K) the factors 1/omega - 1/2 and 1/omega1 - 1/2 of eqs. mu and
 *                   lambda scale with (T / visc_T_ref)^visc_T_exp at each node, which
 *                   sets that node's relaxation rates (LBM_STORE_F64 and _F32 only);
 *                   0: the constants omega, omega1
 *   adjoint         nonzero: the workspace also holds the work buffers of the discrete
 *                   adjoint (lbm_adjoint_*), about 0.48 (M + 1) kB more per node.  The
 *                   adjoint covers LBM_STORE_F64 and _F32, constant transport
 *                   (diff_T_exp = visc_T_exp = 0) and periodic, open and zero-velocity
 *                   faces of one lattice (n_segments <= 1); other descriptors with
 *                   adjoint != 0 get LBM_ERR_UNSUPPORTED
 */
typedef struct {
  int32_t nx, ny, nz;
  int32_t bc[6];
  int32_t n_species;
  int32_t n_reactions;
  const double *molar_mass;
  const double *nasa7;
  const double *diff_ab;
  const int32_t *nu_reac;
  const int32_t *nu_prod;
  const double *arrhenius;
  const uint8_t *reversible;
  double omega, omega1;
  double kappa, dt_phys, rho_ref, p0;
  int32_t storage;
  int32_t adjoint;
  const double *ref_state;
  int32_t n_segments;
  int32_t reserved2;
  const int32_t *segment_lengths;
  double diff_T_ref, diff_T_exp;
  double visc_T_ref, visc_T_exp;
} lbm_desc;

/* Bytes of device workspace the descriptor needs: populations x2 with a ghost
 * layer on open axes, temperature (FP64), a side channel of node fields for the
 * gradient stencils and the ghosts (2M + 7 words) and psi (3 words), the deferred
 * corrections (6 words per node of the padded lattice), all in the storage
 * precision, the constant tables, a copy of the collision constants and a status
 * word (and, for a batch of segments, the segment table, 4 (nx + n_segments + 1)
 * bytes; the x ghost layer is then two cells per segment and row).  Fails with
 * LBM_ERR_ARG when one padded plane of the lattice (its node count with the ghost layers) times 8 bytes for LBM_STORE_F64, 4 otherwise, reaches
 * 2 GiB: the step kernel addresses a plane with 32-bit byte offsets. */
lbm_status lbm_workspace_size(const lbm_desc *desc, size_t *bytes);

/* Validate the descriptor, copy it, and upload its tables into the caller's
 * device workspace (256-byte aligned, >= lbm_workspace_size bytes, must outlive
 * the handle).  The current HIP device must be the workspace's device.  The
 * upload is synchronous.  It then times the shapes of the correction stencil (psi
 * and the deferred corrections of eqs. Xalpha and corrFourier) that suit the lattice
 * (four launches each, on a non-blocking stream that the call creates, waits for and
 * destroys: lbm_create has no stream argument because it returns only when the handle
 * is ready, and the private stream keeps the timing apart from the caller's streams)
 * and keeps the fastest; LBM_CORR_TILE=k in the environment picks shape k instead:
 * 0-2 (psi, then the corrections on tiles of 32x4x4, 64x2x2, 16x4x8 nodes) and 6
 * (both in one pass along z, in chunks of 32 planes) for lattices with a
 * cross-section, with 9 (a tile of 32x8x1) when they are one node thick in z, and 3-5
 * for lattices one node thick in y and z.
 * Every shape gives the same bits.  The timing overwrites the temperature, the side
 * channel and the deferred corrections in the workspace, so a state left there by
 * another handle is not kept: start from lbm_init_fields. */
lbm_status lbm_create(const lbm_desc *desc, void *d_workspace, size_t bytes, lbm_handle *out);

/* Release the host handle (the workspace is untouched). */
lbm_status lbm_destroy(lbm_handle h);

/* Equilibrium initial state (no non-equilibrium part) from device FP64 fields:
 * rho[N], u[3][N], T[N] (K), Y[M][N] mass fractions.  Also sets the stored
 * temperature (Newton start) and clears the anomaly word. */
lbm_status lbm_init_fields(lbm_handle h, const double *d_rho, const double *d_u,
                           const double *d_T, const double *d_Y, void *stream);

/* Advance n_steps >= 0 time steps (one step: moments, temperature, chemistry,
 * Stefan-Maxwell solve, collision of all sets, ghosts, streaming). */
lbm_status lbm_step(lbm_handle h, int32_t n_steps, void *stream);

/* Same as lbm_step, then waits and returns the summed device time of each kernel
 * kind in ms_out[LBM_NUM_KERNELS] (HIP events around every launch). */
#define LBM_NUM_KERNELS 4 /* 0 stream and collide (moments, temperature, chemistry, Stefan-Maxwell,
                             collision of all sets), 1 psi stencil, 2 correction stencil, 3 ghosts */
lbm_status lbm_step_timed(lbm_handle h, int32_t n_steps, void *stream, float *ms_out);

/* Same result as lbm_step, bit for bit.  The launches of n_steps steps are recorded
 * once into a HIP graph (per handle, per n_steps and per parity of the number of steps
 * taken so far; the 8 most recent recordings are kept) and replayed by one graph launch
 * on the stream.  This removes the per-kernel launch cost of small lattices and batches
 * of short ones.  A recording holds kernel launches only (no allocation, no memset);
 * it is captured on a stream of the handle, created at the first call, and released
 * by lbm_destroy. */
lbm_status lbm_step_graph(lbm_handle h, int32_t n_steps, void *stream);

/* Macroscopic fields of the current (pre-collision) state into device FP64
 * arrays, any of which may be NULL: rho[N], u[3][N], T[N], P[N] (lattice
 * pressure rho R T), Y[M][N].  Does not modify the state. */
lbm_status lbm_macros(lbm_handle h, double *d_rho, double *d_u, double *d_T, double *d_P,
                      double *d_Y, void *stream);

/* Pre-collision populations of the current state at the listed nodes (device
 * int64 node ids in [0, N)) as FP64 out[(s*27 + i)*n_nodes + k], and the stored
 * temperature at those nodes in T_out[k] (T_out may be NULL). */
lbm_status lbm_populations(lbm_handle h, const int64_t *d_nodes, int64_t n_nodes, double *d_out,
                           double *d_T_out, void *stream);

/* Diagnostics of the current state (Sec. 5.2), as lbm_macros reports it:
 *   d_hrr[N]     heat release rate -sum_a H_a rho_dot_a at every node, in lattice
 *                units (H_a the species enthalpy R_a T h_a(T), rho_dot_a the production
 *                rate by mass action per step, the same as the collision's source);
 *   d_totals[LBM_DIAG_TOTALS]  sums over the lattice: [0] heat release rate, [1] the
 *                number of nodes with T >= T_iso (the burnt volume), [2] mass sum rho,
 *                [3] total energy sum rho E.
 * Either output may be NULL.  Device FP64 buffers owned by the caller; the sums are
 * formed in a fixed order (the same value on every call for the same state).  Uses
 * the diagnostics section of the workspace: concurrent calls on one handle race. */
#define LBM_DIAG_TOTALS 4
lbm_status lbm_diagnostics(lbm_handle h, double T_iso, double *d_hrr, double *d_totals, void *stream);

/* Flame-front speeds of the current state (Sec. 5.2, eq. sd), all in FP64:
 *   S_d = [ -sum_a H_a rho_dot_a + div(lambda grad T) - rho (sum_a C_p,a Y_a du_a) . grad T ]
 *         / (rho C_p |grad T|)
 * with lambda = (1/omega1 - 1/2) P C_p (eq. lambda, dt = 1), C_p = sum_a Y_a C_p,a, the
 * diffusion velocities du_a of the Stefan-Maxwell system (eq. transform1) and the
 * isotropic lattice gradient for grad and for each term of div; the absolute speed
 * S_a = S_d + u . n with n = -grad T / |grad T| (both 0 where grad T = 0); and the
 * weight w = max(0, 1 - |T - T_iso| / |grad T|) of each node in a mean over the surface
 * T = T_iso (a hat one cell wide across the surface, so that sums over nodes stand for
 * surface integrals as in eq. rmean).  The density-weighted speed of the paper is
 * rho S_d / rho_u.
 *   d_work    device scratch of LBM_FLAME_WORK x N doubles (overwritten)
 *   d_out     [3][N] device: S_d, S_a, w (may be NULL)
 *   d_totals  [LBM_FLAME_TOTALS] device: sum w (isosurface area), sum w S_d, sum w S_a,
 *             sum w rho S_d, sum w |x - centre| (over sum w: the mean radius of eq.
 *             rmean), in a fixed order (may be NULL)
 *   centre    host [3] lattice coordinates (may be NULL: the origin)
 * Uses the workspace's partial-sum area: calls that overlap on one handle race. */
#define LBM_FLAME_WORK 17
#define LBM_FLAME_TOTALS 5
lbm_status lbm_flame_speeds(lbm_handle h, double T_iso, const double *centre, double *d_work,
                            double *d_out, double *d_totals, void *stream);

/* lbm_flame_speeds without the caller's work buffer, for callers that cannot allocate
 * device memory (code under graph capture, serving loops that forbid allocation).  Same
 * kernels and results as lbm_flame_speeds; the work fields and partial sums live in a
 * scratch array of the library in device memory, one per GPU, held until the process
 * ends (LBM_FLAME_STATIC_MAX_NODES x LBM_FLAME_WORK doubles plus the partial sums,
 * about 9 MB).  Allocates nothing.  Lattices of more than LBM_FLAME_STATIC_MAX_NODES
 * nodes are rejected with LBM_ERR_ARG.  Every call on one GPU, from any handle, uses
 * the same scratch array: calls that overlap on one GPU (other streams, other threads)
 * race and must be ordered by the caller.  d_out and d_totals as in lbm_flame_speeds
 * (either may be NULL). */
#define LBM_FLAME_STATIC_MAX_NODES 65536
lbm_status lbm_flame_speeds_static(lbm_handle h, double T_iso, const double *centre, double *d_out,
                                   double *d_totals, void *stream);

/* State snapshots, for checkpoints and for the adjoint's recomputation.  A snapshot is
 * the current pre-collision state as the next step reads it: the populations of the
 * current buffer (with their ghost cells), the deferred corrections and the stored
 * temperature, in lbm_state_size bytes of caller-owned device memory (256-byte aligned).
 * Saving and loading are stream-ordered device copies; loading replaces the handle's
 * current state (the side fields are recomputed by the next step). */
lbm_status lbm_state_size(lbm_handle h, size_t *bytes);
lbm_status lbm_state_save(lbm_handle h, void *d_state, void *stream);
lbm_status lbm_state_load(lbm_handle h, const void *d_state, void *stream);

/* Replace the Arrhenius parameters (host [R][3]: A >= 0 CGS, b, Ta in K; Sec. 4) of the
 * handle's reactions, for sensitivity studies.  Waits for the stream, then copies the
 * rebuilt tables on it and waits again. */
lbm_status lbm_set_arrhenius(lbm_handle h, const double *arrhenius, void *stream);

/*
 * Discrete adjoint (handles created with lbm_desc.adjoint != 0).  Adjoint populations are
 * device FP64 arrays [S][27][N] in node order: the adjoint of the pulled pre-collision
 * populations of a state.  d_state is a snapshot of lbm_state_save, or NULL for the
 * handle's current state.  All arithmetic is FP64 (on an FP32-stored state, the adjoint
 * of the FP32-stored trajectory).  Calls on one handle share the adjoint work buffers of
 * the workspace: they must not overlap.
 *
 * lbm_adjoint_step: one step of the method, F_{n+1} = step(F_n) (Sec. 2-4: moments,
 *   temperature by Newton on the energy (eq. temperature), mass-action rates,
 *   Stefan-Maxwell relaxation (eqs. tauab, transform1, fStar), the stencils of X and
 *   grad Y (eqs. Xalpha, corrFourier), the collisions of eqs. finalNumericalEquations, f
 *   and g, equilibrium ghosts at open faces (Sec. 5.1) and streaming), reversed at the
 *   state F_n held in d_state: d_adj holds lambda_{n+1} on entry and lambda_n =
 *   (dF_{n+1}/dF_n)^T lambda_{n+1} on return, and d_grad_params[R][3] (device, may be
 *   NULL) is incremented by (dF_{n+1}/d(ln A_k, b_k, Ta_k))^T lambda_{n+1}.
 */
lbm_status lbm_adjoint_step(lbm_handle h, const void *d_state, void *d_adj, double *d_grad_params,
                            void *stream);

/* Adjoint of lbm_macros at the state d_state: d_adj[S][27][N] = the gradient with respect
 * to the populations of sum over nodes of w_rho rho + w_u . u + w_T T + w_P P + w_Y . Y
 * (device FP64 weights [N], [3][N], [N], [N], [M][N]; any may be NULL: zero).  T enters
 * through the implicit function of eq. temperature. */
lbm_status lbm_adjoint_macros(lbm_handle h, const void *d_state, const double *d_w_rho, const double *d_w_u,
                              const double *d_w_T, const double *d_w_P, const double *d_w_Y, double *d_adj,
                              void *stream);

/* Adjoint of lbm_init_fields at the fields d_rho[N], d_u[3][N], d_T[N], d_Y[M][N]: from the
 * adjoint d_adj[S][27][N] of the initial populations, the gradients g_rho[N], g_u[3][N],
 * g_T[N], g_Y[M][N] (device FP64, any may be NULL) of the equilibrium initial state
 * (eqs. feq, gieq; each field varied with the others held). */
lbm_status lbm_adjoint_init(lbm_handle h, const double *d_rho, const double *d_u, const double *d_T,
                            const double *d_Y, const double *d_adj, double *d_g_rho, double *d_g_u, double *d_g_T,
                            double *d_g_Y, void *stream);

/* Wait for the stream, return the latched anomaly bits and clear them.  Returns
 * LBM_ERR_DEVICE_ANOMALY when any bit was set. */
lbm_status lbm_status_sync(lbm_handle h, void *stream, uint32_t *anomaly_bits);

/* Growth law of the expanding flame (Sec. 5.2): the least-squares line through
 * (ln t_k, ln R_k), k < n, of mean radii R_k (from lbm_flame_speeds' isosurface sums)
 * sampled at times t_k, as R = a t^alpha.  Host arrays; host arithmetic only (no device
 * work).  LBM_ERR_ARG for n < 2, a null pointer, a t_k or R_k that is not positive and
 * finite, or all t_k equal. */
lbm_status lbm_growth_fit(const double *t, const double *R, int64_t n, double *a, double *alpha);

/* Measurement aid: copy `bytes` (a multiple of 16, 16-byte aligned buffers) with a plain
 * streaming kernel of 16-byte loads and stores, the read + write bandwidth ceiling of a
 * streaming kernel on the device the stream belongs to. */
lbm_status lbm_stream_copy(const void *d_src, void *d_dst, size_t bytes, void *stream);

/* Message of the last failed call on h (or of a handle-less call for NULL);
 * valid until the next call on the same handle. */
const char *lbm_last_error(lbm_handle h);

#ifdef __cplusplus
}
#endif

#endif
