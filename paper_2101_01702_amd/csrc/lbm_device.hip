// HIP kernels (gfx950) of the reactive-mixture lattice Boltzmann step.
//
// Model: Sawant, Dorschner & Karlin, "Reactive mixtures with the lattice Boltzmann
// model" -- species LBE (Sec. 2, eqs. finalNumericalEquations, fStar, tauab,
// transform1, feq, fstar, fsource), mixture f and energy g (Sec. 3, eqs. f, g, Xalpha,
// Ai, gieq, giqeq, geq1mom, geq2mom, gstareq1mom, qdiff, corrFourier, temperature,
// strongest), coupling loop (Sec. 4), equilibrium ghosts at open ends (Sec. 5.1).
//
// Data layout: populations SoA [set][i][z][y][x] with a one-cell ghost layer on open
// axes, two ping-pong buffers, pull streaming.  One thread per node.
//
// The non-local terms of the collision (isotropy correction A_i.X of eq. f and the
// Fourier correction flux q^corr of eq. corrFourier) depend on neighbour macros of
// the same time level.  They enter the post-collision populations additively, so the
// main kernel stores the post-collision populations without them, the stencil
// kernels compute them from a small side channel, and the next pull adds them back
// to each population as it is read (deferred correction).  One step therefore moves
// each population through HBM once in and once out.
#include <type_traits>
#include <utility>

#include "lbm_internal.h"

namespace lbm {

namespace {

__host__ __device__ constexpr int cx_of(int i) { return i % 3 - 1; }
__host__ __device__ constexpr int cy_of(int i) { return (i / 3) % 3 - 1; }
__host__ __device__ constexpr int cz_of(int i) { return i / 9 - 1; }
__host__ __device__ constexpr double w1(int c) { return c == 0 ? 2.0 / 3.0 : 1.0 / 6.0; }
__host__ __device__ constexpr double wgt(int i) { return w1(cx_of(i)) * w1(cy_of(i)) * w1(cz_of(i)); }
__host__ __device__ constexpr int c2_of(int i) {
  return cx_of(i) * cx_of(i) + cy_of(i) * cy_of(i) + cz_of(i) * cz_of(i);
}

// product-form factor Psi_c(xi, zeta) (eq. phis), with s = xi^2 + zeta precomputed
template <typename R>
__device__ __forceinline__ R psi_c(int c, R xi, R s) {
  return c == 0 ? R(1) - s : (c > 0 ? R(0.5) * (xi + s) : R(0.5) * (s - xi));
}

// Psi_c(xi, zeta) - Psi_c(xi + d, zeta) in closed form (eq. phis): for c = 0 it is
// d (2 xi + d), for c = +-1 it is -d (c + 2 xi + d) / 2
template <typename R>
__device__ __forceinline__ R psi_diff(int c, R xi, R d) {
  return c == 0 ? d * (R(2) * xi + d) : R(-0.5) * d * (R(c) + R(2) * xi + d);
}

// Source of the pull along c: byte offset of the source in one (set, direction)
// plane of the padded lattice, and its interior node index (-1 for a ghost cell).
// Plane bases are wave-uniform, so loads use a scalar base and a 32-bit offset (a
// plane of the largest lattice is far below 4 GiB).
struct Src {
  uint32_t ps;  // padded node index of the source
  int32_t ns;   // interior node index of the source, -1 when it is a ghost cell
};

struct AxisSrc {
  int s[3];     // source coordinate for c = -1, 0, +1 (x - c)
  bool out[3];
};

__device__ __forceinline__ AxisSrc axis_src(int x, int n, bool periodic) {
  AxisSrc a;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const int c = k - 1;
    int s = x - c;
    if (periodic) s = s < 0 ? s + n : (s >= n ? s - n : s);
    a.s[k] = s;
    a.out[k] = (s < 0) || (s >= n);
  }
  return a;
}

__device__ __forceinline__ Src make_src(const Geom &g, const AxisSrc &ax, const AxisSrc &ay,
                                        const AxisSrc &az, int kx, int ky, int kz) {
  Src r;
  const uint32_t sx = (uint32_t)(ax.s[kx] + g.px), sy = (uint32_t)(ay.s[ky] + g.py),
                 sz = (uint32_t)(az.s[kz] + g.pz);
  r.ps = (sz * (uint32_t)g.NY + sy) * (uint32_t)g.NX + sx;
  const bool out = ax.out[kx] || ay.out[ky] || az.out[kz];
  r.ns = out ? -1 : (az.s[kz] * g.ny + ay.s[ky]) * g.nx + ax.s[kx];
  return r;
}

// source of the pull for a uniform (cy, cz) and a compile-time x index: the y and z
// coordinates are wrapped or left in the ghost layer without table lookups
struct RowSrc {
  uint32_t prow;   // padded row index (z, y) times NX
  int32_t nrow;    // interior row index times nx, or -1 when (y, z) is in the ghost layer
};

__device__ __forceinline__ RowSrc row_src(const Geom &g, int y, int z, int cy, int cz) {
  int sy = y - cy, sz = z - cz;
  if (g.per[1]) sy = sy < 0 ? sy + g.ny : (sy >= g.ny ? sy - g.ny : sy);
  if (g.per[2]) sz = sz < 0 ? sz + g.nz : (sz >= g.nz ? sz - g.nz : sz);
  const bool out = sy < 0 || sy >= g.ny || sz < 0 || sz >= g.nz;
  RowSrc r;
  r.prow = ((uint32_t)(sz + g.pz) * (uint32_t)g.NY + (uint32_t)(sy + g.py)) * (uint32_t)g.NX;
  r.nrow = out ? -1 : (sz * g.ny + sy) * g.nx;
  return r;
}

__device__ __forceinline__ Src src_from_row(const Geom &g, const RowSrc &row, const AxisSrc &ax, int kx) {
  Src r;
  r.ps = row.prow + (uint32_t)(ax.s[kx] + g.px);
  r.ns = (row.nrow < 0 || ax.out[kx]) ? -1 : row.nrow + ax.s[kx];
  return r;
}

// element `idx` of a plane with a uniform base, addressed by a 32-bit byte offset
template <typename T>
__device__ __forceinline__ T ld(const T *__restrict__ base, uint32_t idx) {
  return *reinterpret_cast<const T *>(reinterpret_cast<const char *>(base) + idx * (uint32_t)sizeof(T));
}
template <typename T>
__device__ __forceinline__ void st(T *__restrict__ base, uint32_t idx, T v) {
  *reinterpret_cast<T *>(reinterpret_cast<char *>(base) + idx * (uint32_t)sizeof(T)) = v;
}

// An empty asm statement that claims to modify v.  Values derived from v inside a loop
// are then recomputed in every iteration instead of being hoisted and kept live, and
// loads through a pointer passed through it stay after it.
template <typename T>
__device__ __forceinline__ void opaque(T &v) {
  asm volatile("" : "+v"(v));
}
template <typename T>
__device__ __forceinline__ void opaque_uniform(T *&p) {
  asm volatile("" : "+s"(p));
}

// ---- storage formats -------------------------------------------------------------
// Populations are stored as ST; side fields, psi and corrections as Side; the
// inter-species term is evaluated in F.  The 16-bit formats store deviations from the
// reference populations: stored = (f - ref[s][i]) / sc[s].
#ifndef LBM_SIDE_F64_FOR_F32
#define LBM_SIDE_F64_FOR_F32 0
#endif
#ifndef LBM_FTERM_F64
#define LBM_FTERM_F64 0
#endif
template <typename ST>
struct Fmt {
  using Side = std::conditional_t<LBM_SIDE_F64_FOR_F32 && sizeof(ST) == 4, double, ST>;
  using F = std::conditional_t<LBM_FTERM_F64 != 0, double, ST>;
  static constexpr bool dev = false;
};
template <>
struct Fmt<_Float16> {
  using Side = float;
  using F = float;
  static constexpr bool dev = true;
};
template <>
struct Fmt<__bf16> {
  using Side = float;
  using F = float;
  static constexpr bool dev = true;
};

// value of a stored population of set s along direction i
template <typename ST>
__device__ __forceinline__ double pop_val(ST raw, int s, int i, const CollideConsts &kc) {
  if constexpr (Fmt<ST>::dev)
    return double(fmaf(kc.sc[s], float(raw), kc.ref[s][i]));
  else
    return double(raw);
}
// stored form of the population value v of set s along direction i
template <typename ST>
__device__ __forceinline__ ST pop_enc(double v, int s, int i, const CollideConsts &kc) {
  if constexpr (Fmt<ST>::dev)
    return ST(float((v - double(kc.ref[s][i])) * double(kc.isc[s])));
  else
    return ST(v);
}

// Workgroups are dispatched round-robin over the 8 XCDs of the chip, each with its own
// L2.  The lattice kernels read rows y-1, y, y+1 of the side fields and corrections,
// so the workgroup -> tile mapping gives each XCD a contiguous range of tiles: rows
// that neighbour each other then share an L2.  A bijection on [0, gridDim.x): the
// first 8 * floor(G / 8) workgroups are regrouped, the rest keep their index.
constexpr int NUM_XCD = 8;
__device__ __forceinline__ int64_t xcd_tile() {
  const int64_t G = gridDim.x, k = blockIdx.x;
  const int64_t q = G / NUM_XCD;
  if (k >= q * NUM_XCD) return k;
  return (k % NUM_XCD) * q + k / NUM_XCD;
}

// neighbour for the isotropic gradient: periodic wrap or clamp at open faces
__device__ __forceinline__ int nb_coord(int x, int c, int n, bool periodic) {
  int s = x + c;
  if (periodic) return s < 0 ? s + n : (s >= n ? s - n : s);
  return s < 0 ? 0 : (s >= n ? n - 1 : s);
}

template <typename CT>
struct Corr {
  const CT *X;    // [3][N]
  const CT *Cg;   // [3][N]
  int64_t N;
};

// pulled value of the mixture f along c = (CX, cy, cz) with the deferred A_i.X term;
// the corrections are held in the storage precision ST and added in FP64, the same
// way in every kernel that pulls
template <int CX, typename ST, typename CT>
__device__ __forceinline__ double pull_f(const ST *__restrict__ base, const Src &r, const Corr<CT> &cr, int cy,
                                         int cz, int s, int i, const CollideConsts &kc) {
  double v = pop_val(ld(base, r.ps), s, i, kc);
  if (r.ns >= 0) {
    const uint32_t ns = (uint32_t)r.ns;
    if constexpr (CX != 0) {
      if (cy == 0 && cz == 0) v += double(CT(0.5 * CX * double(ld(cr.X, ns))));
    } else {
      if (cy != 0 && cz == 0) v += double(CT(0.5 * cy * double(ld(cr.X + cr.N, ns))));
      if (cy == 0 && cz != 0) v += double(CT(0.5 * cz * double(ld(cr.X + 2 * cr.N, ns))));
    }
  }
  return v;
}

// pulled value of g with the deferred Fourier-correction flux 3 w_i c_i . Cg
template <int CX, typename ST, typename CT>
__device__ __forceinline__ double pull_g(const ST *__restrict__ base, const Src &r, const Corr<CT> &cr, int cy,
                                         int cz, int s, int i, const CollideConsts &kc) {
  const double w3 = 3.0 * (w1(CX) * w1(cy) * w1(cz));
  double v = pop_val(ld(base, r.ps), s, i, kc);
  if (r.ns >= 0) {
    const uint32_t ns = (uint32_t)r.ns;
    double d = 0.0;
    if constexpr (CX != 0) d += CX * double(ld(cr.Cg, ns));
    if (cy != 0) d += cy * double(ld(cr.Cg + cr.N, ns));
    if (cz != 0) d += cz * double(ld(cr.Cg + 2 * cr.N, ns));
    v += double(CT(w3 * d));
  }
  return v;
}

template <int... Is, typename F>
__device__ __forceinline__ void static_for_impl(std::integer_sequence<int, Is...>, F &&f) {
  (f(std::integral_constant<int, Is>{}), ...);
}
template <int N, typename F>
__device__ __forceinline__ void static_for(F &&f) {
  static_for_impl(std::make_integer_sequence<int, N>{}, f);
}

// ---- thermodynamics (eqs. specHa, Umix; NASA-7) -------------------------------------
__device__ __forceinline__ double h_RT(const double *a, double T, double invT) {
  return a[0] + T * (a[1] * 0.5 + T * (a[2] * (1.0 / 3.0) + T * (a[3] * 0.25 + T * (a[4] * 0.2)))) +
         a[5] * invT;
}
__device__ __forceinline__ double s_R(const double *a, double T, double lnT) {
  return a[0] * lnT + T * (a[1] + T * (a[2] * 0.5 + T * (a[3] * (1.0 / 3.0) + T * (a[4] * 0.25)))) +
         a[6];
}

// ---- moments of the pulled state (shared by step and macros) -----------------------
template <int M>
struct Macro {
  double rho, u[3], rhoE;
  double P6[6], q[3];            // pressure tensor (xx yy zz xy xz yz), energy flux
  double rs[M];                  // species densities, last one slaved (eq. strongest)
  double du0[M][3];              // u_a - u (right-hand side of eq. transform1)
};

template <int M, typename ST>
__device__ __forceinline__ void node_moments(const Geom &g, const ST *__restrict__ pop,
                                             const Corr<typename Fmt<ST>::Side> &cr, const CollideConsts &kc,
                                             int x, int y, int z, Macro<M> &m) {
  using Side = typename Fmt<ST>::Side;
  const AxisSrc ax = axis_src(x, g.nx, g.per[0]);
  const int64_t NPAD = g.NPAD;
  double rho = 0, jx = 0, jy = 0, jz = 0, pxx = 0, pyy = 0, pzz = 0, pxy = 0, pxz = 0, pyz = 0;
  double rE = 0, qx = 0, qy = 0, qz = 0;
  double ra[M - 1], jax[M - 1], jay[M - 1], jaz[M - 1];
#pragma unroll
  for (int a = 0; a < M - 1; ++a) ra[a] = jax[a] = jay[a] = jaz[a] = 0.0;
#pragma unroll 1
  for (int kyz = 0; kyz < 9; ++kyz) {
    const int ky = kyz % 3, kz = kyz / 3;
    const int cy = ky - 1, cz = kz - 1;
    const RowSrc row = row_src(g, y, z, cy, cz);
    static_for<3>([&](auto Kx) {
      constexpr int kx = decltype(Kx)::value;
      constexpr int cx = kx - 1;
      const int i = kx + 3 * kyz;
      const Src r = src_from_row(g, row, ax, kx);
      const double f = pull_f<cx, ST, Side>(pop + ((int64_t)(M - 1) * Q + i) * NPAD, r, cr, cy, cz, M - 1, i, kc);
      const double gg = pull_g<cx, ST, Side>(pop + ((int64_t)M * Q + i) * NPAD, r, cr, cy, cz, M, i, kc);
      rho += f;
      rE += gg;
      if constexpr (cx != 0) {
        jx += cx * f; qx += cx * gg; pxx += f;
        pxy += (cx * cy) * f; pxz += (cx * cz) * f;
      }
      jy += cy * f; qy += cy * gg; pyy += (cy * cy) * f;
      jz += cz * f; qz += cz * gg; pzz += (cz * cz) * f;
      pyz += (cy * cz) * f;
#pragma unroll
      for (int a = 0; a < M - 1; ++a) {
        const double fa = pop_val(ld(pop + ((int64_t)a * Q + i) * NPAD, r.ps), a, i, kc);
        ra[a] += fa;
        if constexpr (cx != 0) jax[a] += cx * fa;
        jay[a] += cy * fa;
        jaz[a] += cz * fa;
      }
    });
  }
  m.rho = rho;
  m.rhoE = rE;
  m.P6[0] = pxx; m.P6[1] = pyy; m.P6[2] = pzz; m.P6[3] = pxy; m.P6[4] = pxz; m.P6[5] = pyz;
  m.q[0] = qx; m.q[1] = qy; m.q[2] = qz;
  const double inv_rho = 1.0 / rho;
  m.u[0] = jx * inv_rho; m.u[1] = jy * inv_rho; m.u[2] = jz * inv_rho;
  double rsum = 0, jsx = 0, jsy = 0, jsz = 0;
#pragma unroll
  for (int a = 0; a < M - 1; ++a) {
    m.rs[a] = ra[a];
    rsum += ra[a]; jsx += jax[a]; jsy += jay[a]; jsz += jaz[a];
    const bool tiny = fabs(ra[a]) < 1e-300;
    const double inv = tiny ? 0.0 : 1.0 / ra[a];
    m.du0[a][0] = tiny ? 0.0 : jax[a] * inv - m.u[0];
    m.du0[a][1] = tiny ? 0.0 : jay[a] * inv - m.u[1];
    m.du0[a][2] = tiny ? 0.0 : jaz[a] * inv - m.u[2];
  }
  {
    const double rM = rho - rsum;
    const double jM[3] = {jx - jsx, jy - jsy, jz - jsz};
    m.rs[M - 1] = rM;
    const bool tiny = fabs(rM) < 1e-300;
    const double inv = tiny ? 0.0 : 1.0 / rM;
#pragma unroll
    for (int d = 0; d < 3; ++d) m.du0[M - 1][d] = tiny ? 0.0 : jM[d] * inv - m.u[d];
  }
}

// temperature from E - u^2/2 (eq. temperature) by Newton from T0; returns 1 when converged
template <int M>
__device__ __forceinline__ int node_temperature(const Tables &tb, const Macro<M> &m, double T0, double &T_out) {
  double ec[6], dc[5];
#pragma unroll
  for (int k = 0; k < 6; ++k) ec[k] = 0.0;
#pragma unroll
  for (int k = 0; k < 5; ++k) dc[k] = 0.0;
  const double inv_rho = 1.0 / m.rho;
#pragma unroll
  for (int a = 0; a < M; ++a) {
    const double Y = m.rs[a] * inv_rho;
#pragma unroll
    for (int k = 0; k < 6; ++k) ec[k] += Y * tb.ucoef[a][k];
#pragma unroll
    for (int k = 0; k < 5; ++k) dc[k] += Y * tb.cvcoef[a][k];
  }
  const double usq = m.u[0] * m.u[0] + m.u[1] * m.u[1] + m.u[2] * m.u[2];
  const double target = m.rhoE * inv_rho - 0.5 * usq;
  double T = T0;
  int ok = 0;
  for (int it = 0; it < 50; ++it) {
    const double e = ec[0] + T * (ec[1] + T * (ec[2] + T * (ec[3] + T * (ec[4] + T * ec[5])))) - target;
    const double de = dc[0] + T * (dc[1] + T * (dc[2] + T * (dc[3] + T * dc[4])));
    const double dT = -e / de;
    T += dT;
    if (fabs(dT) <= 1e-12 * fabs(T)) {
      ok = 1;
      break;
    }
  }
  T_out = T;
  return ok;
}

template <typename RT>
__device__ __forceinline__ void store_rt(void *base, int64_t idx, RT v) {
  static_cast<RT *>(base)[idx] = v;
}

// ---- the step --------------------------------------------------------------------
constexpr int ISL_BLOCK = 128;    // step kernel

// Per-thread LDS words of the node-local kernel (word w of thread t at w * ISL_BLOCK
// + t: conflict-free).  Values that live across the chemistry and the Stefan-Maxwell
// solve are parked here so that those hold only their own state in registers.  At most
// 40 words for M = 10, so that 512 threads per CU fit in 160 KB.
template <int M>
struct IslWords {
  static constexpr int RS = 0;             // species densities [M]
  static constexpr int G = RS + M;         // g coefficients [10]: A0, A1[3], A2[6]
  static constexpr int C = G + 10;         // concentrations [M], then 1.0; production rates [M-1] after the chemistry
  static constexpr int RD = C;
  static constexpr int BETA = C + M + 1;   // beta_a [M-1]
  static constexpr int WORDS = BETA + M - 1;
};

// The accesses are volatile, through an LDS pointer: the compiler then neither keeps
// the stored values in registers instead of reading them back, nor takes the LDS
// stores for stores that could change the constant tables in global memory.
typedef __attribute__((address_space(3))) volatile double lds_double;

// Phase boundary for the instruction scheduler (emits no instruction): the values a
// later phase reads back from LDS are not pulled up into an earlier one, where they
// would stay live across its register-heavy work.
__device__ __forceinline__ void phase_boundary() { __builtin_amdgcn_sched_barrier(0); }
struct IslStash {
  lds_double *p;   // &words[tid]
  __device__ __forceinline__ void w(int k, double v) const { p[k * ISL_BLOCK] = v; }
  __device__ __forceinline__ double r(int k) const { return p[k * ISL_BLOCK]; }
};

// Precision of the inter-species term F of eq. fStar (a correction whose sum over
// directions vanishes): FP64 for FP64 storage, FP32 for FP32 storage.
template <typename ST>
using FT = typename Fmt<ST>::F;

// coefficients of the collision of one node
template <int M, typename F>
struct CollCoef {
  double u0, u1, u2, rho, zeta;
  double gA0, gA1[3], gA2[6];
  double T;                     // temperature: R_b T = Ra[b] T
  F dv[M][3], tbw[M];
  F omb[M - 1];                 // 1 - 2 beta_a
  double ca[M - 1];             // (1 - omb_a) rho_a + rho_dot_a: exact species mass
  F rcoef[M - 1];
};

// O7 for one direction, mixture f and energy g (eqs. f, g); A_i.X and the q^corr
// part are added by the next pull
template <int M, typename F, typename StFn>
__device__ __forceinline__ void collide_fg(const CollideConsts &kc, const CollCoef<M, F> &cc, int cx, int cy,
                                           int cz, double f, double gv, StFn &&store) {
  const double om = kc.omega;
  const double fcx = cx, fcy = cy, fcz = cz;
  const double wi = w1(cx) * w1(cy) * w1(cz);
  const double u0 = cc.u0, u1 = cc.u1, u2 = cc.u2;
  const double feq = cc.rho * psi_c<double>(cx, u0, u0 * u0 + cc.zeta) * psi_c<double>(cy, u1, u1 * u1 + cc.zeta) *
                     psi_c<double>(cz, u2, u2 * u2 + cc.zeta);
  store(M - 1, (1.0 - om) * f + om * feq);
  const double acc = cc.gA0 + fcx * cc.gA1[0] + fcy * cc.gA1[1] + fcz * cc.gA1[2] + fcx * fcx * cc.gA2[0] +
                     fcy * fcy * cc.gA2[1] + fcz * fcz * cc.gA2[2] + fcx * fcy * cc.gA2[3] + fcx * fcz * cc.gA2[4] +
                     fcy * fcz * cc.gA2[5];
  store(M, (1.0 - om) * gv + wi * acc);
}

// O7 for one direction, the stored species a < M-1 (eq. finalNumericalEquations with
// F_ai of eq. fStar); fa(a) returns the pulled population, store(a, v) writes it.
// Phi_b(u) - Phi_b(u + du_b) is telescoped over the three axis factors, each factor
// difference in closed form, so the difference keeps relative precision:
// Psi_c(xi) - Psi_c(xi + d) = d (s_c (2 xi + d) + t_c), with s_0 = 1, t_0 = 0 and
// s_c = -1/2, t_c = -c/2 for c = +-1 (eq. phis).  Axis factor of species b:
// Psi_c(u_alpha, zeta_b) = A_c(u_alpha) + B_c zeta_b.  The inter-species term is
// evaluated in F; the equilibria that carry the species mass in FP64.
template <int M, typename F, typename FaFn, typename StFn>
__device__ __forceinline__ void collide_species(const CollideConsts &kc, const CollCoef<M, F> &cc, int cx, int cy,
                                                int cz, FaFn &&fa, StFn &&store) {
  const double u0 = cc.u0, u1 = cc.u1, u2 = cc.u2;
  // B_c is -1 or 1/2, so (B_c T) R_b equals B_c (R_b T) exactly
  double BxT = (cx == 0 ? -1.0 : 0.5) * cc.T, ByT = (cy == 0 ? -1.0 : 0.5) * cc.T,
         BzT = (cz == 0 ? -1.0 : 0.5) * cc.T;
  double Ax = psi_c<double>(cx, u0, u0 * u0), Ay = psi_c<double>(cy, u1, u1 * u1),
         Az = psi_c<double>(cz, u2, u2 * u2);
  const F Axf = F(Ax), Ayf = F(Ay), Azf = F(Az), BxTf = F(BxT), ByTf = F(ByT), BzTf = F(BzT);
  const F sx = cx == 0 ? F(1) : F(-0.5), sy = cy == 0 ? F(1) : F(-0.5), sz = cz == 0 ? F(1) : F(-0.5);
  const F tx = F(-0.5) * F(cx), ty = F(-0.5) * F(cy), tz = F(-0.5) * F(cz);
  const F x2 = F(2) * F(u0), y2 = F(2) * F(u1), z2 = F(2) * F(u2);
  // F_a = sum_b invD_ab dd_b, accumulated over b in increasing order
  F Fa[M - 1];
#pragma unroll
  for (int a = 0; a < M - 1; ++a) Fa[a] = F(0);
#pragma unroll
  for (int b = 0; b < M; ++b) {
    F Rb;
    if constexpr (sizeof(F) == 4) Rb = kc.Raf[b]; else Rb = F(kc.Ra[b]);
    const F ex = Axf + BxTf * Rb, ey = Ayf + ByTf * Rb, ez = Azf + BzTf * Rb;
    const F d0 = cc.dv[b][0], d1 = cc.dv[b][1], d2 = cc.dv[b][2];
    const F dx = d0 * (sx * (x2 + d0) + tx), dy = d1 * (sy * (y2 + d1) + ty), dz = d2 * (sz * (z2 + d2) + tz);
    const F rx = ex - dx, ry = ey - dy;
    const F dd = cc.tbw[b] * (dx * ey * ez + rx * dy * ez + rx * ry * dz);
#pragma unroll
    for (int a = 0; a < M - 1; ++a) {
      if (a == b) continue;
      const int lo = a < b ? a : b, hi = a < b ? b : a;
      const int k = lo * M - lo * (lo + 1) / 2 + (hi - lo - 1);
      F c;
      if constexpr (sizeof(F) == 4) c = kc.invDpf[k]; else c = F(kc.invDp[k]);
      Fa[a] += c * dd;
    }
  }
  // the FP64 axis factors are recomputed below rather than kept from above
  opaque(Ax);
  opaque(Ay);
  opaque(Az);
  opaque(BxT);
  opaque(ByT);
  opaque(BzT);
#pragma unroll
  for (int a = 0; a < M - 1; ++a) {
    const double Ra = kc.Ra[a];
    const double phe = (Ax + BxT * Ra) * (Ay + ByT * Ra) * (Az + BzT * Ra);
    store(a, double(cc.omb[a]) * fa(a) + cc.ca[a] * phe + double(cc.rcoef[a] * Fa[a]));
  }
}

// Source of the pull along direction i: padded index of the source cell, and whether
// it is an interior node (then the deferred corrections at it apply) with its index.
struct DirSrc {
  uint32_t ps;
  uint32_t nc;    // interior index of the source, 0 for a ghost source
  bool inner;
};

__device__ __forceinline__ DirSrc dir_src(const Geom &g, int x, int y, int z, int i) {
  const int cx = i % 3 - 1, cy = (i / 3) % 3 - 1, cz = i / 9 - 1;
  const RowSrc row = row_src(g, y, z, cy, cz);
  int sx = x - cx;
  if (g.per[0]) sx = sx < 0 ? sx + g.nx : (sx >= g.nx ? sx - g.nx : sx);
  const bool outx = sx < 0 || sx >= g.nx;
  DirSrc d;
  d.ps = row.prow + (uint32_t)(sx + g.px);
  d.inner = !(row.nrow < 0 || outx);
  d.nc = d.inner ? (uint32_t)(row.nrow + sx) : 0u;
  return d;
}

// Values of f and g pulled along one direction, with the deferred corrections at the
// source; all loads without branches, so that they are issued together (a ghost
// source reads the corrections of node 0 and discards them).
template <typename ST>
struct PulledFG {
  ST f, g;
  typename Fmt<ST>::Side x, cg[3];
  bool inner;
};

template <int M, typename ST>
__device__ __forceinline__ void pull_fg(const Geom &g, const ST *__restrict__ src,
                                        const typename Fmt<ST>::Side *__restrict__ corr,
                                        int x, int y, int z, int i, PulledFG<ST> &p) {
  const int cx = i % 3 - 1, cy = (i / 3) % 3 - 1;
  const DirSrc d = dir_src(g, x, y, z, i);
  const int64_t NPAD = g.NPAD, N = g.N;
  p.inner = d.inner;
  p.f = ld(src + ((int64_t)(M - 1) * Q + i) * NPAD, d.ps);
  p.g = ld(src + ((int64_t)M * Q + i) * NPAD, d.ps);
  const int axis = cx != 0 ? 0 : (cy != 0 ? 1 : 2);
  p.x = ld(corr + axis * N, d.nc);
#pragma unroll
  for (int k = 0; k < 3; ++k) p.cg[k] = ld(corr + (3 + k) * N, d.nc);
}

template <int M, typename ST, typename F>
__device__ __forceinline__ void collide_pulled_fg(const CollideConsts &kc, const CollCoef<M, F> &cc, int i,
                                                  const PulledFG<ST> &p, ST *__restrict__ dst, int64_t NPAD,
                                                  uint32_t pself) {
  const int cx = i % 3 - 1, cy = (i / 3) % 3 - 1, cz = i / 9 - 1;
  using Side = typename Fmt<ST>::Side;
  // deferred A_i.X on the axis directions (eq. Ai), rounded to the side precision
  const double xs = (cx * cx + cy * cy + cz * cz) == 1 ? 0.5 * double(cx + cy + cz) : 0.0;
  const double xc = double(Side(xs * double(p.x)));
  const double f = pop_val(p.f, M - 1, i, kc) + (p.inner ? xc : 0.0);
  // deferred Fourier-correction flux 3 w_i c_i . Cg (eq. corrFourier)
  const double w3 = 3.0 * (w1(cx) * w1(cy) * w1(cz));
  const double d = double(cx) * double(p.cg[0]) + double(cy) * double(p.cg[1]) + double(cz) * double(p.cg[2]);
  const double gc = double(Side(w3 * d));
  const double gv = pop_val(p.g, M, i, kc) + (p.inner ? gc : 0.0);
  collide_fg<M, F>(kc, cc, cx, cy, cz, f, gv, [&](int set, double v) {
    st(dst + ((int64_t)set * Q + i) * NPAD, pself, pop_enc<ST>(v, set, i, kc));
  });
}

template <int M, typename ST>
struct PulledS {
  ST fa[M - 1];
};

template <int M, typename ST>
__device__ __forceinline__ void pull_species(const Geom &g, const ST *__restrict__ src, int x, int y, int z, int i,
                                             PulledS<M, ST> &p) {
  const DirSrc d = dir_src(g, x, y, z, i);
  const int64_t NPAD = g.NPAD;
#pragma unroll
  for (int a = 0; a < M - 1; ++a) p.fa[a] = ld(src + ((int64_t)a * Q + i) * NPAD, d.ps);
}

template <int M, typename F>
__device__ __forceinline__ void opaque_species(CollCoef<M, F> &cc) {
  opaque(cc.u0);
  opaque(cc.u1);
  opaque(cc.u2);
  opaque(cc.T);
#pragma unroll
  for (int a = 0; a < M; ++a) {
    opaque(cc.tbw[a]);
#pragma unroll
    for (int d = 0; d < 3; ++d) opaque(cc.dv[a][d]);
  }
}

template <int M, typename ST, typename F>
__device__ __forceinline__ void collide_pulled_species(const CollideConsts &kc, const CollCoef<M, F> &cc, int i,
                                                       const PulledS<M, ST> &p, ST *__restrict__ dst, int64_t NPAD,
                                                       uint32_t pself) {
  const int cx = i % 3 - 1, cy = (i / 3) % 3 - 1, cz = i / 9 - 1;
  collide_species<M, F>(
      kc, cc, cx, cy, cz, [&](int a) { return pop_val(p.fa[a], a, i, kc); },
      [&](int a, double v) { st(dst + ((int64_t)a * Q + i) * NPAD, pself, pop_enc<ST>(v, a, i, kc)); });
}

// ---- step, part 1: the node-local kernel ----------------------------------------------
// Values of all stored sets pulled along one direction, with the deferred corrections
// at the source (branch-free, so that the loads are issued together).
template <int M, typename ST>
struct PulledAll {
  ST f, g, fa[M - 1];
  typename Fmt<ST>::Side x, cg[3];
  bool inner;
};

template <int M, typename ST>
__device__ __forceinline__ void pull_all(const Geom &g, const ST *__restrict__ src,
                                         const typename Fmt<ST>::Side *__restrict__ corr,
                                         int x, int y, int z, int i, PulledAll<M, ST> &p) {
  const int cx = i % 3 - 1, cy = (i / 3) % 3 - 1;
  const DirSrc d = dir_src(g, x, y, z, i);
  const int64_t NPAD = g.NPAD, N = g.N;
  p.inner = d.inner;
  p.f = ld(src + ((int64_t)(M - 1) * Q + i) * NPAD, d.ps);
  p.g = ld(src + ((int64_t)M * Q + i) * NPAD, d.ps);
#pragma unroll
  for (int a = 0; a < M - 1; ++a) p.fa[a] = ld(src + ((int64_t)a * Q + i) * NPAD, d.ps);
  const int axis = cx != 0 ? 0 : (cy != 0 ? 1 : 2);
  p.x = ld(corr + axis * N, d.nc);
#pragma unroll
  for (int k = 0; k < 3; ++k) p.cg[k] = ld(corr + (3 + k) * N, d.nc);
}

// O1 (eqs. Pa, sumfDotc, g0momTotalEnergy): add direction i to the moments
template <int M, typename ST>
__device__ __forceinline__ void add_moments(int i, const PulledAll<M, ST> &p, const CollideConsts &kc,
                                            double (&mo)[14], double (&sp)[M - 1][4]) {
  using Side = typename Fmt<ST>::Side;
  const int cx = i % 3 - 1, cy = (i / 3) % 3 - 1, cz = i / 9 - 1;
  const double xs = (cx * cx + cy * cy + cz * cz) == 1 ? 0.5 * double(cx + cy + cz) : 0.0;
  const double xc = double(Side(xs * double(p.x)));
  const double f = pop_val(p.f, M - 1, i, kc) + (p.inner ? xc : 0.0);
  const double w3 = 3.0 * (w1(cx) * w1(cy) * w1(cz));
  const double d = double(cx) * double(p.cg[0]) + double(cy) * double(p.cg[1]) + double(cz) * double(p.cg[2]);
  const double gc = double(Side(w3 * d));
  const double gv = pop_val(p.g, M, i, kc) + (p.inner ? gc : 0.0);
  const double fx = cx, fy = cy, fz = cz;
  // rho, j (3), P (xx yy zz xy xz yz), rho E, q (3)
  mo[0] += f;
  mo[1] += fx * f;
  mo[2] += fy * f;
  mo[3] += fz * f;
  mo[4] += (fx * fx) * f;
  mo[5] += (fy * fy) * f;
  mo[6] += (fz * fz) * f;
  mo[7] += (fx * fy) * f;
  mo[8] += (fx * fz) * f;
  mo[9] += (fy * fz) * f;
  mo[10] += gv;
  mo[11] += fx * gv;
  mo[12] += fy * gv;
  mo[13] += fz * gv;
#pragma unroll
  for (int a = 0; a < M - 1; ++a) {
    const double fa = pop_val(p.fa[a], a, i, kc);
    sp[a][0] += fa;
    sp[a][1] += fx * fa;
    sp[a][2] += fy * fa;
    sp[a][3] += fz * fa;
  }
}

// Moments of the pulled state (O1) and everything of the collision that is local to the
// node: temperature (O2), production rates (O3), Stefan-Maxwell solve (O4), the
// collision coefficients cc, and the side channel of the stencils (O5).  No global
// store happens before the side channel at the end, so that the constant tables are
// read with scalar loads throughout.
template <int M, typename ST>
__device__ __forceinline__ void node_local(const Geom &g, const Buffers &b, const CollideConsts &kc,
                                           const IslStash &sh, int64_t n, int x, int y, int z, int cur,
                                           CollCoef<M, FT<ST>> &cc) {
  using SW = IslWords<M>;
  using F = FT<ST>;
  using Side = typename Fmt<ST>::Side;
  const Tables &tb = *b.tab;
  const ST *__restrict__ src = static_cast<const ST *>(b.pop[cur]);
  const Side *__restrict__ corr = static_cast<const Side *>(b.corr);
  const int64_t N = g.N;
  const double T0 = b.T[n];
  (void)N;

  // O1: moments; the loads of direction i+1 are in flight while direction i is summed
  Macro<M> m;
  {
    double mo[14], sp[M - 1][4];
#pragma unroll
    for (int k = 0; k < 14; ++k) mo[k] = 0.0;
#pragma unroll
    for (int a = 0; a < M - 1; ++a)
#pragma unroll
      for (int k = 0; k < 4; ++k) sp[a][k] = 0.0;
    PulledAll<M, ST> pa, pb;
    pull_all<M, ST>(g, src, corr, x, y, z, 0, pa);
#pragma unroll 1
    for (int i = 0; i < Q - 1; i += 2) {
      pull_all<M, ST>(g, src, corr, x, y, z, i + 1, pb);
      add_moments<M, ST>(i, pa, kc, mo, sp);
      pull_all<M, ST>(g, src, corr, x, y, z, i + 2, pa);
      add_moments<M, ST>(i + 1, pb, kc, mo, sp);
    }
    add_moments<M, ST>(Q - 1, pa, kc, mo, sp);
    m.rho = mo[0];
    const double inv_rho = 1.0 / mo[0];
    m.u[0] = mo[1] * inv_rho;
    m.u[1] = mo[2] * inv_rho;
    m.u[2] = mo[3] * inv_rho;
#pragma unroll
    for (int k = 0; k < 6; ++k) m.P6[k] = mo[4 + k];
    m.rhoE = mo[10];
#pragma unroll
    for (int d = 0; d < 3; ++d) m.q[d] = mo[11 + d];
    // species a < M-1, and the slaved species M-1 (eq. strongest); u_a - u guarded
    double rsum = 0, jsx = 0, jsy = 0, jsz = 0;
#pragma unroll
    for (int a = 0; a < M - 1; ++a) {
      m.rs[a] = sp[a][0];
      rsum += sp[a][0]; jsx += sp[a][1]; jsy += sp[a][2]; jsz += sp[a][3];
      const bool tiny = fabs(sp[a][0]) < 1e-300;
      const double inv = tiny ? 0.0 : 1.0 / sp[a][0];
#pragma unroll
      for (int d = 0; d < 3; ++d) m.du0[a][d] = tiny ? 0.0 : sp[a][1 + d] * inv - m.u[d];
    }
    const double rM = mo[0] - rsum;
    const double jM[3] = {mo[1] - jsx, mo[2] - jsy, mo[3] - jsz};
    m.rs[M - 1] = rM;
    const bool tiny = fabs(rM) < 1e-300;
    const double inv = tiny ? 0.0 : 1.0 / rM;
#pragma unroll
    for (int d = 0; d < 3; ++d) m.du0[M - 1][d] = tiny ? 0.0 : jM[d] * inv - m.u[d];
  }

  phase_boundary();
  uint32_t anom = 0;
  const double rho = m.rho;
  const double inv_rho = 1.0 / rho;
  if (!(rho > 0.0) || !(m.rs[M - 1] > 0.0)) anom |= LBM_ANOM_NEG_DENSITY;
  // O2: temperature, mixture gas constant, pressure, enthalpies
  double T;
  if (!node_temperature<M>(tb, m, T0, T)) anom |= LBM_ANOM_NEWTON;
  if (!isfinite(T) || !isfinite(rho) || !isfinite(m.rhoE)) anom |= LBM_ANOM_NONFINITE;
  const double invT = 1.0 / T;
  double zeta = 0.0;
#pragma unroll
  for (int a = 0; a < M; ++a) zeta += m.rs[a] * inv_rho * tb.Ra[a];
  zeta *= T;
  const double P = rho * zeta;
  double Hmix = 0.0;
#pragma unroll
  for (int a = 0; a < M; ++a) {
    const double Ha = tb.Ra[a] * T * h_RT(tb.nasa[a], T, invT);
    Hmix += m.rs[a] * inv_rho * Ha;
    sh.w(SW::RS + a, m.rs[a]);
  }
  const double u0 = m.u[0], u1 = m.u[1], u2 = m.u[2];
  // g collision coefficients (eq. g folded with eqs. gieq, geq1mom, geq2mom,
  // gstareq1mom): g' = (1-omega) g + w_i [A0 + A1.c + A2 : c c] with
  // A1 = 3 omega q^eq + 3 V, V = (omega-omega1)(q - u.(P - P^eq) - q^eq)
  //      + omega1 rho sum_a H_a Y_a du_a (the last term is added after the solve)
  {
    const double usq = m.u[0] * m.u[0] + m.u[1] * m.u[1] + m.u[2] * m.u[2];
    const double h2 = Hmix + 0.5 * usq;
    const double *u = m.u;
    double qeq[3], Peq[6], Req[6];
#pragma unroll
    for (int d = 0; d < 3; ++d) qeq[d] = h2 * rho * u[d];
    const int ia[6] = {0, 1, 2, 0, 0, 1}, ib[6] = {0, 1, 2, 1, 2, 2};
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      Peq[k] = (k < 3 ? rho * zeta : 0.0) + rho * u[ia[k]] * u[ib[k]];
      Req[k] = h2 * Peq[k] + P * u[ia[k]] * u[ib[k]];
    }
    const double om_d = tb.omega, om1 = tb.omega1;
    const int sym[3][3] = {{0, 3, 4}, {3, 1, 5}, {4, 5, 2}};
    const double trR = Req[0] + Req[1] + Req[2];
    sh.w(SW::G + 0, om_d * (2.5 * m.rhoE - 1.5 * trR));
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      double uP = 0.0;
#pragma unroll
      for (int c = 0; c < 3; ++c) uP += u[c] * (m.P6[sym[c][d]] - Peq[sym[c][d]]);
      sh.w(SW::G + 1 + d, om_d * 3.0 * qeq[d] + 3.0 * (om_d - om1) * (m.q[d] - uP - qeq[d]));
    }
#pragma unroll
    for (int k = 0; k < 6; ++k)
      sh.w(SW::G + 4 + k, om_d * (k < 3 ? 4.5 * Req[k] - 1.5 * m.rhoE : 9.0 * Req[k]));  // off-diagonal twice
  }
  // right-hand side u_a - u of eq. transform1, kept in registers for the solve
  double du[M][3];
#pragma unroll
  for (int a = 0; a < M; ++a)
#pragma unroll
    for (int d = 0; d < 3; ++d) du[a][d] = m.du0[a][d];

  phase_boundary();
  // O3: production rates (mass action, K_c from the NASA-7 Gibbs function).  The
  // concentrations sit in LDS with a constant 1 after them, so that each side of a
  // reaction is a product over a padded list of species indices.
  {
    const double lnT = log(T);
    double gib[M], wd[M];
#pragma unroll
    for (int a = 0; a < M; ++a) {
      sh.w(SW::C + a, sh.r(SW::RS + a) * tb.conc_scale[a]);
      wd[a] = 0.0;
      gib[a] = h_RT(tb.nasa[a], T, invT) - s_R(tb.nasa[a], T, lnT);
    }
    sh.w(SW::C + M, 1.0);
    const double ln_c0 = tb.ln_c0_const - lnT;
    for (int k = 0; k < tb.R; ++k) {
      const double lnkf = tb.lnA[k] + tb.bexp[k] * lnT - tb.Ta[k] * invT;
      double fwd = exp(lnkf);
      for (int r = 0; r < tb.nreac[k]; ++r) fwd *= sh.r(SW::C + tb.reac_idx[k][r]);
      double rev = 0.0;
      if (tb.rev[k]) {
        double dG = 0.0;
#pragma unroll
        for (int a = 0; a < M; ++a) dG += tb.dnu_a[k][a] * gib[a];
        const double lnKc = -dG + tb.dnu[k] * ln_c0;
        rev = exp(lnkf - lnKc);
        for (int r = 0; r < tb.nprod[k]; ++r) rev *= sh.r(SW::C + tb.prod_idx[k][r]);
      }
      const double qk = fwd - rev;
#pragma unroll
      for (int a = 0; a < M; ++a) wd[a] += tb.dnu_a[k][a] * qk;
    }
#pragma unroll
    for (int a = 0; a < M - 1; ++a) sh.w(SW::RD + a, tb.rdot_scale[a] * wd[a]);
  }

  phase_boundary();
  // O4: Stefan-Maxwell relaxation and diffusion velocities (eqs. tauab, transform1).
  // The matrix is A_ab = -K_ab Y_b / 2 (a != b), A_aa = 1 + 1/(2 tau_a), with the
  // symmetric 1/tau_ab = K_ab = (R_a T)(R_b T) / ((R T) D_ab).  A = B diag(Y) with B
  // symmetric, and every Schur complement of Gaussian elimination on A keeps that
  // form, so the elimination (no pivoting: A is strictly row-diagonally dominant) runs
  // on the lower triangle of B and the diagonal of A, with the multipliers of the
  // elimination on A itself.
  {
    constexpr int NP = M * (M - 1) / 2;
    double Bl[NP], Ad[M], Yb[M], zl[M];
    const double inv_zeta = 1.0 / zeta;
#pragma unroll
    for (int a = 0; a < M; ++a) {
      Yb[a] = sh.r(SW::RS + a) * inv_rho;
      zl[a] = tb.Ra[a] * T;
      Ad[a] = 0.0;
    }
    // packed lower triangle: (r, c), c < r, at r (r - 1) / 2 + c
#pragma unroll
    for (int a = 0; a < M; ++a)
#pragma unroll
      for (int c = a + 1; c < M; ++c) {
        const int k = a * M - a * (a + 1) / 2 + (c - a - 1);
        const double K = zl[a] * zl[c] * tb.invDp[k] * inv_zeta;
        Bl[c * (c - 1) / 2 + a] = -0.5 * K;
        Ad[a] += Yb[c] * K;
        Ad[c] += Yb[a] * K;
      }
#pragma unroll
    for (int a = 0; a < M; ++a) {
      // beta_a = dt / (2 tau_a + dt) with 1/tau_a = sum_b Y_b / tau_ab (eqs. fStar, tauab)
      if (a < M - 1) sh.w(SW::BETA + a, Ad[a] / (Ad[a] + 2.0));
      Ad[a] = 1.0 + 0.5 * Ad[a];
    }
#pragma unroll
    for (int k = 0; k < M; ++k) {
      const double piv = 1.0 / Ad[k];
#pragma unroll
      for (int r = k + 1; r < M; ++r) {
        const double brk = Bl[r * (r - 1) / 2 + k];
        const double l = brk * Yb[k] * piv;      // A_rk / A_kk
#pragma unroll
        for (int c = k + 1; c < r; ++c) Bl[r * (r - 1) / 2 + c] -= l * Bl[c * (c - 1) / 2 + k];
        Ad[r] -= l * (brk * Yb[r]);               // A_rr -= l A_kr, A_kr = B_rk Y_r
#pragma unroll
        for (int d = 0; d < 3; ++d) du[r][d] -= l * du[k][d];
      }
    }
#pragma unroll
    for (int r = M - 1; r >= 0; --r) {
      const double inv = 1.0 / Ad[r];
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        double v = du[r][d];
#pragma unroll
        for (int c = r + 1; c < M; ++c) v -= (Bl[c * (c - 1) / 2 + r] * Yb[c]) * du[c][d];
        du[r][d] = v * inv;
      }
    }
  }

  // the solution is materialised here: otherwise the solve is sunk into its uses below
  // and its whole working set stays live into the coefficient phase
#pragma unroll
  for (int a = 0; a < M; ++a)
#pragma unroll
    for (int d = 0; d < 3; ++d) opaque(du[a][d]);
  phase_boundary();
  // O7: collision coefficients.  Everything taken from the constant tables is read
  // before the first store.
  double Ha[M];
#pragma unroll
  for (int a = 0; a < M; ++a) Ha[a] = tb.Ra[a] * T * h_RT(tb.nasa[a], T, invT);
  const double om1 = tb.omega1;
  const bool open_any = tb.open_any != 0;
  {
    const double inv_zeta = 1.0 / zeta;
    double hyd[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int a = 0; a < M; ++a) {
      const double za = tb.Ra[a] * T;
      const double ra = sh.r(SW::RS + a);
      const double HY = Ha[a] * ra * inv_rho;
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        hyd[d] += HY * du[a][d];
        cc.dv[a][d] = F(du[a][d]);
      }
      cc.tbw[a] = F(ra * za);
      if (a < M - 1) {
        const double bt = sh.r(SW::BETA + a);
        const double rdot = sh.r(SW::RD + a);
        // with 1 - 2 beta_a rounded to F, the source coefficient takes 2 beta_a from
        // the rounded value, so that sum_i f_ai' = rho_a + rho_dot_a holds exactly
        cc.omb[a] = F(1.0 - 2.0 * bt);
        if constexpr (sizeof(F) == 4)
          cc.ca[a] = (1.0 - double(cc.omb[a])) * ra + rdot;
        else
          cc.ca[a] = 2.0 * bt * ra + rdot;
        cc.rcoef[a] = F((bt - 1.0) * ra * inv_rho * za * inv_zeta);
      }
    }
    cc.rho = rho;
    cc.u0 = u0;
    cc.u1 = u1;
    cc.u2 = u2;
    cc.zeta = zeta;
    cc.T = T;
    cc.gA0 = sh.r(SW::G + 0);
#pragma unroll
    for (int d = 0; d < 3; ++d) cc.gA1[d] = sh.r(SW::G + 1 + d) + 3.0 * om1 * rho * hyd[d];
#pragma unroll
    for (int k = 0; k < 6; ++k) cc.gA2[k] = sh.r(SW::G + 4 + k);
  }
  // O5: side channel of the stencils and the ghosts
  {
    // in the side precision: the corrections computed from them are held in it
    Side *sY = static_cast<Side *>(b.side_Y), *sw = static_cast<Side *>(b.side_w);
    Side *sphi = static_cast<Side *>(b.side_phi);
    const uint32_t i = (uint32_t)n;
    const double wc = 0.5 * (2.0 - om1) * P;
#pragma unroll
    for (int a = 0; a < M; ++a) {
      st(sY + a * N, i, Side(sh.r(SW::RS + a) * inv_rho));
      st(sw + a * N, i, Side(wc * Ha[a]));
    }
    const double uu[3] = {u0, u1, u2};
#pragma unroll
    for (int d = 0; d < 3; ++d)
      st(sphi + d * N, i, Side(rho * uu[d] * (1.0 - 3.0 * zeta) - rho * uu[d] * uu[d] * uu[d]));
    if (open_any) {
      st(static_cast<Side *>(b.side_rho), i, Side(rho));
#pragma unroll
      for (int d = 0; d < 3; ++d) st(static_cast<Side *>(b.side_u) + d * N, i, Side(uu[d]));
    }
    st(b.T, i, T);
    if (anom) atomicOr(b.status, anom);
  }
}

// O7 + O8 for f and g over the 27 directions: the loads of direction i+1 are in flight
// while direction i is collided; unrolled twice so that the two sets of pulled values
// alternate in registers.
template <int M, typename ST, typename F>
__device__ __forceinline__ void fg_pass(const Geom &g, const ST *__restrict__ src, ST *__restrict__ dst,
                                        const typename Fmt<ST>::Side *__restrict__ corr, const CollideConsts &kc,
                                        const CollCoef<M, F> &cc, int x, int y, int z, uint32_t pself) {
  const int64_t NPAD = g.NPAD;
  PulledFG<ST> pa, pb;
  pull_fg<M, ST>(g, src, corr, x, y, z, 0, pa);
#pragma unroll 1
  for (int i = 0; i < Q - 1; i += 2) {
    pull_fg<M, ST>(g, src, corr, x, y, z, i + 1, pb);
    collide_pulled_fg<M, ST, F>(kc, cc, i, pa, dst, NPAD, pself);
    pull_fg<M, ST>(g, src, corr, x, y, z, i + 2, pa);
    collide_pulled_fg<M, ST, F>(kc, cc, i + 1, pb, dst, NPAD, pself);
  }
  collide_pulled_fg<M, ST, F>(kc, cc, Q - 1, pa, dst, NPAD, pself);
}

// O7 + O8 for the stored species, pipelined like fg_pass
template <int M, typename ST, typename F>
__device__ __forceinline__ void species_pass(const Geom &g, const ST *__restrict__ src, ST *__restrict__ dst,
                                             const CollideConsts &kc, CollCoef<M, F> &cc, int x, int y, int z,
                                             uint32_t pself) {
  const int64_t NPAD = g.NPAD;
  PulledS<M, ST> pa, pb;
  pull_species<M, ST>(g, src, x, y, z, 0, pa);
#pragma unroll 1
  for (int i = 0; i < Q - 1; i += 2) {
    pull_species<M, ST>(g, src, x, y, z, i + 1, pb);
    opaque_species<M, F>(cc);
    collide_pulled_species<M, ST, F>(kc, cc, i, pa, dst, NPAD, pself);
    pull_species<M, ST>(g, src, x, y, z, i + 2, pa);
    opaque_species<M, F>(cc);
    collide_pulled_species<M, ST, F>(kc, cc, i + 1, pb, dst, NPAD, pself);
  }
  collide_pulled_species<M, ST, F>(kc, cc, Q - 1, pa, dst, NPAD, pself);
}

// Fused step: the node-local part, then the collide passes from the coefficients in
// registers.  The populations are read twice, the second time mostly from cache, and
// no record goes through memory.
template <int M, typename ST>
__global__ __launch_bounds__(ISL_BLOCK, 2) void k_step(Geom g, Buffers b, CollideConsts kc, int cur) {
  using F = FT<ST>;
  __shared__ double words[IslWords<M>::WORDS * ISL_BLOCK];
  const IslStash sh{(lds_double *)&words[threadIdx.x]};
  const int64_t n = xcd_tile() * blockDim.x + threadIdx.x;
  if (n >= g.N) return;
  const int x = (int)(n % g.nx);
  const int y = (int)((n / g.nx) % g.ny);
  const int z = (int)(n / ((int64_t)g.nx * g.ny));
  CollCoef<M, F> cc;
  node_local<M, ST>(g, b, kc, sh, n, x, y, z, cur, cc);
  const ST *__restrict__ src = static_cast<const ST *>(b.pop[cur]);
  ST *__restrict__ dst = static_cast<ST *>(b.pop[cur ^ 1]);
  const typename Fmt<ST>::Side *__restrict__ corr = static_cast<const typename Fmt<ST>::Side *>(b.corr);
  const uint32_t pself = ((uint32_t)(z + g.pz) * (uint32_t)g.NY + (uint32_t)(y + g.py)) * (uint32_t)g.NX +
                         (uint32_t)(x + g.px);
  fg_pass<M, ST, F>(g, src, dst, corr, kc, cc, x, y, z, pself);
  species_pass<M, ST, F>(g, src, dst, kc, cc, x, y, z, pself);
}

// ---- psi_alpha = (1/omega - 1/2) d_alpha phi_alpha (isotropic gradient) ------------
template <typename RT>
__global__ __launch_bounds__(256) void k_psi(Geom g, Buffers b) {
  const int64_t n = xcd_tile() * blockDim.x + threadIdx.x;
  if (n >= g.N) return;
  const int x = (int)(n % g.nx), y = (int)((n / g.nx) % g.ny), z = (int)(n / ((int64_t)g.nx * g.ny));
  const RT *phi = static_cast<const RT *>(b.side_phi);
  const int64_t N = g.N;
  const double coef = 1.0 / b.tab->omega - 0.5;
  int xs[3], ys[3], zs[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    xs[k] = nb_coord(x, k - 1, g.nx, g.per[0]);
    ys[k] = nb_coord(y, k - 1, g.ny, g.per[1]);
    zs[k] = nb_coord(z, k - 1, g.nz, g.per[2]);
  }
  double acc[3] = {0, 0, 0};
  static_for<27>([&](auto Ic) {
    constexpr int I = decltype(Ic)::value;
    constexpr int cx = cx_of(I), cy = cy_of(I), cz = cz_of(I);
    const int64_t nn = ((int64_t)zs[cz + 1] * g.ny + ys[cy + 1]) * g.nx + xs[cx + 1];
    constexpr double w = 3.0 * wgt(I);
    if constexpr (cx != 0) acc[0] += (cx * w) * double(phi[0 * N + nn]);
    if constexpr (cy != 0) acc[1] += (cy * w) * double(phi[1 * N + nn]);
    if constexpr (cz != 0) acc[2] += (cz * w) * double(phi[2 * N + nn]);
  });
  RT *psi = static_cast<RT *>(b.psi);
#pragma unroll
  for (int d = 0; d < 3; ++d) psi[d * N + n] = RT(coef * acc[d]);
}

// ---- X_alpha = -d_alpha psi_alpha; Cg = sum_a w_a grad Y_a ---------------------------
template <int M, typename RT, typename CT>
__global__ __launch_bounds__(256) void k_corr(Geom g, Buffers b) {
  const int64_t n = xcd_tile() * blockDim.x + threadIdx.x;
  if (n >= g.N) return;
  const int x = (int)(n % g.nx), y = (int)((n / g.nx) % g.ny), z = (int)(n / ((int64_t)g.nx * g.ny));
  const RT *psi = static_cast<const RT *>(b.psi);
  const RT *Yf = static_cast<const RT *>(b.side_Y);
  const RT *wf = static_cast<const RT *>(b.side_w);
  const int64_t N = g.N;
  int xs[3], ys[3], zs[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    xs[k] = nb_coord(x, k - 1, g.nx, g.per[0]);
    ys[k] = nb_coord(y, k - 1, g.ny, g.per[1]);
    zs[k] = nb_coord(z, k - 1, g.nz, g.per[2]);
  }
  // side fields in RT, sums in FP64
  double wa[M];
#pragma unroll
  for (int a = 0; a < M; ++a) wa[a] = double(wf[a * N + n]);
  double X[3] = {0, 0, 0}, C[3] = {0, 0, 0};
  static_for<27>([&](auto Ic) {
    constexpr int I = decltype(Ic)::value;
    constexpr int cx = cx_of(I), cy = cy_of(I), cz = cz_of(I);
    if constexpr (I != 13) {
      const int64_t nn = ((int64_t)zs[cz + 1] * g.ny + ys[cy + 1]) * g.nx + xs[cx + 1];
      constexpr double w = 3.0 * wgt(I);
      if constexpr (cx != 0) X[0] -= (cx * w) * double(psi[0 * N + nn]);
      if constexpr (cy != 0) X[1] -= (cy * w) * double(psi[1 * N + nn]);
      if constexpr (cz != 0) X[2] -= (cz * w) * double(psi[2 * N + nn]);
      double hy = 0.0;
#pragma unroll
      for (int a = 0; a < M; ++a) hy += wa[a] * double(Yf[a * N + nn]);
      if constexpr (cx != 0) C[0] += (cx * w) * hy;
      if constexpr (cy != 0) C[1] += (cy * w) * hy;
      if constexpr (cz != 0) C[2] += (cz * w) * hy;
    }
  });
  CT *corr = static_cast<CT *>(b.corr);
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    corr[d * N + n] = CT(X[d]);
    corr[(3 + d) * N + n] = CT(C[d]);
  }
}

// ---- equilibria of one state (init and ghosts) --------------------------------------
template <int M, typename ST>
__device__ __forceinline__ void write_equilibria(const Tables &tb, const CollideConsts &kc,
                                                 ST *__restrict__ dst, int64_t NPAD, const int64_t (&pidx)[27],
                                                 double rho, const double *u, double T, const double *Y) {
  double zeta_a[M], zeta = 0.0, H = 0.0, U = 0.0;
  const double invT = 1.0 / T;
#pragma unroll
  for (int a = 0; a < M; ++a) {
    zeta_a[a] = tb.Ra[a] * T;
    zeta += Y[a] * zeta_a[a];
    const double h = h_RT(tb.nasa[a], T, invT);
    H += Y[a] * zeta_a[a] * h;
    U += Y[a] * zeta_a[a] * (h - 1.0);
  }
  const double usq = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
  const double rhoE = rho * (U + 0.5 * usq);
  const double h2 = H + 0.5 * usq, P = rho * zeta;
  double qeq[3], Req[6];
  const int ia[6] = {0, 1, 2, 0, 0, 1}, ib[6] = {0, 1, 2, 1, 2, 2};
  for (int d = 0; d < 3; ++d) qeq[d] = h2 * rho * u[d];
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    const double Peq = (k < 3 ? rho * zeta : 0.0) + rho * u[ia[k]] * u[ib[k]];
    Req[k] = h2 * Peq + P * u[ia[k]] * u[ib[k]];
  }
  const double trR = Req[0] + Req[1] + Req[2];
  const double A0 = 2.5 * rhoE - 1.5 * trR;
  double su[3];
  for (int d = 0; d < 3; ++d) su[d] = u[d] * u[d];
  static_for<27>([&](auto Ic) {
    constexpr int I = decltype(Ic)::value;
    constexpr int cx = cx_of(I), cy = cy_of(I), cz = cz_of(I);
    const int64_t p = pidx[I];
    if (p < 0) return;
    const double fe = rho * psi_c<double>(cx, u[0], su[0] + zeta) * psi_c<double>(cy, u[1], su[1] + zeta) *
                      psi_c<double>(cz, u[2], su[2] + zeta);
    dst[(int64_t)((M - 1) * Q + I) * NPAD + p] = pop_enc<ST>(fe, M - 1, I, kc);
    double acc = A0 + 3.0 * (cx * qeq[0] + cy * qeq[1] + cz * qeq[2]);
    acc += cx * cx * (4.5 * Req[0] - 1.5 * rhoE) + cy * cy * (4.5 * Req[1] - 1.5 * rhoE) +
           cz * cz * (4.5 * Req[2] - 1.5 * rhoE);
    acc += 9.0 * (cx * cy * Req[3] + cx * cz * Req[4] + cy * cz * Req[5]);
    dst[(int64_t)(M * Q + I) * NPAD + p] = pop_enc<ST>(wgt(I) * acc, M, I, kc);
#pragma unroll
    for (int a = 0; a < M - 1; ++a) {
      const double z = zeta_a[a];
      const double fa = rho * Y[a] * psi_c<double>(cx, u[0], su[0] + z) * psi_c<double>(cy, u[1], su[1] + z) *
                        psi_c<double>(cz, u[2], su[2] + z);
      dst[(int64_t)(a * Q + I) * NPAD + p] = pop_enc<ST>(fa, a, I, kc);
    }
  });
}

// initial state: equilibria pushed to where the first pull reads them
template <int M, typename ST>
__global__ __launch_bounds__(128) void k_init(Geom g, Buffers b, CollideConsts kc, const double *rho,
                                              const double *u, const double *T, const double *Y, int cur) {
  const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= g.N) return;
  const int x = (int)(n % g.nx), y = (int)((n / g.nx) % g.ny), z = (int)(n / ((int64_t)g.nx * g.ny));
  const AxisSrc ax = axis_src(x, g.nx, g.per[0]);
  const AxisSrc ay = axis_src(y, g.ny, g.per[1]);
  const AxisSrc az = axis_src(z, g.nz, g.per[2]);
  int64_t pidx[27];
  static_for<27>([&](auto Ic) {
    constexpr int I = decltype(Ic)::value;
    pidx[I] = make_src(g, ax, ay, az, cx_of(I) + 1, cy_of(I) + 1, cz_of(I) + 1).ps;
  });
  const int64_t N = g.N;
  double uu[3] = {u[n], u[N + n], u[2 * N + n]};
  double Yl[M];
#pragma unroll
  for (int a = 0; a < M; ++a) Yl[a] = Y[a * N + n];
  write_equilibria<M, ST>(*b.tab, kc, static_cast<ST *>(b.pop[cur]), g.NPAD, pidx, rho[n], uu, T[n], Yl);
  b.T[n] = T[n];
}

// ghost layer of open faces: equilibria at the adjacent boundary node (Sec. 5.1)
template <int M, typename ST, typename RT>
__global__ __launch_bounds__(128) void k_ghost(Geom g, Buffers b, CollideConsts kc, int cur, int64_t nx_slab,
                                               int64_t ny_slab,
                                               int64_t nz_slab) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int gx, gy, gz;
  if (t < nx_slab) {          // x = -1 or nx, all padded y, z
    const int64_t per = (int64_t)g.NY * g.NZ;
    gx = (t < per) ? -1 : g.nx;
    const int64_t r = t % per;
    gy = (int)(r % g.NY) - g.py;
    gz = (int)(r / g.NY) - g.pz;
  } else if ((t -= nx_slab) < ny_slab) {   // y = -1 or ny, interior x, padded z
    const int64_t per = (int64_t)g.nx * g.NZ;
    gy = (t < per) ? -1 : g.ny;
    const int64_t r = t % per;
    gx = (int)(r % g.nx);
    gz = (int)(r / g.nx) - g.pz;
  } else if ((t -= ny_slab) < nz_slab) {   // z = -1 or nz, interior x, y
    const int64_t per = (int64_t)g.nx * g.ny;
    gz = (t < per) ? -1 : g.nz;
    const int64_t r = t % per;
    gx = (int)(r % g.nx);
    gy = (int)(r / g.nx);
  } else {
    return;
  }
  bool zero_u = false;
  const int gc[3] = {gx, gy, gz};
  const int nn[3] = {g.nx, g.ny, g.nz};
  int a3[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    int v = gc[d];
    if (v < 0) {
      zero_u |= (g.bc[2 * d] == LBM_BC_OPEN_EQ_U0);
      v = 0;
    } else if (v >= nn[d]) {
      zero_u |= (g.bc[2 * d + 1] == LBM_BC_OPEN_EQ_U0);
      v = nn[d] - 1;
    }
    a3[d] = v;
  }
  const int64_t N = g.N;
  const int64_t na = ((int64_t)a3[2] * g.ny + a3[1]) * g.nx + a3[0];
  const RT *srho = static_cast<const RT *>(b.side_rho);
  const RT *su = static_cast<const RT *>(b.side_u);
  const RT *sY = static_cast<const RT *>(b.side_Y);
  double u[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) u[d] = zero_u ? 0.0 : double(su[d * N + na]);
  double Y[M];
#pragma unroll
  for (int a = 0; a < M; ++a) Y[a] = double(sY[a * N + na]);
  const int64_t p = ((int64_t)(gz + g.pz) * g.NY + (gy + g.py)) * g.NX + (gx + g.px);
  // only the directions along which an interior node pulls from this ghost cell
  int64_t pidx[27];
#pragma unroll
  for (int i = 0; i < 27; ++i) {
    const int c[3] = {cx_of(i), cy_of(i), cz_of(i)};
    bool need = true;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const int t = gc[d] + c[d];
      need = need && (g.per[d] || (t >= 0 && t < nn[d]));
    }
    pidx[i] = need ? p : -1;
  }
  write_equilibria<M, ST>(*b.tab, kc, static_cast<ST *>(b.pop[cur ^ 1]), g.NPAD, pidx, double(srho[na]), u,
                          b.T[na], Y);
}

// macroscopic fields of the current state (no state change)
template <int M, typename ST, typename RT>
__global__ __launch_bounds__(128) void k_macros(Geom g, Buffers b, CollideConsts kc, int cur, double *rho,
                                                double *u, double *T, double *P, double *Y) {
  const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= g.N) return;
  const int x = (int)(n % g.nx), y = (int)((n / g.nx) % g.ny), z = (int)(n / ((int64_t)g.nx * g.ny));
  const int64_t N = g.N;
  using Side = typename Fmt<ST>::Side;
  const Corr<Side> cr{static_cast<const Side *>(b.corr), static_cast<const Side *>(b.corr) + 3 * N, N};
  Macro<M> m;
  node_moments<M, ST>(g, static_cast<const ST *>(b.pop[cur]), cr, kc, x, y, z, m);
  const Tables &tb = *b.tab;
  double Tn;
  node_temperature<M>(tb, m, b.T[n], Tn);
  const double inv_rho = 1.0 / m.rho;
  if (rho) rho[n] = m.rho;
  if (u)
    for (int d = 0; d < 3; ++d) u[d * N + n] = m.u[d];
  if (T) T[n] = Tn;
  if (P) {
    double zeta = 0.0;
#pragma unroll
    for (int a = 0; a < M; ++a) zeta += m.rs[a] * inv_rho * tb.Ra[a];
    P[n] = m.rho * zeta * Tn;
  }
  if (Y)
#pragma unroll
    for (int a = 0; a < M; ++a) Y[a * N + n] = m.rs[a] * inv_rho;
}

// pre-collision populations at listed nodes
template <int M, typename ST, typename RT>
__global__ __launch_bounds__(128) void k_export(Geom g, Buffers b, CollideConsts kc, int cur,
                                                const int64_t *nodes, int64_t nn, double *out, double *T_out) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nn) return;
  const int64_t n = nodes[k];
  if (n < 0 || n >= g.N) return;
  const int x = (int)(n % g.nx), y = (int)((n / g.nx) % g.ny), z = (int)(n / ((int64_t)g.nx * g.ny));
  const int64_t N = g.N, NPAD = g.NPAD;
  using Side = typename Fmt<ST>::Side;
  const ST *pop = static_cast<const ST *>(b.pop[cur]);
  const Corr<Side> cr{static_cast<const Side *>(b.corr), static_cast<const Side *>(b.corr) + 3 * N, N};
  const AxisSrc ax = axis_src(x, g.nx, g.per[0]);
  const AxisSrc ay = axis_src(y, g.ny, g.per[1]);
  const AxisSrc az = axis_src(z, g.nz, g.per[2]);
  for (int kyz = 0; kyz < 9; ++kyz) {
    const int ky = kyz % 3, kz = kyz / 3;
    const int cy = ky - 1, cz = kz - 1;
    static_for<3>([&](auto Kx) {
      constexpr int kx = decltype(Kx)::value;
      constexpr int cx = kx - 1;
      const int i = kx + 3 * kyz;
      const Src r = make_src(g, ax, ay, az, kx, ky, kz);
      out[((int64_t)(M - 1) * Q + i) * nn + k] =
          pull_f<cx, ST, Side>(pop + ((int64_t)(M - 1) * Q + i) * NPAD, r, cr, cy, cz, M - 1, i, kc);
      out[((int64_t)M * Q + i) * nn + k] =
          pull_g<cx, ST, Side>(pop + ((int64_t)M * Q + i) * NPAD, r, cr, cy, cz, M, i, kc);
      for (int a = 0; a < M - 1; ++a)
        out[((int64_t)a * Q + i) * nn + k] = pop_val(ld(pop + ((int64_t)a * Q + i) * NPAD, r.ps), a, i, kc);
    });
  }
  if (T_out) T_out[k] = b.T[n];
}

__global__ void k_zero(uint32_t *p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0u;
}

inline unsigned blocks_for(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

// dispatch on (species count, storage)
template <template <int, typename, typename> class K, typename... Args>
hipError_t dispatch(int M, int store, Args &&...args) {
#define LBM_CASE(MM)                                                              \
  case MM:                                                                        \
    switch (store) {                                                              \
      case LBM_STORE_F64: return K<MM, double, Fmt<double>::Side>::run(args...);   \
      case LBM_STORE_F32: return K<MM, float, Fmt<float>::Side>::run(args...);     \
      case LBM_STORE_F16_DEV: return K<MM, _Float16, Fmt<_Float16>::Side>::run(args...); \
      case LBM_STORE_BF16_DEV: return K<MM, __bf16, Fmt<__bf16>::Side>::run(args...);    \
      default: return hipErrorInvalidValue;                                         \
    }
  switch (M) {
    LBM_CASE(2) LBM_CASE(3) LBM_CASE(4) LBM_CASE(5) LBM_CASE(6) LBM_CASE(7) LBM_CASE(8) LBM_CASE(9)
    LBM_CASE(10)
    default: return hipErrorInvalidValue;
  }
#undef LBM_CASE
}

template <int M, typename ST, typename RT>
struct RunStep {
  static hipError_t run(const Geom &g, const Buffers &b, const CollideConsts &kc, int cur, hipStream_t st) {
    hipLaunchKernelGGL((k_step<M, ST>), dim3(blocks_for(g.N, ISL_BLOCK)), dim3(ISL_BLOCK), 0, st, g, b, kc, cur);
    return hipGetLastError();
  }
};
template <int M, typename ST, typename RT>
struct RunCorr {
  static hipError_t run(const Geom &g, const Buffers &b, hipStream_t st) {
    hipLaunchKernelGGL((k_corr<M, RT, RT>), dim3(blocks_for(g.N, 256)), dim3(256), 0, st, g, b);
    return hipGetLastError();
  }
};
template <int M, typename ST, typename RT>
struct RunInit {
  static hipError_t run(const Geom &g, const Buffers &b, const CollideConsts &kc, const double *rho,
                        const double *u, const double *T, const double *Y, int cur, hipStream_t st) {
    hipLaunchKernelGGL((k_init<M, ST>), dim3(blocks_for(g.N, 128)), dim3(128), 0, st, g, b, kc, rho, u, T, Y,
                       cur);
    return hipGetLastError();
  }
};
template <int M, typename ST, typename RT>
struct RunGhost {
  static hipError_t run(const Geom &g, const Buffers &b, const CollideConsts &kc, int cur, hipStream_t st) {
    const int64_t sx = g.px ? 2LL * g.NY * g.NZ : 0;
    const int64_t sy = g.py ? 2LL * g.nx * g.NZ : 0;
    const int64_t sz = g.pz ? 2LL * g.nx * g.ny : 0;
    const int64_t tot = sx + sy + sz;
    if (tot == 0) return hipSuccess;
    hipLaunchKernelGGL((k_ghost<M, ST, RT>), dim3(blocks_for(tot, 128)), dim3(128), 0, st, g, b, kc, cur, sx, sy,
                       sz);
    return hipGetLastError();
  }
};
template <int M, typename ST, typename RT>
struct RunMacros {
  static hipError_t run(const Geom &g, const Buffers &b, const CollideConsts &kc, int cur, double *rho,
                        double *u, double *T, double *P, double *Y, hipStream_t st) {
    hipLaunchKernelGGL((k_macros<M, ST, RT>), dim3(blocks_for(g.N, 128)), dim3(128), 0, st, g, b, kc, cur, rho, u,
                       T, P, Y);
    return hipGetLastError();
  }
};
template <int M, typename ST, typename RT>
struct RunExport {
  static hipError_t run(const Geom &g, const Buffers &b, const CollideConsts &kc, int cur, const int64_t *nodes,
                        int64_t nn, double *out, double *T_out, hipStream_t st) {
    if (nn == 0) return hipSuccess;
    hipLaunchKernelGGL((k_export<M, ST, RT>), dim3(blocks_for(nn, 128)), dim3(128), 0, st, g, b, kc, cur, nodes,
                       nn, out, T_out);
    return hipGetLastError();
  }
};

}  // namespace

hipError_t launch_step(const Geom &g, const Buffers &b, const CollideConsts &kc, int store, int cur,
                       hipStream_t st) {
  return dispatch<RunStep>(g.M, store, g, b, kc, cur, st);
}

hipError_t launch_psi(const Geom &g, const Buffers &b, int store, hipStream_t st) {
  if (store == LBM_STORE_F64)
    hipLaunchKernelGGL((k_psi<Fmt<double>::Side>), dim3(blocks_for(g.N, 256)), dim3(256), 0, st, g, b);
  else if (store == LBM_STORE_F32)
    hipLaunchKernelGGL((k_psi<Fmt<float>::Side>), dim3(blocks_for(g.N, 256)), dim3(256), 0, st, g, b);
  else
    hipLaunchKernelGGL((k_psi<float>), dim3(blocks_for(g.N, 256)), dim3(256), 0, st, g, b);
  return hipGetLastError();
}

hipError_t launch_corr(const Geom &g, const Buffers &b, int store, hipStream_t st) {
  return dispatch<RunCorr>(g.M, store, g, b, st);
}

hipError_t launch_init(const Geom &g, const Buffers &b, const CollideConsts &kc, int store, const double *rho,
                       const double *u, const double *T, const double *Y, int cur, hipStream_t st) {
  return dispatch<RunInit>(g.M, store, g, b, kc, rho, u, T, Y, cur, st);
}

hipError_t launch_ghost(const Geom &g, const Buffers &b, const CollideConsts &kc, int store, int cur,
                        hipStream_t st) {
  return dispatch<RunGhost>(g.M, store, g, b, kc, cur, st);
}

hipError_t launch_macros(const Geom &g, const Buffers &b, const CollideConsts &kc, int store, int cur,
                         double *rho, double *u, double *T, double *P, double *Y, hipStream_t st) {
  return dispatch<RunMacros>(g.M, store, g, b, kc, cur, rho, u, T, P, Y, st);
}

hipError_t launch_export(const Geom &g, const Buffers &b, const CollideConsts &kc, int store, int cur,
                         const int64_t *nodes, int64_t n_nodes, double *out, double *T_out, hipStream_t st) {
  return dispatch<RunExport>(g.M, store, g, b, kc, cur, nodes, n_nodes, out, T_out, st);
}

hipError_t launch_zero(void *p, int64_t n_words32, hipStream_t st) {
  if (n_words32 <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_zero, dim3(blocks_for(n_words32, 256)), dim3(256), 0, st, static_cast<uint32_t *>(p),
                     n_words32);
  return hipGetLastError();
}

}  // namespace lbm
