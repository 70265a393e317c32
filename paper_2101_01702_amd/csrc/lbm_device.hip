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
#include <mutex>
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

// first and last x of the segment that holds x, and the segment's index
struct XSeg {
  int x0, x1, s;
};
__device__ __forceinline__ XSeg x_segment(const Geom &g, int x) {
  if (g.nseg <= 1) return XSeg{0, g.nx - 1, 0};
  const int s = g.x_seg[x];
  return XSeg{g.seg_off[s], g.seg_off[s + 1] - 1, s};
}

// x ghost cells are coded as x = -1 - q, q = 2 s (before segment s) or 2 s + 1 (after it)
__device__ __forceinline__ int x_ghost_code(int s, int side) { return -1 - (2 * s + side); }

// index in a plane of cell x of padded row prow: in the row, or, for a coded x ghost
// cell, one of the x ghost cells after the rows
__device__ __forceinline__ uint32_t cell_index(const Geom &g, int x, uint32_t prow) {
  if (x < 0) return (uint32_t)(g.XG + (int64_t)(-1 - x) * g.NY * g.NZ) + prow;
  return prow * (uint32_t)g.NX + (uint32_t)x;
}

// x sources x - c for c = -1, 0, +1: wrapped on a periodic axis; on an open one a
// source beyond the end of the lane's segment is that end's coded x ghost cell
__device__ __forceinline__ AxisSrc axis_src_x(const Geom &g, int x) {
  AxisSrc a;
  if (g.per[0]) return axis_src(x, g.nx, true);
  const XSeg sg = x_segment(g, x);
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const int v = x - (k - 1);
    a.out[k] = v < sg.x0 || v > sg.x1;
    a.s[k] = v < sg.x0 ? x_ghost_code(sg.s, 0) : (v > sg.x1 ? x_ghost_code(sg.s, 1) : v);
  }
  return a;
}

__device__ __forceinline__ Src make_src(const Geom &g, const AxisSrc &ax, const AxisSrc &ay,
                                        const AxisSrc &az, int kx, int ky, int kz) {
  Src r;
  const uint32_t sy = (uint32_t)(ay.s[ky] + g.py), sz = (uint32_t)(az.s[kz] + g.pz);
  r.ps = cell_index(g, ax.s[kx], sz * (uint32_t)g.NY + sy);
  const bool out = ax.out[kx] || ay.out[ky] || az.out[kz];
  r.ns = out ? -1 : (az.s[kz] * g.ny + ay.s[ky]) * g.nx + ax.s[kx];
  return r;
}

// source of the pull for a uniform (cy, cz) and a compile-time x index: the y and z
// coordinates are wrapped or left in the ghost layer without table lookups
struct RowSrc {
  uint32_t prow;   // padded row index (z + pz) NY + (y + py)
  int32_t nrow;    // interior row index times nx, or -1 when (y, z) is in the ghost layer
};

__device__ __forceinline__ RowSrc row_src(const Geom &g, int y, int z, int cy, int cz) {
  int sy = y - cy, sz = z - cz;
  if (g.per[1]) sy = sy < 0 ? sy + g.ny : (sy >= g.ny ? sy - g.ny : sy);
  if (g.per[2]) sz = sz < 0 ? sz + g.nz : (sz >= g.nz ? sz - g.nz : sz);
  const bool out = sy < 0 || sy >= g.ny || sz < 0 || sz >= g.nz;
  RowSrc r;
  r.prow = (uint32_t)(sz + g.pz) * (uint32_t)g.NY + (uint32_t)(sy + g.py);
  r.nrow = out ? -1 : (sz * g.ny + sy) * g.nx;
  return r;
}

__device__ __forceinline__ Src src_from_row(const Geom &g, const RowSrc &row, const AxisSrc &ax, int kx) {
  Src r;
  r.ps = cell_index(g, ax.s[kx], row.prow);
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
template <typename ST, typename K>
__device__ __forceinline__ double pop_val(ST raw, int s, int i, const K &kc) {
  if constexpr (Fmt<ST>::dev)
    return double(fmaf(kc.sc[s], float(raw), kc.ref[s][i]));
  else
    return double(raw);
}
// stored form of the population value v of set s along direction i: rounded to FP32,
// then to the 16-bit format.  The FP32 value is made opaque so that the two roundings
// stay two hardware conversions; folded into one double -> half conversion, the
// compiler emulates it in integer instructions (about 30 per value).
template <typename ST, typename K>
__device__ __forceinline__ ST pop_enc(double v, int s, int i, const K &kc) {
  if constexpr (Fmt<ST>::dev) {
    float t = float((v - double(kc.ref[s][i])) * double(kc.isc[s]));
    opaque(t);
    return ST(t);
  } else {
    return ST(v);
  }
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

// deferred corrections, in padded planes whose ghost cells hold zero
template <typename CT>
struct Corr {
  const CT *X;    // [3][NPAD]
  const CT *Cg;   // [3][NPAD]
  int64_t NPAD;
};

// pulled value of the mixture f along c = (CX, cy, cz) with the deferred A_i.X term;
// the corrections are held in the storage precision ST and added in FP64, the same
// way in every kernel that pulls
template <int CX, typename ST, typename CT>
__device__ __forceinline__ double pull_f(const ST *__restrict__ base, const Src &r, const Corr<CT> &cr, int cy,
                                         int cz, int s, int i, const CollideConsts &kc) {
  double v = pop_val(ld(base, r.ps), s, i, kc);
  {
    // the correction loads are unconditional and the terms selected: a branch around a
    // load would wait for every load in flight at its join
    const uint32_t ns = r.ps;   // padded planes: zero at open ghosts, mirrored at symmetry ghosts
    if constexpr (CX != 0) {
      const double x0 = double(ld(cr.X, ns));
      v += (cy == 0 && cz == 0) ? double(CT(0.5 * CX * x0)) : 0.0;
    } else {
      const double x1 = double(ld(cr.X + cr.NPAD, ns)), x2 = double(ld(cr.X + 2 * cr.NPAD, ns));
      v += (cy != 0 && cz == 0) ? double(CT(0.5 * cy * x1)) : 0.0;
      v += (cy == 0 && cz != 0) ? double(CT(0.5 * cz * x2)) : 0.0;
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
  {
    const uint32_t ns = r.ps;   // padded planes: zero at open ghosts, mirrored at symmetry ghosts
    double d = 0.0;
    if constexpr (CX != 0) d += CX * double(ld(cr.Cg, ns));
    const double c1 = double(ld(cr.Cg + cr.NPAD, ns)), c2 = double(ld(cr.Cg + 2 * cr.NPAD, ns));
    d += cy != 0 ? cy * c1 : 0.0;
    d += cz != 0 ? cz * c2 : 0.0;
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

// factor of the diffusivities at temperature T, 1 / (T / T_ref)^n = exp(n (ln T_ref - ln T)):
// 1/D_ab(T) = s 1/D_ab (exactly 1 for constant diffusivities)
template <typename TB>
__device__ __forceinline__ double inv_diff_scale(const TB &tb, double T) {
  return tb.dexp != 0.0 ? exp(tb.dexp * (tb.ln_dTref - log(T))) : 1.0;
}

// relaxation rates at temperature T: the constants omega, omega1, or the rates whose
// factors 1/omega - 1/2 and 1/omega1 - 1/2 (eqs. mu, lambda) scale with (T / T_ref)^n
template <bool VT = true, typename TB>
__device__ __forceinline__ void relax_rates(const TB &tb, double T, double &om, double &om1) {
  if (!VT || tb.vexp == 0.0) {
    om = tb.omega;
    om1 = tb.omega1;
  } else {
    const double s = exp(tb.vexp * (log(T) - tb.ln_vTref));
    om = 1.0 / (0.5 + tb.c_om * s);
    om1 = 1.0 / (0.5 + tb.c_om1 * s);
  }
}

// ---- thermodynamics (eqs. specHa, Umix; NASA-7) -------------------------------------
template <typename P>
__device__ __forceinline__ double h_RT(P a, double T, double invT) {
  return a[0] + T * (a[1] * 0.5 + T * (a[2] * (1.0 / 3.0) + T * (a[3] * 0.25 + T * (a[4] * 0.2)))) +
         a[5] * invT;
}
template <typename P>
__device__ __forceinline__ double s_R(P a, double T, double lnT) {
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
  const AxisSrc ax = axis_src_x(g, x);
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
template <int M, typename TB>
__device__ __forceinline__ int node_temperature(const TB &tb, const Macro<M> &m, double T0, double &T_out) {
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

// ---- lattice passes of the step kernel ------------------------------------------------
// The passes over the 27 directions go row by row: row r = (cy+1) + 3 (cz+1) holds the
// directions i = 3 r + cx + 1, cx = -1, 0, 1.  cy and cz are uniform and cx is a
// compile-time constant, so that every factor that depends on (cy, cz) alone is formed
// once per row.
//
// Each (set, direction) plane is read and written through a buffer resource (base and
// size in scalar registers) with the lane's byte offset in one vector register: the
// address arithmetic of a load or store is scalar.  An offset outside the plane reads
// zero and drops a store instead of touching other memory.
using Rsrc = __amdgpu_buffer_rsrc_t;
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ Rsrc plane_rsrc(const void *p, uint32_t bytes) {
  // word 3 of an untyped buffer with a 32-bit data format (gfx9 family)
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0, (int)bytes, 0x00020000);
}
template <typename T>
__device__ __forceinline__ T bld(Rsrc r, uint32_t off) {
  if constexpr (sizeof(T) == 8)
    return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(r, (int)off, 0, 0));
  else if constexpr (sizeof(T) == 4)
    return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(r, (int)off, 0, 0));
  else
    return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b16(r, (int)off, 0, 0));
}
template <typename T>
__device__ __forceinline__ void bst(Rsrc r, uint32_t off, T v) {
  if constexpr (sizeof(T) == 8)
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, (int)off, 0, 0);
  else if constexpr (sizeof(T) == 4)
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, (int)off, 0, 0);
  else
    __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(unsigned short, v), r, (int)off, 0, 0);
}
// plane k of NPAD elements of type T starting at buf (a padded plane is below 2 GiB)
template <typename T>
__device__ __forceinline__ Rsrc plane(const void *buf, const Geom &g, int k) {
  const uint32_t bytes = (uint32_t)g.NPAD * (uint32_t)sizeof(T);
  return plane_rsrc(static_cast<const char *>(buf) + (uint64_t)k * bytes, bytes);
}

// The constants of the collision, read through a constant-address-space pointer: loads
// through it are scalar, and a pointer passed through opaque_uniform() in each row makes
// them be loaded again there instead of being held in scalar registers over the passes.
typedef const __attribute__((address_space(4))) CollideConsts KC4;
typedef const __attribute__((address_space(4))) Tables TB4;

// A lane's node for the pulls: its coordinates, whether it is the first (lo) or last
// (hi) x of its segment, and the first x ghost cell of its segment (XG + 2 s NY NZ).
struct LaneSrc {
  int x, y, z;
  bool lo, hi;
  uint32_t xq;
};
__device__ __forceinline__ LaneSrc lane_src(const Geom &g, int64_t n) {
  LaneSrc l;
  l.x = (int)(n % g.nx);
  l.y = (int)((n / g.nx) % g.ny);
  l.z = (int)(n / ((int64_t)g.nx * g.ny));
  const XSeg sg = x_segment(g, l.x);
  l.lo = l.x == sg.x0;
  l.hi = l.x == sg.x1;
  l.xq = (uint32_t)(g.XG + 2LL * sg.s * g.NY * g.NZ);
  return l;
}

// source row of the directions (*, cy, cz), y - cy and z - cz wrapped on periodic axes
// (an open axis has a ghost layer and never wraps): the padded row and the index of
// its cell x (32-bit products: a padded plane has fewer than 2^31 cells)
struct RowPos {
  uint32_t row, p0;
};
__device__ __forceinline__ RowPos row_source(const Geom &g, const LaneSrc &l, int cy, int cz) {
  int sy = l.y - cy, sz = l.z - cz;
  if (g.per[1] && cy != 0) sy += (l.y == (cy > 0 ? 0 : g.ny - 1)) ? cy * g.ny : 0;
  if (g.per[2] && cz != 0) sz += (l.z == (cz > 0 ? 0 : g.nz - 1)) ? cz * g.nz : 0;
  RowPos r;
  r.row = (uint32_t)(sz + g.pz) * (uint32_t)g.NY + (uint32_t)(sy + g.py);
  r.p0 = r.row * (uint32_t)g.NX + (uint32_t)l.x;
  return r;
}
// index of the source of direction (CX, cy, cz) in its row: x - CX, wrapped on a
// periodic x axis, or the x ghost cell of the segment's end on an open one
template <int CX>
__device__ __forceinline__ uint32_t dir_source(const Geom &g, const LaneSrc &l, const RowPos &r) {
  uint32_t p = r.p0 - (uint32_t)CX;
  if constexpr (CX != 0) {
    const bool edge = CX > 0 ? l.lo : l.hi;
    if (g.per[0]) p += edge ? (uint32_t)(CX * g.nx) : 0u;
    if (g.xg) p = edge ? l.xq + (CX > 0 ? 0u : (uint32_t)(g.NY * g.NZ)) + r.row : p;
  }
  return p;
}

// f and g pulled along one direction, with the deferred corrections at the source.  The
// corrections live in padded planes whose ghost cells hold zero, so a ghost source adds
// nothing.  The loads carry no branch, so that they are all in flight together: X is
// read from the plane of the direction's axis (any plane off the axis directions, where
// it is multiplied by zero), and the y and z components of Cg are read in every row.
template <typename ST>
struct PulledFG {
  ST f, g;
  typename Fmt<ST>::Side x, c[3];
};

template <int M, typename ST, int CX>
__device__ __forceinline__ void pull_fg(const Geom &g, const void *src, const void *corr, int i, int cy, int cz,
                                        uint32_t ps, PulledFG<ST> &p) {
  using Side = typename Fmt<ST>::Side;
  const uint32_t po = ps * (uint32_t)sizeof(ST), co = ps * (uint32_t)sizeof(Side);
  p.f = bld<ST>(plane<ST>(src, g, (M - 1) * Q + i), po);
  p.g = bld<ST>(plane<ST>(src, g, M * Q + i), po);
  const int xa = __builtin_amdgcn_readfirstlane(CX != 0 ? 0 : (cy != 0 ? 1 : 2));
  p.x = bld<Side>(plane<Side>(corr, g, xa), co);
  if constexpr (CX != 0)
    p.c[0] = bld<Side>(plane<Side>(corr, g, 3), co);
  else
    p.c[0] = Side(0);
  p.c[1] = bld<Side>(plane<Side>(corr, g, 4), co);
  p.c[2] = bld<Side>(plane<Side>(corr, g, 5), co);
}

// values of f and g along (CX, cy, cz) with their deferred corrections: 1/2 c.X on the
// axis directions (eq. Ai) and the Fourier-correction flux 3 w_i c_i.Cg (eq.
// corrFourier), each rounded to the side precision and added in FP64, the same way in
// every kernel that pulls
template <int M, typename ST, int CX, typename K>
__device__ __forceinline__ void fg_values(const PulledFG<ST> &p, int i, int cy, int cz, const K &kc, double &f,
                                          double &gv) {
  using Side = typename Fmt<ST>::Side;
  const double xs = (CX * CX + cy * cy + cz * cz) == 1 ? 0.5 * double(CX + cy + cz) : 0.0;
  f = pop_val(p.f, M - 1, i, kc) + double(Side(xs * double(p.x)));
  const double w3 = 3.0 * (w1(CX) * w1(cy) * w1(cz));
  const double d = double(CX) * double(p.c[0]) + double(cy) * double(p.c[1]) + double(cz) * double(p.c[2]);
  gv = pop_val(p.g, M, i, kc) + double(Side(w3 * d));
}

template <int M, typename ST>
struct PulledAll {
  PulledFG<ST> fg;
  ST fa[M - 1];
};

template <int M, typename ST, int CX>
__device__ __forceinline__ void pull_all(const Geom &g, const void *src, const void *corr, int i, int cy, int cz,
                                         uint32_t ps, PulledAll<M, ST> &p) {
  pull_fg<M, ST, CX>(g, src, corr, i, cy, cz, ps, p.fg);
  const uint32_t po = ps * (uint32_t)sizeof(ST);
#pragma unroll
  for (int a = 0; a < M - 1; ++a) p.fa[a] = bld<ST>(plane<ST>(src, g, a * Q + i), po);
}

// Row partial sums of one pulled quantity v over cx: P0 = sum v, P1 = sum cx v,
// P2 = sum cx^2 v, built from the three directions in the order cx = -1, 0, 1.
struct RowSum {
  double m, z;   // v at cx = -1 and cx = 0
};

template <int M>
struct RowMoments {
  RowSum f, g, a[M - 1];
};

template <int M, typename ST, int CX, typename K>
__device__ __forceinline__ void row_moments_dir(const PulledAll<M, ST> &p, int i, int cy, int cz, const K &kc,
                                                RowMoments<M> &rm, double (&mo)[14], double (&sp)[M - 1][4]) {
  double f, gv;
  fg_values<M, ST, CX>(p.fg, i, cy, cz, kc, f, gv);
  double fa[M - 1];
#pragma unroll
  for (int a = 0; a < M - 1; ++a) fa[a] = pop_val(p.fa[a], a, i, kc);
  if constexpr (CX == -1) {
    rm.f.m = f;
    rm.g.m = gv;
#pragma unroll
    for (int a = 0; a < M - 1; ++a) rm.a[a].m = fa[a];
  } else if constexpr (CX == 0) {
    rm.f.z = f;
    rm.g.z = gv;
#pragma unroll
    for (int a = 0; a < M - 1; ++a) rm.a[a].z = fa[a];
  } else {
    // the row is complete: add it to the moments (eqs. Pa, sumfDotc, g0momTotalEnergy)
    const double dy = cy, dz = cz;
    const double f2 = rm.f.m + f, f1 = f - rm.f.m, f0 = f2 + rm.f.z;
    mo[0] += f0;
    mo[1] += f1;
    mo[2] += dy * f0;
    mo[3] += dz * f0;
    mo[4] += f2;
    mo[5] += (dy * dy) * f0;
    mo[6] += (dz * dz) * f0;
    mo[7] += dy * f1;
    mo[8] += dz * f1;
    mo[9] += (dy * dz) * f0;
    const double g1 = gv - rm.g.m, g0 = (rm.g.m + gv) + rm.g.z;
    mo[10] += g0;
    mo[11] += g1;
    mo[12] += dy * g0;
    mo[13] += dz * g0;
#pragma unroll
    for (int a = 0; a < M - 1; ++a) {
      const double s1 = fa[a] - rm.a[a].m, s0 = (rm.a[a].m + fa[a]) + rm.a[a].z;
      sp[a][0] += s0;
      sp[a][1] += s1;
      sp[a][2] += dy * s0;
      sp[a][3] += dz * s0;
    }
  }
}

// O1: moments of all sets over the 27 directions; the loads of the next direction are in
// flight while the current one is summed
template <int M, typename ST>
__device__ __forceinline__ void moments_pass(const Geom &g, const void *src, const void *corr, const LaneSrc &l,
                                             KC4 *kp, double (&mo)[14], double (&sp)[M - 1][4]) {
#pragma unroll
  for (int k = 0; k < 14; ++k) mo[k] = 0.0;
#pragma unroll
  for (int a = 0; a < M - 1; ++a)
#pragma unroll
    for (int k = 0; k < 4; ++k) sp[a][k] = 0.0;
  PulledAll<M, ST> pa, pb, pc;
  RowMoments<M> rm;
  pull_all<M, ST, -1>(g, src, corr, 0, -1, -1, dir_source<-1>(g, l, row_source(g, l, -1, -1)), pa);
#pragma unroll 1
  for (int r = 0; r < 9; ++r) {
    const int cy = __builtin_amdgcn_readfirstlane(r % 3 - 1), cz = __builtin_amdgcn_readfirstlane(r / 3 - 1);
    KC4 *k = kp;
    opaque_uniform(k);
    const RowPos s0 = row_source(g, l, cy, cz);
    pull_all<M, ST, 0>(g, src, corr, 3 * r + 1, cy, cz, dir_source<0>(g, l, s0), pb);
    row_moments_dir<M, ST, -1>(pa, 3 * r, cy, cz, *k, rm, mo, sp);
    pull_all<M, ST, 1>(g, src, corr, 3 * r + 2, cy, cz, dir_source<1>(g, l, s0), pc);
    row_moments_dir<M, ST, 0>(pb, 3 * r + 1, cy, cz, *k, rm, mo, sp);
    {
      const int rn = r < 8 ? r + 1 : 8;
      const int ny = __builtin_amdgcn_readfirstlane(rn % 3 - 1), nz = __builtin_amdgcn_readfirstlane(rn / 3 - 1);
      pull_all<M, ST, -1>(g, src, corr, 3 * rn, ny, nz, dir_source<-1>(g, l, row_source(g, l, ny, nz)), pa);
    }
    row_moments_dir<M, ST, 1>(pc, 3 * r + 2, cy, cz, *k, rm, mo, sp);
  }
}

// Moments of the pulled state (O1) and everything of the collision that is local to the
// node: temperature (O2), production rates (O3), Stefan-Maxwell solve (O4), the
// collision coefficients cc, and the side channel of the stencils (O5).  No global
// store happens before the side channel at the end, so that the constant tables are
// read with scalar loads throughout.
template <int M, typename ST, bool VT>
__device__ __forceinline__ void node_local_post(const Geom &g, const Buffers &b, const IslStash &sh, int64_t n,
                                                const double (&mo)[14], const double (&sp)[M - 1][4],
                                                CollCoef<M, FT<ST>> &cc);

template <int M, typename ST, bool VT>
__device__ __forceinline__ void node_local(const Geom &g, const Buffers &b, KC4 *kp, const IslStash &sh,
                                           int64_t n, const LaneSrc &l, int cur, CollCoef<M, FT<ST>> &cc) {
  // O1: moments of the pulled populations
  double mo[14], sp[M - 1][4];
  moments_pass<M, ST>(g, b.pop[cur], b.corr, l, kp, mo, sp);
  node_local_post<M, ST, VT>(g, b, sh, n, mo, sp, cc);
}

// Everything of the step that is local to the node, from its moments: temperature (O2),
// production rates (O3), Stefan-Maxwell solve (O4), the collision coefficients cc and
// the side channel of the stencils (O5).
template <int M, typename ST, bool VT>
__device__ __forceinline__ void node_local_post(const Geom &g, const Buffers &b, const IslStash &sh, int64_t n,
                                                const double (&mo)[14], const double (&sp)[M - 1][4],
                                                CollCoef<M, FT<ST>> &cc) {
  using SW = IslWords<M>;
  using F = FT<ST>;
  using Side = typename Fmt<ST>::Side;
  // the constant tables through the constant address space: their loads are scalar
  // wherever they stand, also after stores and opaque() barriers
  TB4 &tb = *(TB4 *)b.tab;
  const int64_t N = g.N;
  const double T0 = b.T[n];

  Macro<M> m;
  {
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
    double om_d, om1;
    relax_rates<VT>(tb, T, om_d, om1);
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
    const double inv_zeta = inv_diff_scale(tb, T) / zeta;   // with the T factor of 1/D_ab
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
  double om_n, om1;
  relax_rates<VT>(tb, T, om_n, om1);
  const bool open_any = tb.open_any != 0;
  {
    const double inv_zeta = inv_diff_scale(tb, T) / zeta;   // with the T factor of 1/D_ab (F term)
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

// O7 + O8 for f and g of one direction (eqs. f, g) from the factors of its row:
// f^eq = (rho Psi_y Psi_z) Psi_x, and g' = (1 - omega) g + w_i [A0 + A1.c + A2 : cc]
// with the (cy, cz) part of the bracket summed once per row.  A_i.X and the q^corr part
// are added by the next pull.
struct RowFG {
  double om;       // relaxation rate of f and g at the node (temperature law only)
  double rf;       // rho Psi_cy(u_y) Psi_cz(u_z)
  double R0, R1;   // bracket = R0 + cx R1 + cx^2 A2_xx
  double wyz;      // w1(cy) w1(cz)
};

template <int M, typename F, bool VT>
__device__ __forceinline__ RowFG fg_row(const CollCoef<M, F> &cc, int cy, int cz, KC4 *kp) {
  RowFG rw;
  // the node's rate: the constant, or with a temperature law formed again in each row
  // rather than held over the pass (the expression of relax_rates, so the same value)
  const KC4 &kc = *kp;
  if constexpr (VT)
    rw.om = kc.vexp == 0.0 ? kc.omega : 1.0 / (0.5 + kc.c_om * exp(kc.vexp * (log(cc.T) - kc.ln_vTref)));
  const double u1 = cc.u1, u2 = cc.u2;
  rw.rf = cc.rho * psi_c<double>(cy, u1, u1 * u1 + cc.zeta) * psi_c<double>(cz, u2, u2 * u2 + cc.zeta);
  const double dy = cy, dz = cz;
  rw.R0 = cc.gA0 + dy * cc.gA1[1] + dz * cc.gA1[2] + (dy * dy) * cc.gA2[1] + (dz * dz) * cc.gA2[2] +
          (dy * dz) * cc.gA2[5];
  rw.R1 = cc.gA1[0] + dy * cc.gA2[3] + dz * cc.gA2[4];
  rw.wyz = w1(cy) * w1(cz);
  return rw;
}

template <int M, typename ST, typename F, int CX, bool VT, typename K>
__device__ __forceinline__ void collide_fg_core(const Geom &g, void *dst, const CollCoef<M, F> &cc, const RowFG &rw,
                                                double f, double gv, int i, const K &kc, uint32_t so);

template <int M, typename ST, typename F, int CX, bool VT, typename K>
__device__ __forceinline__ void collide_fg_dir(const Geom &g, void *dst, const CollCoef<M, F> &cc, const RowFG &rw,
                                               const PulledFG<ST> &p, int i, int cy, int cz, const K &kc,
                                               uint32_t so) {
  double f, gv;
  fg_values<M, ST, CX>(p, i, cy, cz, kc, f, gv);
  collide_fg_core<M, ST, F, CX, VT>(g, dst, cc, rw, f, gv, i, kc, so);
}

// f and g of one direction from their pulled values (with the deferred corrections)
template <int M, typename ST, typename F, int CX, bool VT, typename K>
__device__ __forceinline__ void collide_fg_core(const Geom &g, void *dst, const CollCoef<M, F> &cc, const RowFG &rw,
                                                double f, double gv, int i, const K &kc, uint32_t so) {
  const double om = VT ? rw.om : kc.omega;
  const double u0 = cc.u0;
  const double feq = rw.rf * psi_c<double>(CX, u0, u0 * u0 + cc.zeta);
  bst<ST>(plane<ST>(dst, g, (M - 1) * Q + i), so, pop_enc<ST>((1.0 - om) * f + om * feq, M - 1, i, kc));
  const double acc = CX == 0 ? rw.R0 : rw.R0 + double(CX) * rw.R1 + cc.gA2[0];
  bst<ST>(plane<ST>(dst, g, M * Q + i), so, pop_enc<ST>((1.0 - om) * gv + (w1(CX) * rw.wyz) * acc, M, i, kc));
}

// O7 + O8 for the stored species a < M-1 (eq. finalNumericalEquations with F_ai of eq.
// fStar).  Phi_b(u) - Phi_b(u + du_b) is telescoped over the three axis factors, each
// factor difference in closed form so that the difference keeps its relative precision:
// Psi_c(xi) - Psi_c(xi + d) = d (s_c d + s_c 2 xi + t_c), with s_0 = 1, t_0 = 0 and
// s_c = -1/2, t_c = -c/2 for c = +-1 (eq. phis).  With e = Psi_c(u_alpha, zeta_b) =
// A_c(u_alpha) + B_c zeta_b per axis, d the factor differences and r = e - d,
//   Phi_b(u) - Phi_b(u + du_b) = d_x (e_y e_z) + r_x (d_y e_z + r_y d_z),
// whose two brackets depend on (cy, cz) only.  The inter-species term is evaluated in
// F; the equilibria that carry the species mass in FP64.
// The FP64 (y, z) factor of the species equilibria is kept per row when F is FP32;
// with an FP64 F term it is formed per direction from the row's axis factors, which
// holds fewer registers.
template <typename F>
constexpr bool kRowEquilibrium = sizeof(F) == 4;

template <int M, typename F>
struct RowSpecies {
  F Y1[M], Y2[M];       // rho_b zeta_b e_y e_z and rho_b zeta_b (d_y e_z + r_y d_z)
  double pyz[kRowEquilibrium<F> ? M - 1 : 1];   // c_a (A_y + B_y zeta_a)(A_z + B_z zeta_a)
  double Ay, Az, ByT, BzT;                        // axis factors, without kRowEquilibrium
};

template <typename F, typename K>
__device__ __forceinline__ F gas_const(const K &kc, int b) {
  if constexpr (sizeof(F) == 4) return kc.Raf[b]; else return F(kc.Ra[b]);
}
template <int M, typename F, typename K>
__device__ __forceinline__ F inv_diff(const K &kc, int a, int b) {
  const int lo = a < b ? a : b, hi = a < b ? b : a;
  const int k = lo * M - lo * (lo + 1) / 2 + (hi - lo - 1);
  if constexpr (sizeof(F) == 4) return kc.invDpf[k]; else return F(kc.invDp[k]);
}

template <int M, typename F, typename K>
__device__ __forceinline__ void species_row(const CollCoef<M, F> &cc, double T, int cy, int cz, const K &kc,
                                            RowSpecies<M, F> &rs) {
  const double u1 = cc.u1, u2 = cc.u2;
  // B_c is -1 or 1/2, so (B_c T) R_b equals B_c (R_b T) exactly
  const double Ay = psi_c<double>(cy, u1, u1 * u1), Az = psi_c<double>(cz, u2, u2 * u2);
  const double ByT = (cy == 0 ? -1.0 : 0.5) * T, BzT = (cz == 0 ? -1.0 : 0.5) * T;
  const F Ayf = F(Ay), Azf = F(Az), ByTf = F(ByT), BzTf = F(BzT);
  const F sy = cy == 0 ? F(1) : F(-0.5), sz = cz == 0 ? F(1) : F(-0.5);
  const F ky = sy * (F(2) * F(u1)) + F(-0.5) * F(cy), kz = sz * (F(2) * F(u2)) + F(-0.5) * F(cz);
#pragma unroll
  for (int b = 0; b < M; ++b) {
    const F Rb = gas_const<F>(kc, b);
    const F ey = Ayf + ByTf * Rb, ez = Azf + BzTf * Rb;
    const F d1 = cc.dv[b][1], d2 = cc.dv[b][2];
    const F dy = d1 * (sy * d1 + ky), dz = d2 * (sz * d2 + kz);
    const F ry = ey - dy;
    rs.Y1[b] = cc.tbw[b] * (ey * ez);
    rs.Y2[b] = cc.tbw[b] * (dy * ez + ry * dz);
  }
  if constexpr (kRowEquilibrium<F>) {
#pragma unroll
    for (int a = 0; a < M - 1; ++a) {
      const double Ra = kc.Ra[a];
      rs.pyz[a] = cc.ca[a] * ((Ay + ByT * Ra) * (Az + BzT * Ra));
    }
  } else {
    rs.Ay = Ay;
    rs.Az = Az;
    rs.ByT = ByT;
    rs.BzT = BzT;
  }
}

template <int M, typename ST, typename F, int CX, typename K>
__device__ __forceinline__ void collide_species_dir(const Geom &g, void *dst, const CollCoef<M, F> &cc,
                                                    double u0, double T, const RowSpecies<M, F> &rs,
                                                    const ST (&fa)[M - 1], int i, const K &kc, uint32_t so) {
  const double Ax = psi_c<double>(CX, u0, u0 * u0);
  const double BxT = (CX == 0 ? -1.0 : 0.5) * T;
  const F Axf = F(Ax), BxTf = F(BxT);
  constexpr F sx = CX == 0 ? F(1) : F(-0.5);
  const F kx = sx * (F(2) * F(u0)) + F(-0.5 * CX);
  // F_a = sum_b (1/D_ab) dd_b, accumulated over b in increasing order
  F Fa[M - 1];
#pragma unroll
  for (int a = 0; a < M - 1; ++a) Fa[a] = F(0);
#pragma unroll
  for (int b = 0; b < M; ++b) {
    const F ex = Axf + BxTf * gas_const<F>(kc, b);
    const F d0 = cc.dv[b][0];
    const F dx = d0 * (sx * d0 + kx);
    const F rx = ex - dx;
    const F dd = dx * rs.Y1[b] + rx * rs.Y2[b];
#pragma unroll
    for (int a = 0; a < M - 1; ++a)
      if (a != b) Fa[a] += inv_diff<M, F>(kc, a, b) * dd;
  }
#pragma unroll
  for (int a = 0; a < M - 1; ++a) {
    const double Ra = kc.Ra[a];
    const double ex = Ax + BxT * Ra;
    double eq;
    if constexpr (kRowEquilibrium<F>)
      eq = rs.pyz[a] * ex;
    else
      eq = cc.ca[a] * (((rs.Ay + rs.ByT * Ra) * (rs.Az + rs.BzT * Ra)) * ex);
    const double v = double(cc.omb[a]) * pop_val(fa[a], a, i, kc) + eq + double(cc.rcoef[a] * Fa[a]);
    bst<ST>(plane<ST>(dst, g, a * Q + i), so, pop_enc<ST>(v, a, i, kc));
  }
}

// O7 + O8 for f and g alone over the 27 directions (the two-pass form of the
// collision, for formats whose one-pass form holds too many registers)
template <int M, typename ST, typename F, bool VT>
__device__ __forceinline__ void fg_pass(const Geom &g, const void *src, void *dst, const void *corr, KC4 *kp,
                                        const CollCoef<M, F> &cc, const LaneSrc &l) {
  const uint32_t so = row_source(g, l, 0, 0).p0 * (uint32_t)sizeof(ST);
  PulledFG<ST> pa, pb, pc;
  pull_fg<M, ST, -1>(g, src, corr, 0, -1, -1, dir_source<-1>(g, l, row_source(g, l, -1, -1)), pa);
#pragma unroll 1
  for (int r = 0; r < 9; ++r) {
    const int cy = __builtin_amdgcn_readfirstlane(r % 3 - 1), cz = __builtin_amdgcn_readfirstlane(r / 3 - 1);
    KC4 *k = kp;
    opaque_uniform(k);
    const RowPos s0 = row_source(g, l, cy, cz);
    const RowFG rw = fg_row<M, F, VT>(cc, cy, cz, k);
    pull_fg<M, ST, 0>(g, src, corr, 3 * r + 1, cy, cz, dir_source<0>(g, l, s0), pb);
    collide_fg_dir<M, ST, F, -1, VT>(g, dst, cc, rw, pa, 3 * r, cy, cz, *k, so);
    pull_fg<M, ST, 1>(g, src, corr, 3 * r + 2, cy, cz, dir_source<1>(g, l, s0), pc);
    collide_fg_dir<M, ST, F, 0, VT>(g, dst, cc, rw, pb, 3 * r + 1, cy, cz, *k, so);
    {
      const int rn = r < 8 ? r + 1 : 8;
      const int ny = __builtin_amdgcn_readfirstlane(rn % 3 - 1), nz = __builtin_amdgcn_readfirstlane(rn / 3 - 1);
      pull_fg<M, ST, -1>(g, src, corr, 3 * rn, ny, nz, dir_source<-1>(g, l, row_source(g, l, ny, nz)), pa);
    }
    collide_fg_dir<M, ST, F, 1, VT>(g, dst, cc, rw, pc, 3 * r + 2, cy, cz, *k, so);
  }
}

template <int M, typename ST>
__device__ __forceinline__ void pull_species(const Geom &g, const void *src, int i, uint32_t ps, ST (&fa)[M - 1]) {
  const uint32_t po = ps * (uint32_t)sizeof(ST);
#pragma unroll
  for (int a = 0; a < M - 1; ++a) fa[a] = bld<ST>(plane<ST>(src, g, a * Q + i), po);
}

// O7 + O8 for the stored species alone, pipelined like fg_pass
template <int M, typename ST, typename F>
__device__ __forceinline__ void species_pass(const Geom &g, const void *src, void *dst, KC4 *kp,
                                             const CollCoef<M, F> &cc, const LaneSrc &l) {
  const uint32_t so = row_source(g, l, 0, 0).p0 * (uint32_t)sizeof(ST);
  ST pa[M - 1], pb[M - 1], pc[M - 1];
  pull_species<M, ST>(g, src, 0, dir_source<-1>(g, l, row_source(g, l, -1, -1)), pa);
#pragma unroll 1
  for (int r = 0; r < 9; ++r) {
    const int cy = __builtin_amdgcn_readfirstlane(r % 3 - 1), cz = __builtin_amdgcn_readfirstlane(r / 3 - 1);
    KC4 *k = kp;
    opaque_uniform(k);
    double u0 = cc.u0, T = cc.T;
    opaque(u0);
    opaque(T);
    const RowPos s0 = row_source(g, l, cy, cz);
    RowSpecies<M, F> rs;
    species_row<M, F>(cc, T, cy, cz, *k, rs);
    pull_species<M, ST>(g, src, 3 * r + 1, dir_source<0>(g, l, s0), pb);
    collide_species_dir<M, ST, F, -1>(g, dst, cc, u0, T, rs, pa, 3 * r, *k, so);
    pull_species<M, ST>(g, src, 3 * r + 2, dir_source<1>(g, l, s0), pc);
    collide_species_dir<M, ST, F, 0>(g, dst, cc, u0, T, rs, pb, 3 * r + 1, *k, so);
    {
      const int rn = r < 8 ? r + 1 : 8;
      const int ny = __builtin_amdgcn_readfirstlane(rn % 3 - 1), nz = __builtin_amdgcn_readfirstlane(rn / 3 - 1);
      pull_species<M, ST>(g, src, 3 * rn, dir_source<-1>(g, l, row_source(g, l, ny, nz)), pa);
    }
    collide_species_dir<M, ST, F, 1>(g, dst, cc, u0, T, rs, pc, 3 * r + 2, *k, so);
  }
}

// O7 + O8 over the 27 directions: f, g and the stored species of one direction from
// the factors of its row, with the loads of the next direction in flight while the
// current one is collided.  The directions go in the reverse order of the moments pass
// (last row first, cx = +1, 0, -1), so that the populations read last by the moments
// pass, the likeliest to be still in cache, are read again first.
#ifndef LBM_COLLIDE_REVERSED
#define LBM_COLLIDE_REVERSED 1
#endif
template <int M, typename ST, typename F, bool VT>
__device__ __forceinline__ void collide_pass(const Geom &g, const void *src, void *dst, const void *corr, KC4 *kp,
                                             const CollCoef<M, F> &cc, const LaneSrc &l) {
  const uint32_t so = row_source(g, l, 0, 0).p0 * (uint32_t)sizeof(ST);
  PulledAll<M, ST> pa, pb, pc;
#if LBM_COLLIDE_REVERSED
  pull_all<M, ST, 1>(g, src, corr, 26, 1, 1, dir_source<1>(g, l, row_source(g, l, 1, 1)), pc);
#pragma unroll 1
  for (int rr = 0; rr < 9; ++rr) {
    const int r = 8 - rr;
    const int cy = __builtin_amdgcn_readfirstlane(r % 3 - 1), cz = __builtin_amdgcn_readfirstlane(r / 3 - 1);
    KC4 *k = kp;
    opaque_uniform(k);
    double u0 = cc.u0, T = cc.T;
    opaque(u0);
    opaque(T);
    const RowPos s0 = row_source(g, l, cy, cz);
    const RowFG rw = fg_row<M, F, VT>(cc, cy, cz, k);
    RowSpecies<M, F> rs;
    species_row<M, F>(cc, T, cy, cz, *k, rs);
    pull_all<M, ST, 0>(g, src, corr, 3 * r + 1, cy, cz, dir_source<0>(g, l, s0), pb);
    collide_fg_dir<M, ST, F, 1, VT>(g, dst, cc, rw, pc.fg, 3 * r + 2, cy, cz, *k, so);
    collide_species_dir<M, ST, F, 1>(g, dst, cc, u0, T, rs, pc.fa, 3 * r + 2, *k, so);
    pull_all<M, ST, -1>(g, src, corr, 3 * r, cy, cz, dir_source<-1>(g, l, s0), pa);
    collide_fg_dir<M, ST, F, 0, VT>(g, dst, cc, rw, pb.fg, 3 * r + 1, cy, cz, *k, so);
    collide_species_dir<M, ST, F, 0>(g, dst, cc, u0, T, rs, pb.fa, 3 * r + 1, *k, so);
    {
      // last direction of the next row (the last row reloads its own: no branch, so
      // that the wait counts stay exact)
      const int rn = r > 0 ? r - 1 : 0;
      const int ny = __builtin_amdgcn_readfirstlane(rn % 3 - 1), nz = __builtin_amdgcn_readfirstlane(rn / 3 - 1);
      pull_all<M, ST, 1>(g, src, corr, 3 * rn + 2, ny, nz, dir_source<1>(g, l, row_source(g, l, ny, nz)), pc);
    }
    collide_fg_dir<M, ST, F, -1, VT>(g, dst, cc, rw, pa.fg, 3 * r, cy, cz, *k, so);
    collide_species_dir<M, ST, F, -1>(g, dst, cc, u0, T, rs, pa.fa, 3 * r, *k, so);
  }
#else
  pull_all<M, ST, -1>(g, src, corr, 0, -1, -1, dir_source<-1>(g, l, row_source(g, l, -1, -1)), pa);
#pragma unroll 1
  for (int r = 0; r < 9; ++r) {
    const int cy = __builtin_amdgcn_readfirstlane(r % 3 - 1), cz = __builtin_amdgcn_readfirstlane(r / 3 - 1);
    KC4 *k = kp;
    opaque_uniform(k);
    double u0 = cc.u0, T = cc.T;
    opaque(u0);
    opaque(T);
    const RowPos s0 = row_source(g, l, cy, cz);
    const RowFG rw = fg_row<M, F, VT>(cc, cy, cz, k);
    RowSpecies<M, F> rs;
    species_row<M, F>(cc, T, cy, cz, *k, rs);
    pull_all<M, ST, 0>(g, src, corr, 3 * r + 1, cy, cz, dir_source<0>(g, l, s0), pb);
    collide_fg_dir<M, ST, F, -1, VT>(g, dst, cc, rw, pa.fg, 3 * r, cy, cz, *k, so);
    collide_species_dir<M, ST, F, -1>(g, dst, cc, u0, T, rs, pa.fa, 3 * r, *k, so);
    pull_all<M, ST, 1>(g, src, corr, 3 * r + 2, cy, cz, dir_source<1>(g, l, s0), pc);
    collide_fg_dir<M, ST, F, 0, VT>(g, dst, cc, rw, pb.fg, 3 * r + 1, cy, cz, *k, so);
    collide_species_dir<M, ST, F, 0>(g, dst, cc, u0, T, rs, pb.fa, 3 * r + 1, *k, so);
    {
      const int rn = r < 8 ? r + 1 : 8;
      const int ny = __builtin_amdgcn_readfirstlane(rn % 3 - 1), nz = __builtin_amdgcn_readfirstlane(rn / 3 - 1);
      pull_all<M, ST, -1>(g, src, corr, 3 * rn, ny, nz, dir_source<-1>(g, l, row_source(g, l, ny, nz)), pa);
    }
    collide_fg_dir<M, ST, F, 1, VT>(g, dst, cc, rw, pc.fg, 3 * r + 2, cy, cz, *k, so);
    collide_species_dir<M, ST, F, 1>(g, dst, cc, u0, T, rs, pc.fa, 3 * r + 2, *k, so);
  }
#endif
}

// Fused step: the node-local part, then the collide pass from the coefficients in
// registers (FP32 storage; the other formats collide f and g, then the species, in
// two passes that each hold fewer registers).  The populations are read twice, and no
// record goes through memory.
// VT: relaxation rates from the temperature law of the transport (a separate build of
// the kernel, so that the constant-rate kernel carries none of it)
#ifndef LBM_STEP_WAVES_PER_SIMD
#define LBM_STEP_WAVES_PER_SIMD 2
#endif
template <int M, typename ST, bool VT>
__global__ __launch_bounds__(ISL_BLOCK, LBM_STEP_WAVES_PER_SIMD) void k_step(Geom g, Buffers b, int cur) {
  using F = FT<ST>;
  __shared__ double words[IslWords<M>::WORDS * ISL_BLOCK];
  const IslStash sh{(lds_double *)&words[threadIdx.x]};
  const int64_t n = xcd_tile() * blockDim.x + threadIdx.x;
  if (n >= g.N) return;
  const LaneSrc l = lane_src(g, n);

  KC4 *kp = (KC4 *)b.kc;
  CollCoef<M, F> cc;
  node_local<M, ST, VT>(g, b, kp, sh, n, l, cur, cc);
  if constexpr (sizeof(ST) == 4 && sizeof(F) == 4) {
    collide_pass<M, ST, F, VT>(g, b.pop[cur], b.pop[cur ^ 1], b.corr, kp, cc, l);
  } else {
    fg_pass<M, ST, F, VT>(g, b.pop[cur], b.pop[cur ^ 1], b.corr, kp, cc, l);
    species_pass<M, ST, F>(g, b.pop[cur], b.pop[cur ^ 1], kp, cc, l);
  }
}

// ---- psi_alpha = (1/omega - 1/2) d_alpha phi_alpha (isotropic gradient) ------------
// One node's sums for psi, term by term in the order of the directions, from the phi
// components of its neighbours (get(I, d): component d of the neighbour along
// direction I).  sg holds the sign of the mirror image of phi_alpha beyond a symmetry
// face (phi_alpha is odd in u_alpha); SYM = false when no face of the lattice is one:
// every sign is then 1, and leaving the factor out changes no bit.
template <bool SYM, typename G>
__device__ __forceinline__ void psi_terms(G &&get, const double (&sg)[3][3], double (&acc)[3]) {
  static_for<27>([&](auto Ic) {
    constexpr int I = decltype(Ic)::value;
    constexpr int cx = cx_of(I), cy = cy_of(I), cz = cz_of(I);
    constexpr double w = 3.0 * wgt(I);
    if constexpr (SYM) {
      if constexpr (cx != 0) acc[0] += (cx * w) * (sg[0][cx + 1] * get(Ic, 0));
      if constexpr (cy != 0) acc[1] += (cy * w) * (sg[1][cy + 1] * get(Ic, 1));
      if constexpr (cz != 0) acc[2] += (cz * w) * (sg[2][cz + 1] * get(Ic, 2));
    } else {
      if constexpr (cx != 0) acc[0] += (cx * w) * get(Ic, 0);
      if constexpr (cy != 0) acc[1] += (cy * w) * get(Ic, 1);
      if constexpr (cz != 0) acc[2] += (cz * w) * get(Ic, 2);
    }
  });
}

template <typename RT, bool SYM>
__global__ __launch_bounds__(256) void k_psi(Geom g, Buffers b) {
  const int64_t n = xcd_tile() * blockDim.x + threadIdx.x;
  if (n >= g.N) return;
  const int x = (int)(n % g.nx), y = (int)((n / g.nx) % g.ny), z = (int)(n / ((int64_t)g.nx * g.ny));
  const RT *phi = static_cast<const RT *>(b.side_phi);
  const int64_t N = g.N;
  double om, om1;
  relax_rates(*b.tab, b.T[n], om, om1);
  const double coef = 1.0 / om - 0.5;
  // x neighbours within the node's segment (the whole axis when it is periodic)
  const XSeg xsg = x_segment(g, x);
  int xs[3], ys[3], zs[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    xs[k] = g.per[0] ? nb_coord(x, k - 1, g.nx, true) : min(max(x + k - 1, xsg.x0), xsg.x1);
    ys[k] = nb_coord(y, k - 1, g.ny, g.per[1]);
    zs[k] = nb_coord(z, k - 1, g.nz, g.per[2]);
  }
  double sg[3][3];
  if constexpr (SYM) {
    const int xyz[3] = {x, y, z}, lo3[3] = {xsg.x0, 0, 0}, hi3[3] = {xsg.x1, g.ny - 1, g.nz - 1};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      sg[a][0] = (xyz[a] == lo3[a] && g.bc[2 * a] == LBM_BC_SYMMETRY) ? -1.0 : 1.0;
      sg[a][1] = 1.0;
      sg[a][2] = (xyz[a] == hi3[a] && g.bc[2 * a + 1] == LBM_BC_SYMMETRY) ? -1.0 : 1.0;
    }
  }
  double acc[3] = {0, 0, 0};
  psi_terms<SYM>([&](auto Ic, int d) {
    constexpr int I = decltype(Ic)::value;
    const int64_t nn = ((int64_t)zs[cz_of(I) + 1] * g.ny + ys[cy_of(I) + 1]) * g.nx + xs[cx_of(I) + 1];
    return double(phi[d * N + nn]);
  }, sg, acc);
  RT *psi = static_cast<RT *>(b.psi);
#pragma unroll
  for (int d = 0; d < 3; ++d) psi[d * N + n] = RT(coef * acc[d]);
}

// ---- X_alpha = -d_alpha psi_alpha; Cg = sum_a w_a grad Y_a ---------------------------
// One workgroup per tile of X x Y x Z nodes (32 x 4 x 4 measured fastest of
// 16x4x4, 32x4x2, 32x4x4 and 64x2x2).  psi (3 fields) and Y_a (M fields)
// of the tile and its one-cell halo are staged in LDS with loads along x, and each node
// then sums its 26 neighbours from LDS.  A halo cell holds the neighbour the gradient
// stencil takes: wrapped on periodic axes, clamped on open ones (zero gradient).
// A lattice one node thick in y and z (quasi-1D flames and their batches) takes a tile
// of 256 x 1 x 1 with no y or z halo: its y and z neighbours are the node's own row
// (wrapped on periodic axes, clamped on open ones), so 32 x 4 x 4 tiles would leave 15
// of 16 threads idle.  A lattice one node thick in z alone (2D flames) can take a tile
// of 32 x 8 x 1 with no z halo, for the same reason.
template <int TX, int TY, int TZ, bool TH>
struct CorrTileT {
  static constexpr bool THIN = TH, FLAT = !TH && TZ == 1;
  static constexpr int X = TX, Y = TY, Z = TZ, HX = X + 2, HY = TH ? 1 : Y + 2, HZ = (TH || FLAT) ? 1 : Z + 2;
  static constexpr int THREADS = X * Y * Z, CELLS = HX * HY * HZ;
};
// the tile shapes a lattice chooses from (corr_tile_candidates): 0-2 for lattices with a
// cross-section, 3-5 for lattices one node thick in y and z
template <int K>
struct CorrTile;
template <> struct CorrTile<0> : CorrTileT<32, 4, 4, false> {};
template <> struct CorrTile<1> : CorrTileT<64, 2, 2, false> {};
template <> struct CorrTile<2> : CorrTileT<16, 4, 8, false> {};
template <> struct CorrTile<3> : CorrTileT<256, 1, 1, true> {};
template <> struct CorrTile<4> : CorrTileT<128, 1, 1, true> {};
template <> struct CorrTile<5> : CorrTileT<512, 1, 1, true> {};
template <> struct CorrTile<9> : CorrTileT<32, 8, 1, false> {};

__device__ __forceinline__ int halo_coord(int v, int n, bool periodic) {
  if (periodic) {
    v %= n;
    return v < 0 ? v + n : v;
  }
  return v < 0 ? 0 : (v >= n ? n - 1 : v);
}

template <int K>
inline int64_t corr_tiles(const Geom &g) {
  using T = CorrTile<K>;
  return (int64_t)((g.nx + T::X - 1) / T::X) * ((g.ny + T::Y - 1) / T::Y) * ((g.nz + T::Z - 1) / T::Z);
}

template <int M, typename RT, typename CT, int K>
__global__ __launch_bounds__(CorrTile<K>::THREADS) void k_corr(Geom g, Buffers b) {
  using T = CorrTile<K>;
  constexpr bool THIN = T::THIN, FLAT = T::FLAT;
  constexpr int CH_X = T::HX, CH_Y = T::HY, CH_CELLS = T::CELLS;
  __shared__ RT sh[(M + 3) * CH_CELLS];   // field f of halo cell c at f * CH_CELLS + c
  const int tiles_x = (g.nx + T::X - 1) / T::X, tiles_y = (g.ny + T::Y - 1) / T::Y;
  const int64_t t = xcd_tile();
  const int x0 = (int)(t % tiles_x) * T::X, y0 = (int)((t / tiles_x) % tiles_y) * T::Y,
            z0 = (int)(t / ((int64_t)tiles_x * tiles_y)) * T::Z;
  const RT *psi = static_cast<const RT *>(b.psi);
  const RT *Yf = static_cast<const RT *>(b.side_Y);
  const RT *wf = static_cast<const RT *>(b.side_w);
  const int64_t N = g.N;
  for (int c = threadIdx.x; c < CH_CELLS; c += T::THREADS) {
    const int hx = c % CH_X, hy = (c / CH_X) % CH_Y, hz = c / (CH_X * CH_Y);
    const int gx = halo_coord(x0 + hx - 1, g.nx, g.per[0]);
    const int gy = THIN ? 0 : halo_coord(y0 + hy - 1, g.ny, g.per[1]);
    const int gz = (THIN || FLAT) ? 0 : halo_coord(z0 + hz - 1, g.nz, g.per[2]);
    const int64_t nn = ((int64_t)gz * g.ny + gy) * g.nx + gx;
#pragma unroll
    for (int f = 0; f < 3; ++f) sh[f * CH_CELLS + c] = psi[f * N + nn];
#pragma unroll
    for (int a = 0; a < M; ++a) sh[(3 + a) * CH_CELLS + c] = Yf[a * N + nn];
  }
  __syncthreads();
  const int lx = threadIdx.x % T::X, ly = (threadIdx.x / T::X) % T::Y, lz = threadIdx.x / (T::X * T::Y);
  const int x = x0 + lx, y = y0 + ly, z = z0 + lz;
  if (x >= g.nx || y >= g.ny || z >= g.nz) return;
  const int64_t n = ((int64_t)z * g.ny + y) * g.nx + x;
  const int c0 = THIN ? lx + 1 : ((FLAT ? 0 : (lz + 1) * CH_Y) + (ly + 1)) * CH_X + (lx + 1);
  // x neighbours stay within the node's segment: at its ends the stencil takes the node
  // itself (the halo cell beyond the lattice's ends holds the same value)
  const XSeg xsg = x_segment(g, x);
  const int dxm = (!g.per[0] && x == xsg.x0) ? 0 : -1, dxp = (!g.per[0] && x == xsg.x1) ? 0 : 1;
  // side fields in RT, sums in FP64
  double wa[M];
#pragma unroll
  for (int a = 0; a < M; ++a) wa[a] = double(wf[a * N + n]);
  double X[3] = {0, 0, 0}, C[3] = {0, 0, 0};
  static_for<27>([&](auto Ic) {
    constexpr int I = decltype(Ic)::value;
    constexpr int cx = cx_of(I), cy = cy_of(I), cz = cz_of(I);
    if constexpr (I != 13) {
      const int nc = c0 + (THIN ? 0 : ((FLAT ? 0 : cz * CH_Y) + cy) * CH_X) + (cx < 0 ? dxm : (cx > 0 ? dxp : 0));
      constexpr double w = 3.0 * wgt(I);
      if constexpr (cx != 0) X[0] -= (cx * w) * double(sh[0 * CH_CELLS + nc]);
      if constexpr (cy != 0) X[1] -= (cy * w) * double(sh[1 * CH_CELLS + nc]);
      if constexpr (cz != 0) X[2] -= (cz * w) * double(sh[2 * CH_CELLS + nc]);
      double hy = 0.0;
#pragma unroll
      for (int a = 0; a < M; ++a) hy += wa[a] * double(sh[(3 + a) * CH_CELLS + nc]);
      if constexpr (cx != 0) C[0] += (cx * w) * hy;
      if constexpr (cy != 0) C[1] += (cy * w) * hy;
      if constexpr (cz != 0) C[2] += (cz * w) * hy;
    }
  });
  // padded planes: the ghost cells keep the zero they are cleared to at init
  CT *corr = static_cast<CT *>(b.corr);
  const int64_t NPAD = g.NPAD;
  const int64_t pn = ((int64_t)(z + g.pz) * g.NY + (y + g.py)) * g.NX + x;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    corr[d * NPAD + pn] = CT(X[d]);
    corr[(3 + d) * NPAD + pn] = CT(C[d]);
  }
}

// ---- psi and the corrections in one pass, marching along z ---------------------------
// The values of k_psi followed by k_corr, bit for bit, without psi's round trip through
// HBM and without its launch.  A workgroup takes a column of X x Y nodes over a range of
// ZC planes and walks it along z.  Three planes of phi (X+4 by Y+4 cells: the psi tile
// and its own one-cell halo), of psi and of Y_a (X+2 by Y+2 cells) rotate through LDS.
// At plane z the workgroup stores phi of plane z+2, then stores Y_a of z+1 and forms psi
// of z+1 from phi, then sums X and Cg of plane z from psi and Y_a; the loads of the next
// plane are issued before the sums of the current one, and two barriers a plane order
// the slots' reuse.
// A cell of a tile holds the field at the node the gradient stencil takes (wrapped on
// periodic axes, clamped on open ones), as in k_corr.  psi of a cell is formed at that
// node from the phi tile: on a periodic axis its neighbours are the next cells of the
// tile, on an open axis the clamped neighbours of the node, which the tile also covers.
// In z a psi plane beyond an open face is never formed: the stencil takes the face plane.
template <int TXv, int TYv, int ZCv>
struct MarchTileT {
  static constexpr int X = TXv, Y = TYv, ZC = ZCv, THREADS = X * Y;
  static constexpr int PX = X + 4, PCELLS = PX * (Y + 4);   // phi tile
  static constexpr int SX = X + 2, SCELLS = SX * (Y + 2);   // psi and Y_a tiles
  static constexpr int PPT = (PCELLS + THREADS - 1) / THREADS, SPT = (SCELLS + THREADS - 1) / THREADS;
  static_assert(SCELLS >= THREADS, "every thread holds a cell of each tile");
};
// shape 6 (corr_tile_candidates): chunks of 32 planes (16 measured no faster); narrower
// in y for FP64 fields, whose tiles take twice the LDS
template <int K, typename RT>
struct MarchTile;
template <typename RT> struct MarchTile<6, RT> : MarchTileT<32, sizeof(RT) == 8 ? 4 : 8, 32> {};

template <int K, typename RT>
inline int64_t march_tiles(const Geom &g) {
  using T = MarchTile<K, RT>;
  return (int64_t)((g.nx + T::X - 1) / T::X) * ((g.ny + T::Y - 1) / T::Y) * ((g.nz + T::ZC - 1) / T::ZC);
}

// LDS slot of plane q (q >= -2)
__device__ __forceinline__ int mslot(int q) { return (q + 3) % 3; }

// A psi cell of the tile: the phi-tile columns of its x neighbours, the offsets of the
// rows of its y neighbours, and the signs of the mirror images at symmetry faces (bit 0
// x-, 1 x+, 2 y-, 3 y+); the same for every plane
struct MarchCell {
  int ox[3], oy[3], sym;
};
template <typename T>
__device__ __forceinline__ MarchCell march_cell(const Geom &g, int c, int x0, int y0) {
  const int hx = c % T::SX, hy = c / T::SX;
  const int x = halo_coord(x0 - 1 + hx, g.nx, g.per[0]), y = halo_coord(y0 - 1 + hy, g.ny, g.per[1]);
  const XSeg xsg = x_segment(g, x);
  MarchCell m;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    m.ox[k] = g.per[0] ? hx + k : min(max(x + k - 1, xsg.x0), xsg.x1) - (x0 - 2);
    m.oy[k] = (g.per[1] ? hy + k : nb_coord(y, k - 1, g.ny, false) - (y0 - 2)) * T::PX;
  }
  m.sym = (x == xsg.x0 && g.bc[0] == LBM_BC_SYMMETRY ? 1 : 0) | (x == xsg.x1 && g.bc[1] == LBM_BC_SYMMETRY ? 2 : 0) |
          (y == 0 && g.bc[2] == LBM_BC_SYMMETRY ? 4 : 0) | (y == g.ny - 1 && g.bc[3] == LBM_BC_SYMMETRY ? 8 : 0);
  return m;
}

template <int M, typename RT, typename CT, int K, bool SYM>
__global__ __launch_bounds__((MarchTile<K, RT>::THREADS)) void k_corr_march(Geom g, Buffers b) {
  using T = MarchTile<K, RT>;
  constexpr int NT = T::THREADS, PC = T::PCELLS, SC = T::SCELLS, PPT = T::PPT, SPT = T::SPT;
  __shared__ RT sphi[3][3 * PC];   // plane q in slot mslot(q); component d at d * PC + cell
  __shared__ RT spsi[3][3 * SC];
  __shared__ RT sY[3][M * SC];
  const int tiles_x = (g.nx + T::X - 1) / T::X, tiles_y = (g.ny + T::Y - 1) / T::Y;
  const int64_t t = xcd_tile();
  const int x0 = (int)(t % tiles_x) * T::X, y0 = (int)((t / tiles_x) % tiles_y) * T::Y;
  const int zb = (int)(t / ((int64_t)tiles_x * tiles_y)) * T::ZC, ze = min(zb + T::ZC, g.nz);
  const int tid = threadIdx.x;
  const RT *phi = static_cast<const RT *>(b.side_phi);
  const RT *Yf = static_cast<const RT *>(b.side_Y);
  const RT *wf = static_cast<const RT *>(b.side_w);
  const int64_t N = g.N, NXY = (int64_t)g.nx * g.ny;
  // a cell j > 0 of this thread exists when c(j) is within its tile (cell 0 always does)
  auto has = [&](int j, int cells) { return j == 0 || tid + j * NT < cells; };
  // in-plane index of the node each tile cell of this thread holds
  int pxy[PPT], sxy[SPT];
  MarchCell mc[SPT];
#pragma unroll
  for (int j = 0; j < PPT; ++j) {
    const int c = min(tid + j * NT, PC - 1);
    pxy[j] = halo_coord(y0 - 2 + c / T::PX, g.ny, g.per[1]) * g.nx + halo_coord(x0 - 2 + c % T::PX, g.nx, g.per[0]);
  }
#pragma unroll
  for (int j = 0; j < SPT; ++j) {
    const int c = min(tid + j * NT, SC - 1);
    sxy[j] = halo_coord(y0 - 1 + c / T::SX, g.ny, g.per[1]) * g.nx + halo_coord(x0 - 1 + c % T::SX, g.nx, g.per[0]);
    mc[j] = march_cell<T>(g, c, x0, y0);
  }
  const int lx = tid % T::X, ly = tid / T::X, x = x0 + lx, y = y0 + ly;
  const bool inb = x < g.nx && y < g.ny;
  const int nxy = inb ? y * g.nx + x : 0;
  const int c0 = (ly + 1) * T::SX + (lx + 1);
  const XSeg xsg = x_segment(g, inb ? x : 0);
  const int dxm = (!g.per[0] && x == xsg.x0) ? 0 : -1, dxp = (!g.per[0] && x == xsg.x1) ? 0 : 1;
  const bool vt = g.vt != 0;
  double coef0 = 0.0;
  if (!vt) {
    double om, om1;
    relax_rates(*b.tab, 1.0, om, om1);
    coef0 = 1.0 / om - 0.5;
  }
  // a psi or Y_a plane exists within the lattice, or by wrapping
  auto live = [&](int q) { return g.per[2] || (q >= 0 && q < g.nz); };
  auto plane = [&](int q) { return (int64_t)halo_coord(q, g.nz, g.per[2]) * NXY; };
  auto load_phi = [&](int q, RT (&v)[PPT][3]) {
    const int64_t o = plane(q);
#pragma unroll
    for (int j = 0; j < PPT; ++j)
#pragma unroll
      for (int d = 0; d < 3; ++d) v[j][d] = phi[d * N + o + pxy[j]];
  };
  auto store_phi = [&](int q, const RT (&v)[PPT][3]) {
#pragma unroll
    for (int j = 0; j < PPT; ++j)
      if (has(j, PC)) {
#pragma unroll
        for (int d = 0; d < 3; ++d) sphi[mslot(q)][d * PC + tid + j * NT] = v[j][d];
      }
  };
  auto load_Y = [&](int q, RT (&v)[SPT][M]) {
    const int64_t o = plane(q);
#pragma unroll
    for (int j = 0; j < SPT; ++j)
#pragma unroll
      for (int a = 0; a < M; ++a) v[j][a] = Yf[a * N + o + sxy[j]];
  };
  auto store_Y = [&](int q, const RT (&v)[SPT][M]) {
#pragma unroll
    for (int j = 0; j < SPT; ++j)
      if (has(j, SC)) {
#pragma unroll
        for (int a = 0; a < M; ++a) sY[mslot(q)][a * SC + tid + j * NT] = v[j][a];
      }
  };
  // stored temperature at the psi cells (read only for temperature-dependent rates)
  auto load_T = [&](int q, double (&v)[SPT]) {
    if (!vt) return;
    const int64_t o = plane(q);
#pragma unroll
    for (int j = 0; j < SPT; ++j) v[j] = b.T[o + sxy[j]];
  };
  // psi of plane q at this thread's cells (the arithmetic of k_psi)
  auto form_psi = [&](int q, const double (&tq)[SPT]) {
    if (!live(q)) return;
    int zs[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) zs[k] = mslot(g.per[2] ? q + k - 1 : nb_coord(q, k - 1, g.nz, false));
    const int z = g.per[2] ? halo_coord(q, g.nz, true) : q;
    const bool zlo = z == 0 && g.bc[4] == LBM_BC_SYMMETRY, zhi = z == g.nz - 1 && g.bc[5] == LBM_BC_SYMMETRY;
    RT *ps = spsi[mslot(q)];
#pragma unroll
    for (int j = 0; j < SPT; ++j) {
      if (!has(j, SC)) continue;
      const MarchCell &m = mc[j];
      double coef = coef0;
      if (vt) {
        double om, om1;
        relax_rates(*b.tab, tq[j], om, om1);
        coef = 1.0 / om - 0.5;
      }
      double sg[3][3];
      if constexpr (SYM) {
        sg[0][0] = (m.sym & 1) ? -1.0 : 1.0;
        sg[0][2] = (m.sym & 2) ? -1.0 : 1.0;
        sg[1][0] = (m.sym & 4) ? -1.0 : 1.0;
        sg[1][2] = (m.sym & 8) ? -1.0 : 1.0;
        sg[2][0] = zlo ? -1.0 : 1.0;
        sg[2][2] = zhi ? -1.0 : 1.0;
        sg[0][1] = sg[1][1] = sg[2][1] = 1.0;
      }
      double acc[3] = {0, 0, 0};
      psi_terms<SYM>([&](auto Ic, int d) {
        constexpr int I = decltype(Ic)::value;
        return double(sphi[zs[cz_of(I) + 1]][d * PC + m.oy[cy_of(I) + 1] + m.ox[cx_of(I) + 1]]);
      }, sg, acc);
      const int c = tid + j * NT;
#pragma unroll
      for (int d = 0; d < 3; ++d) ps[d * SC + c] = RT(coef * acc[d]);
    }
  };
  auto load_w = [&](int q, RT (&v)[M]) {
    if (!inb) return;
#pragma unroll
    for (int a = 0; a < M; ++a) v[a] = wf[a * N + (int64_t)q * NXY + nxy];
  };

  RT ph[PPT][3], yv[SPT][M], wv[M];
  double tv[SPT] = {};
  // prologue: phi of planes zb-2 .. zb+1, psi and Y_a of planes zb-1 and zb
  load_phi(zb - 2, ph);
  store_phi(zb - 2, ph);
  load_phi(zb - 1, ph);
  store_phi(zb - 1, ph);
  load_phi(zb, ph);
  store_phi(zb, ph);
  load_Y(zb - 1, yv);
  if (live(zb - 1)) store_Y(zb - 1, yv);
  load_Y(zb, yv);
  store_Y(zb, yv);
  load_T(zb - 1, tv);
  __syncthreads();
  form_psi(zb - 1, tv);
  load_phi(zb + 1, ph);
  load_T(zb, tv);
  __syncthreads();
  store_phi(zb + 1, ph);
  __syncthreads();
  form_psi(zb, tv);
  load_phi(zb + 2, ph);
  load_Y(zb + 1, yv);
  load_T(zb + 1, tv);
  load_w(zb, wv);
  __syncthreads();

  CT *corr = static_cast<CT *>(b.corr);
  const int64_t NPAD = g.NPAD;
  for (int z = zb; z < ze; ++z) {
    store_phi(z + 2, ph);
    __syncthreads();
    if (live(z + 1)) store_Y(z + 1, yv);
    double tq[SPT];
#pragma unroll
    for (int j = 0; j < SPT; ++j) tq[j] = tv[j];
    RT wz[M];
#pragma unroll
    for (int a = 0; a < M; ++a) wz[a] = wv[a];
    if (z + 1 < ze) {   // the next plane's loads, in flight during the sums
      load_phi(z + 3, ph);
      load_Y(z + 2, yv);
      load_T(z + 2, tv);
      load_w(z + 1, wv);
    }
    form_psi(z + 1, tq);
    __syncthreads();
    if (!inb) continue;
    int zs[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) zs[k] = mslot(g.per[2] ? z + k - 1 : nb_coord(z, k - 1, g.nz, false));
    double wa[M];
#pragma unroll
    for (int a = 0; a < M; ++a) wa[a] = double(wz[a]);
    double X[3] = {0, 0, 0}, C[3] = {0, 0, 0};
    static_for<27>([&](auto Ic) {
      constexpr int I = decltype(Ic)::value;
      constexpr int cx = cx_of(I), cy = cy_of(I), cz = cz_of(I);
      if constexpr (I != 13) {
        const int nc = c0 + cy * T::SX + (cx < 0 ? dxm : (cx > 0 ? dxp : 0));
        const RT *ps = spsi[zs[cz + 1]], *yy = sY[zs[cz + 1]];
        constexpr double w = 3.0 * wgt(I);
        if constexpr (cx != 0) X[0] -= (cx * w) * double(ps[0 * SC + nc]);
        if constexpr (cy != 0) X[1] -= (cy * w) * double(ps[1 * SC + nc]);
        if constexpr (cz != 0) X[2] -= (cz * w) * double(ps[2 * SC + nc]);
        double hy = 0.0;
#pragma unroll
        for (int a = 0; a < M; ++a) hy += wa[a] * double(yy[a * SC + nc]);
        if constexpr (cx != 0) C[0] += (cx * w) * hy;
        if constexpr (cy != 0) C[1] += (cy * w) * hy;
        if constexpr (cz != 0) C[2] += (cz * w) * hy;
      }
    });
    const int64_t pn = ((int64_t)(z + g.pz) * g.NY + (y + g.py)) * g.NX + x;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      corr[d * NPAD + pn] = CT(X[d]);
      corr[(3 + d) * NPAD + pn] = CT(C[d]);
    }
  }
}

// ---- equilibria of one state (init and ghosts) --------------------------------------
// The moments of the equilibria of one state (eqs. feq, gieq): the species temperature
// factors, and the Grad coefficients of g^eq.
template <int M>
struct EqState {
  double rho, u[3], su[3], zeta, zeta_a[M], Y[M];
  double A0, qeq[3], Rd[3], Ro[3];   // Rd: 4.5 R_dd - 1.5 rho E; Ro: 9 R_xy, R_xz, R_yz
};

template <int M, typename TB>
__device__ __forceinline__ void eq_state(const TB &tb, double rho, const double *u, double T, const double *Y,
                                         EqState<M> &e) {
  double zeta = 0.0, H = 0.0, U = 0.0;
  const double invT = 1.0 / T;
#pragma unroll
  for (int a = 0; a < M; ++a) {
    e.zeta_a[a] = tb.Ra[a] * T;
    e.Y[a] = Y[a];
    zeta += Y[a] * e.zeta_a[a];
    const double h = h_RT(tb.nasa[a], T, invT);
    H += Y[a] * e.zeta_a[a] * h;
    U += Y[a] * e.zeta_a[a] * (h - 1.0);
  }
  const double usq = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
  const double rhoE = rho * (U + 0.5 * usq);
  const double h2 = H + 0.5 * usq, P = rho * zeta;
  double Req[6];
  const int ia[6] = {0, 1, 2, 0, 0, 1}, ib[6] = {0, 1, 2, 1, 2, 2};
#pragma unroll
  for (int d = 0; d < 3; ++d) e.qeq[d] = h2 * rho * u[d];
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    const double Peq = (k < 3 ? rho * zeta : 0.0) + rho * u[ia[k]] * u[ib[k]];
    Req[k] = h2 * Peq + P * u[ia[k]] * u[ib[k]];
  }
  e.A0 = 2.5 * rhoE - 1.5 * (Req[0] + Req[1] + Req[2]);
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    e.Rd[d] = 4.5 * Req[d] - 1.5 * rhoE;
    e.Ro[d] = Req[3 + d];
  }
  e.rho = rho;
  e.zeta = zeta;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    e.u[d] = u[d];
    e.su[d] = u[d] * u[d];
  }
}

// the equilibria of all sets along direction i = (cx, cy, cz), stored at padded index p
template <int M, typename ST, typename K>
__device__ __forceinline__ void write_eq_dir(const EqState<M> &e, const K &kc, ST *__restrict__ dst, int64_t NPAD,
                                             int i, int cx, int cy, int cz, int64_t p) {
  const double fe = e.rho * psi_c<double>(cx, e.u[0], e.su[0] + e.zeta) *
                    psi_c<double>(cy, e.u[1], e.su[1] + e.zeta) * psi_c<double>(cz, e.u[2], e.su[2] + e.zeta);
  dst[(int64_t)((M - 1) * Q + i) * NPAD + p] = pop_enc<ST>(fe, M - 1, i, kc);
  const double fx = cx, fy = cy, fz = cz;
  double acc = e.A0 + 3.0 * (fx * e.qeq[0] + fy * e.qeq[1] + fz * e.qeq[2]);
  acc += fx * fx * e.Rd[0] + fy * fy * e.Rd[1] + fz * fz * e.Rd[2];
  acc += 9.0 * (fx * fy * e.Ro[0] + fx * fz * e.Ro[1] + fy * fz * e.Ro[2]);
  dst[(int64_t)(M * Q + i) * NPAD + p] = pop_enc<ST>(w1(cx) * w1(cy) * w1(cz) * acc, M, i, kc);
#pragma unroll
  for (int a = 0; a < M - 1; ++a) {
    const double z = e.zeta_a[a];
    const double fa = e.rho * e.Y[a] * psi_c<double>(cx, e.u[0], e.su[0] + z) *
                      psi_c<double>(cy, e.u[1], e.su[1] + z) * psi_c<double>(cz, e.u[2], e.su[2] + z);
    dst[(int64_t)(a * Q + i) * NPAD + p] = pop_enc<ST>(fa, a, i, kc);
  }
}

template <int M, typename ST>
__device__ __forceinline__ void write_equilibria(const Tables &tb, const CollideConsts &kc,
                                                 ST *__restrict__ dst, int64_t NPAD, const int64_t (&pidx)[27],
                                                 double rho, const double *u, double T, const double *Y) {
  EqState<M> e;
  eq_state<M>(tb, rho, u, T, Y, e);
  static_for<27>([&](auto Ic) {
    constexpr int I = decltype(Ic)::value;
    const int64_t p = pidx[I];
    if (p < 0) return;
    write_eq_dir<M, ST>(e, kc, dst, NPAD, I, cx_of(I), cy_of(I), cz_of(I), p);
  });
}

// initial state: equilibria pushed to where the first pull reads them
template <int M, typename ST>
__global__ __launch_bounds__(128) void k_init(Geom g, Buffers b, CollideConsts kc, const double *rho,
                                              const double *u, const double *T, const double *Y, int cur) {
  const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= g.N) return;
  const int x = (int)(n % g.nx), y = (int)((n / g.nx) % g.ny), z = (int)(n / ((int64_t)g.nx * g.ny));
  const AxisSrc ax = axis_src_x(g, x);
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

// Ghost cell t of the slabs beyond the non-periodic faces: the x ghost cells (two per
// segment and padded row, in their order after the rows), then the y slabs (interior
// x, padded z), then the z slabs (interior x, y).  gc holds its coordinates, x relative
// to the first x (x0) of its segment of length len; for the y and z slabs the segment
// is the whole row.  p is its index in a plane.
struct GhostCell {
  int gc[3];
  int x0, len;
  uint32_t p;
};
__device__ __forceinline__ bool ghost_cell(const Geom &g, int64_t t, int64_t nx_slab, int64_t ny_slab,
                                           int64_t nz_slab, GhostCell &c) {
  c.x0 = 0;
  c.len = g.nx;
  if (t < nx_slab) {          // before or after a segment: x ghost cell XG + t
    const int64_t per = (int64_t)g.NY * g.NZ;
    const int q = (int)(t / per);
    const int64_t r = t % per;
    if (g.nseg > 1) {
      c.x0 = g.seg_off[q >> 1];
      c.len = g.seg_off[(q >> 1) + 1] - c.x0;
    }
    c.gc[0] = (q & 1) ? c.len : -1;
    c.gc[1] = (int)(r % g.NY) - g.py;
    c.gc[2] = (int)(r / g.NY) - g.pz;
    c.p = (uint32_t)(g.XG + t);
    return true;
  }
  if ((t -= nx_slab) < ny_slab) {   // y = -1 or ny
    const int64_t per = (int64_t)g.nx * g.NZ;
    c.gc[1] = (t < per) ? -1 : g.ny;
    const int64_t r = t % per;
    c.gc[0] = (int)(r % g.nx);
    c.gc[2] = (int)(r / g.nx) - g.pz;
  } else if ((t -= ny_slab) < nz_slab) {   // z = -1 or nz
    const int64_t per = (int64_t)g.nx * g.ny;
    c.gc[2] = (t < per) ? -1 : g.nz;
    const int64_t r = t % per;
    c.gc[0] = (int)(r % g.nx);
    c.gc[1] = (int)(r / g.nx);
  } else {
    return false;
  }
  c.p = cell_index(g, c.gc[0], (uint32_t)(c.gc[2] + g.pz) * (uint32_t)g.NY + (uint32_t)(c.gc[1] + g.py));
  return true;
}

// The boundary node a ghost cell stands for: the ghost reflected back across every face
// it lies beyond (for the one-cell layer, the nearest node), and its index pa in a
// plane.  mirror gets a bit per crossed symmetry face, open is set when an open face is
// crossed, zero_u when a zero-velocity face is.
struct GhostSrc {
  int a3[3];        // lattice coordinates (x global)
  uint32_t pa;
  int mirror;
  bool open, zero_u;
};
__device__ __forceinline__ GhostSrc ghost_src(const Geom &g, const GhostCell &c) {
  const int nn[3] = {c.len, g.ny, g.nz};
  GhostSrc r;
  r.mirror = 0;
  r.open = r.zero_u = false;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    int v = c.gc[d];
    if (v < 0 || v >= nn[d]) {
      const int bc = g.bc[2 * d + (v < 0 ? 0 : 1)];
      if (bc == LBM_BC_SYMMETRY) {
        r.mirror |= 1 << d;
      } else {
        r.open = true;
        r.zero_u |= (bc == LBM_BC_OPEN_EQ_U0);
      }
      v = v < 0 ? -1 - v : 2 * nn[d] - 1 - v;
    }
    r.a3[d] = v;
  }
  r.a3[0] += c.x0;
  r.pa = cell_index(g, r.a3[0], (uint32_t)(r.a3[2] + g.pz) * (uint32_t)g.NY + (uint32_t)(r.a3[1] + g.py));
  return r;
}

// Ghost layer of the non-periodic faces, after the collision.  Beyond an open face the
// ghost is the equilibrium at the adjacent boundary node (Sec. 5.1); beyond symmetry
// faces only, it is the mirror image: the post-collision population of the mirrored
// direction at the mirrored node (the quarter-domain flame of Sec. 5.2); beyond a
// symmetry and an open face, the equilibrium of the mirrored direction.
// SPLIT: one thread per (ghost cell, direction), the direction from the grid's y index
// (lattices with few ghost cells, where one thread per cell would run the 27 directions
// one after the other); otherwise one thread per cell.  Both give the same bits.
template <int M, typename ST, typename RT, bool SPLIT>
__global__ __launch_bounds__(128) void k_ghost(Geom g, Buffers b, CollideConsts kc, int cur, int64_t nx_slab,
                                               int64_t ny_slab, int64_t nz_slab) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  GhostCell c;
  if (!ghost_cell(g, t, nx_slab, ny_slab, nz_slab, c)) return;
  const GhostSrc gs = ghost_src(g, c);
  const int nn[3] = {c.len, g.ny, g.nz};
  const int64_t N = g.N;
  const int64_t na = ((int64_t)gs.a3[2] * g.ny + gs.a3[1]) * g.nx + gs.a3[0];
  const int64_t p = c.p, pa = gs.pa;
  ST *dst = static_cast<ST *>(b.pop[cur ^ 1]);
  if (SPLIT) {
    // leave before the equilibrium when no node pulls this direction from the cell
    const int i = blockIdx.y;
    const int cv[3] = {cx_of(i), cy_of(i), cz_of(i)};
    bool need = true;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const int t2 = c.gc[d] + cv[d];
      need = need && (g.per[d] || (t2 >= 0 && t2 < nn[d]));
    }
    if (!need) return;
  }
  EqState<M> e;
  if (gs.open) {
    const RT *srho = static_cast<const RT *>(b.side_rho);
    const RT *su = static_cast<const RT *>(b.side_u);
    const RT *sY = static_cast<const RT *>(b.side_Y);
    double u[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) u[d] = gs.zero_u ? 0.0 : double(su[d * N + na]);
    double Y[M];
#pragma unroll
    for (int a = 0; a < M; ++a) Y[a] = double(sY[a * N + na]);
    eq_state<M>(*b.tab, double(srho[na]), u, b.T[na], Y, e);
  }
  // only the directions along which a node of the lattice (of the segment, for x) pulls
  // from this ghost cell (a face cell serves 9, an edge cell 3, a corner cell 1); a
  // runtime loop keeps the kernel small
  const int i_lo = SPLIT ? (int)blockIdx.y : 0, i_hi = SPLIT ? (int)blockIdx.y + 1 : 27;
#pragma unroll 1
  for (int i = i_lo; i < i_hi; ++i) {
    const int cv[3] = {cx_of(i), cy_of(i), cz_of(i)};
    bool need = true;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const int t2 = c.gc[d] + cv[d];
      need = need && (g.per[d] || (t2 >= 0 && t2 < nn[d]));
    }
    if (!need) continue;
    int cm[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) cm[d] = (gs.mirror >> d & 1) ? -cv[d] : cv[d];
    if (gs.open) {
      write_eq_dir<M, ST>(e, kc, dst, g.NPAD, i, cm[0], cm[1], cm[2], p);
    } else {
      // the rest equilibria of the 16-bit formats are mirror-symmetric, so the stored
      // form copies as it is
      const int im = (cm[0] + 1) + 3 * (cm[1] + 1) + 9 * (cm[2] + 1);
#pragma unroll
      for (int s2 = 0; s2 <= M; ++s2)
        dst[((int64_t)s2 * Q + i) * g.NPAD + p] = dst[((int64_t)s2 * Q + im) * g.NPAD + pa];
    }
  }
}

// Deferred corrections of the ghost cells beyond symmetry faces only: the mirror image of
// those at the mirrored node, X and Cg with their components normal to the crossed
// faces reversed (both are odd under such a mirror).  After k_corr; other ghost cells
// keep zero.
template <typename CT>
__global__ __launch_bounds__(128) void k_ghost_corr(Geom g, Buffers b, int64_t nx_slab, int64_t ny_slab,
                                                    int64_t nz_slab) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  GhostCell gcl;
  if (!ghost_cell(g, t, nx_slab, ny_slab, nz_slab, gcl)) return;
  const GhostSrc gs = ghost_src(g, gcl);
  if (gs.open || gs.mirror == 0) return;
  const int64_t p = gcl.p, pa = gs.pa;
  CT *corr = static_cast<CT *>(b.corr);
  const int64_t NPAD = g.NPAD;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const bool flip = gs.mirror >> d & 1;
    const CT x = corr[d * NPAD + pa], c = corr[(3 + d) * NPAD + pa];
    corr[d * NPAD + p] = flip ? CT(-x) : x;
    corr[(3 + d) * NPAD + p] = flip ? CT(-c) : c;
  }
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
  const Corr<Side> cr{static_cast<const Side *>(b.corr), static_cast<const Side *>(b.corr) + 3 * g.NPAD, g.NPAD};
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
__global__ __launch_bounds__(64) void k_export(Geom g, Buffers b, CollideConsts kc, int cur,
                                                const int64_t *nodes, int64_t nn, double *out, double *T_out) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nn) return;
  const int64_t n = nodes[k];
  if (n < 0 || n >= g.N) return;
  // a lattice has fewer than 2^30 nodes: 32-bit division
  const uint32_t un = (uint32_t)n, unx = (uint32_t)g.nx, uny = (uint32_t)g.ny;
  const int x = (int)(un % unx), y = (int)((un / unx) % uny), z = (int)(un / (unx * uny));
  const int64_t NPAD = g.NPAD;
  using Side = typename Fmt<ST>::Side;
  const ST *pop = static_cast<const ST *>(b.pop[cur]);
  const Corr<Side> cr{static_cast<const Side *>(b.corr), static_cast<const Side *>(b.corr) + 3 * g.NPAD, g.NPAD};
  const AxisSrc ax = axis_src_x(g, x);
  const AxisSrc ay = axis_src(y, g.ny, g.per[1]);
  const AxisSrc az = axis_src(z, g.nz, g.per[2]);
  // one direction per grid row: 27 times the threads of a node loop
  const int kyz = blockIdx.y / 3, kx_run = blockIdx.y % 3;
  const int ky = kyz % 3, kz = kyz / 3;
  const int cy = ky - 1, cz = kz - 1;
  const int i = kx_run + 3 * kyz;
  const Src r = make_src(g, ax, ay, az, kx_run, ky, kz);
  // every set's value first, then the stores: a store between two loads would wait for
  // the first load, one round trip per set.  The species loads go out ahead of the
  // branch on the direction's x component, in which f and g are pulled with their
  // corrections, so that all the loads of the direction are in flight together.
  ST sp[M - 1];
#pragma unroll
  for (int a = 0; a < M - 1; ++a) sp[a] = ld(pop + ((int64_t)a * Q + i) * NPAD, r.ps);
  double v[M + 1];
  static_for<3>([&](auto Kx) {
    constexpr int kx = decltype(Kx)::value;
    constexpr int cx = kx - 1;
    if (kx != kx_run) return;
    v[M - 1] = pull_f<cx, ST, Side>(pop + ((int64_t)(M - 1) * Q + i) * NPAD, r, cr, cy, cz, M - 1, i, kc);
    v[M] = pull_g<cx, ST, Side>(pop + ((int64_t)M * Q + i) * NPAD, r, cr, cy, cz, M, i, kc);
  });
#pragma unroll
  for (int a = 0; a < M - 1; ++a) v[a] = pop_val(sp[a], a, i, kc);
#pragma unroll
  for (int s2 = 0; s2 <= M; ++s2) out[((int64_t)s2 * Q + i) * nn + k] = v[s2];
  if (T_out && blockIdx.y == 0) T_out[k] = b.T[n];
}

// ---- diagnostics (Sec. 5.2) -----------------------------------------------------------
// Production rates rho_dot_a of one node by mass action (Sec. 4): forward rate
// k_f = A T^b exp(-T_a / T) in log form, reverse rate k_f / K_c with K_c from the NASA-7
// Gibbs function at p0, concentrations rho_a rho_ref / m_a.
template <int M, typename TB>
__device__ __forceinline__ void node_rates(const TB &tb, const double *rs, double T, double *rdot) {
  const double invT = 1.0 / T, lnT = log(T);
  double c[M], gib[M], wd[M];
#pragma unroll
  for (int a = 0; a < M; ++a) {
    c[a] = rs[a] * tb.conc_scale[a];
    gib[a] = h_RT(tb.nasa[a], T, invT) - s_R(tb.nasa[a], T, lnT);
    wd[a] = 0.0;
  }
  const double ln_c0 = tb.ln_c0_const - lnT;
  for (int k = 0; k < tb.R; ++k) {
    const double lnkf = tb.lnA[k] + tb.bexp[k] * lnT - tb.Ta[k] * invT;
    double fwd = exp(lnkf);
#pragma unroll
    for (int a = 0; a < M; ++a)
      for (int r = 0; r < tb.nu_r[k][a]; ++r) fwd *= c[a];
    double rev = 0.0;
    if (tb.rev[k]) {
      double dG = 0.0;
#pragma unroll
      for (int a = 0; a < M; ++a) dG += tb.dnu_a[k][a] * gib[a];
      rev = exp(lnkf + dG - tb.dnu[k] * ln_c0);
#pragma unroll
      for (int a = 0; a < M; ++a)
        for (int r = 0; r < tb.nu_p[k][a]; ++r) rev *= c[a];
    }
    const double q = fwd - rev;
#pragma unroll
    for (int a = 0; a < M; ++a) wd[a] += tb.dnu_a[k][a] * q;
  }
#pragma unroll
  for (int a = 0; a < M; ++a) rdot[a] = tb.rdot_scale[a] * wd[a];
}

// Heat release rate -sum_a H_a rho_dot_a (Sec. 5.2) at every node of the current state,
// and per-workgroup partial sums of LBM_DIAG_TOTALS quantities, added up in a fixed
// order by k_diag_sum: heat release, cells with T >= T_iso, mass, total energy.
constexpr int DIAG_BLOCK = 128;
template <int M, typename ST, typename RT>
__global__ __launch_bounds__(DIAG_BLOCK) void k_diag(Geom g, Buffers b, CollideConsts kc, int cur, double T_iso,
                                                    double *hrr) {
  __shared__ double red[LBM_DIAG_TOTALS][DIAG_BLOCK];
  const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double v[LBM_DIAG_TOTALS] = {0.0, 0.0, 0.0, 0.0};
  if (n < g.N) {
    const int x = (int)(n % g.nx), y = (int)((n / g.nx) % g.ny), z = (int)(n / ((int64_t)g.nx * g.ny));
    using Side = typename Fmt<ST>::Side;
    const Corr<Side> cr{static_cast<const Side *>(b.corr), static_cast<const Side *>(b.corr) + 3 * g.NPAD,
                        g.NPAD};
    Macro<M> m;
    node_moments<M, ST>(g, static_cast<const ST *>(b.pop[cur]), cr, kc, x, y, z, m);
    const Tables &tb = *b.tab;
    double T;
    node_temperature<M>(tb, m, b.T[n], T);
    double rdot[M];
    node_rates<M>(tb, m.rs, T, rdot);
    const double invT = 1.0 / T;
    double h = 0.0;
#pragma unroll
    for (int a = 0; a < M; ++a) h -= tb.Ra[a] * T * h_RT(tb.nasa[a], T, invT) * rdot[a];
    if (hrr) hrr[n] = h;
    v[0] = h;
    v[1] = T >= T_iso ? 1.0 : 0.0;
    v[2] = m.rho;
    v[3] = m.rhoE;
  }
#pragma unroll
  for (int k = 0; k < LBM_DIAG_TOTALS; ++k) red[k][threadIdx.x] = v[k];
  __syncthreads();
  for (int w = DIAG_BLOCK / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w)
#pragma unroll
      for (int k = 0; k < LBM_DIAG_TOTALS; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0)
#pragma unroll
    for (int k = 0; k < LBM_DIAG_TOTALS; ++k) b.diag[(int64_t)k * gridDim.x + blockIdx.x] = red[k][0];
}

// total k of the partial sums: one workgroup per total, a fixed strided order and a
// fixed tree, so that the result does not depend on scheduling
constexpr int DIAG_SUM_BLOCK = 256;
__global__ __launch_bounds__(DIAG_SUM_BLOCK) void k_diag_sum(const double *part, int64_t nparts,
                                                              double *totals) {
  __shared__ double red[DIAG_SUM_BLOCK];
  const int k = blockIdx.x;
  double acc = 0.0;
  for (int64_t j = threadIdx.x; j < nparts; j += DIAG_SUM_BLOCK) acc += part[(int64_t)k * nparts + j];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = DIAG_SUM_BLOCK / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) totals[k] = red[0];
}

// ---- flame-front speeds (Sec. 5.2, eq. sd) --------------------------------------------
// Work fields [FS_WORK][N] of the caller: node-local values, then the gradients.
enum { FS_T, FS_LAM, FS_HRR, FS_RHOCP, FS_V, FS_U = FS_V + 3, FS_RHO = FS_U + 3, FS_GT, FS_G = FS_GT + 3,
       FS_WORK = FS_G + 3 };
static_assert(FS_WORK == LBM_FLAME_WORK, "work fields of lbm_flame_speeds");

// Node-local part: T (Newton), heat release -sum_a H_a rho_dot_a, C_p = sum_a Y_a C_p,a,
// the conductivity lambda = (1/omega1 - 1/2) P C_p (eq. lambda, dt = 1), and the
// enthalpy-diffusion vector V = sum_a C_p,a Y_a du_a with du_a from the Stefan-Maxwell
// system (1 + 1/(2 tau_a)) du_a - 1/2 sum_b K_ab Y_b du_b = u_a - u (eqs. tauab,
// transform1), solved by elimination without pivoting (strictly diagonally dominant).
template <int M, typename ST, typename RT>
__global__ __launch_bounds__(128) void k_fs_local(Geom g, Buffers b, CollideConsts kc, int cur, double *work) {
  const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= g.N) return;
  const int x = (int)(n % g.nx), y = (int)((n / g.nx) % g.ny), z = (int)(n / ((int64_t)g.nx * g.ny));
  using Side = typename Fmt<ST>::Side;
  const Corr<Side> cr{static_cast<const Side *>(b.corr), static_cast<const Side *>(b.corr) + 3 * g.NPAD, g.NPAD};
  Macro<M> m;
  node_moments<M, ST>(g, static_cast<const ST *>(b.pop[cur]), cr, kc, x, y, z, m);
  const Tables &tb = *b.tab;
  double T;
  node_temperature<M>(tb, m, b.T[n], T);
  double rdot[M];
  node_rates<M>(tb, m.rs, T, rdot);
  const double invT = 1.0 / T, inv_rho = 1.0 / m.rho;
  double Y[M], cpa[M], za[M];
  double hrr = 0.0, cp = 0.0, zeta = 0.0;
#pragma unroll
  for (int a = 0; a < M; ++a) {
    Y[a] = m.rs[a] * inv_rho;
    const double *c = tb.nasa[a];
    za[a] = tb.Ra[a] * T;
    cpa[a] = tb.Ra[a] * (c[0] + T * (c[1] + T * (c[2] + T * (c[3] + T * c[4]))));
    hrr -= za[a] * h_RT(c, T, invT) * rdot[a];
    cp += Y[a] * cpa[a];
    zeta += Y[a] * za[a];
  }
  double A[M][M], r[M][3];
  const double sD = inv_diff_scale(tb, T) / zeta;
#pragma unroll
  for (int a = 0; a < M; ++a) {
    double it = 0.0;
#pragma unroll
    for (int c = 0; c < M; ++c) {
      const double K = (a == c) ? 0.0 : za[a] * za[c] * tb.invD[a][c] * sD;
      A[a][c] = -0.5 * K * Y[c];
      it += Y[c] * K;
    }
    A[a][a] = 1.0 + 0.5 * it;
#pragma unroll
    for (int d = 0; d < 3; ++d) r[a][d] = m.du0[a][d];
  }
#pragma unroll
  for (int k = 0; k < M; ++k)
#pragma unroll
    for (int q = k + 1; q < M; ++q) {
      const double l = A[q][k] / A[k][k];
#pragma unroll
      for (int c = k; c < M; ++c) A[q][c] -= l * A[k][c];
#pragma unroll
      for (int d = 0; d < 3; ++d) r[q][d] -= l * r[k][d];
    }
  double V[3] = {0.0, 0.0, 0.0};
#pragma unroll
  for (int q = M - 1; q >= 0; --q)
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      double v = r[q][d];
#pragma unroll
      for (int c = q + 1; c < M; ++c) v -= A[q][c] * r[c][d];
      r[q][d] = v / A[q][q];
      V[d] += cpa[q] * Y[q] * r[q][d];
    }
  const int64_t N = g.N;
  work[FS_T * N + n] = T;
  double om, om1;
  relax_rates(tb, T, om, om1);
  work[FS_LAM * N + n] = (1.0 / om1 - 0.5) * m.rho * zeta * cp;
  work[FS_HRR * N + n] = hrr;
  work[FS_RHOCP * N + n] = m.rho * cp;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    work[(FS_V + d) * N + n] = V[d];
    work[(FS_U + d) * N + n] = m.u[d];
  }
  work[FS_RHO * N + n] = m.rho;
}

// neighbour coordinates of the isotropic gradient (wrapped on periodic axes, clamped at
// open and symmetry faces and at the ends of a segment), and the sign of a component
// normal to a symmetry face across it
struct Nbr {
  int xs[3], ys[3], zs[3];
  double sg[3][3];
};
__device__ __forceinline__ Nbr neighbours(const Geom &g, int x, int y, int z) {
  const XSeg xsg = x_segment(g, x);
  Nbr r;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    r.xs[k] = g.per[0] ? nb_coord(x, k - 1, g.nx, true) : min(max(x + k - 1, xsg.x0), xsg.x1);
    r.ys[k] = nb_coord(y, k - 1, g.ny, g.per[1]);
    r.zs[k] = nb_coord(z, k - 1, g.nz, g.per[2]);
  }
  const int xyz[3] = {x, y, z}, lo3[3] = {xsg.x0, 0, 0}, hi3[3] = {xsg.x1, g.ny - 1, g.nz - 1};
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    r.sg[a][0] = (xyz[a] == lo3[a] && g.bc[2 * a] == LBM_BC_SYMMETRY) ? -1.0 : 1.0;
    r.sg[a][1] = 1.0;
    r.sg[a][2] = (xyz[a] == hi3[a] && g.bc[2 * a + 1] == LBM_BC_SYMMETRY) ? -1.0 : 1.0;
  }
  return r;
}

// grad T, and G = lambda grad T
__global__ __launch_bounds__(256) void k_fs_grad(Geom g, double *work) {
  const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= g.N) return;
  const int x = (int)(n % g.nx), y = (int)((n / g.nx) % g.ny), z = (int)(n / ((int64_t)g.nx * g.ny));
  const Nbr nb = neighbours(g, x, y, z);
  const int64_t N = g.N;
  const double *T = work + FS_T * N;
  double gr[3] = {0.0, 0.0, 0.0};
  static_for<27>([&](auto Ic) {
    constexpr int I = decltype(Ic)::value;
    constexpr int cx = cx_of(I), cy = cy_of(I), cz = cz_of(I);
    if constexpr (I != 13) {
      const int64_t nn = ((int64_t)nb.zs[cz + 1] * g.ny + nb.ys[cy + 1]) * g.nx + nb.xs[cx + 1];
      constexpr double w = 3.0 * wgt(I);
      const double v = T[nn];
      if constexpr (cx != 0) gr[0] += (cx * w) * v;
      if constexpr (cy != 0) gr[1] += (cy * w) * v;
      if constexpr (cz != 0) gr[2] += (cz * w) * v;
    }
  });
  const double lam = work[FS_LAM * N + n];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    work[(FS_GT + d) * N + n] = gr[d];
    work[(FS_G + d) * N + n] = lam * gr[d];
  }
}

// S_d (eq. sd), S_a = S_d + u.n, isosurface weight w, and per-workgroup partial sums
// [w, w S_d, w S_a, w rho S_d, w |x - centre|] (fixed tree, added by k_diag_sum)
__global__ __launch_bounds__(DIAG_BLOCK) void k_fs_final(Geom g, const double *work, double T_iso, double cx0,
                                                         double cy0, double cz0, double *out, double *part) {
  __shared__ double red[LBM_FLAME_TOTALS][DIAG_BLOCK];
  const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double v[LBM_FLAME_TOTALS] = {0.0, 0.0, 0.0, 0.0, 0.0};
  if (n < g.N) {
    const int x = (int)(n % g.nx), y = (int)((n / g.nx) % g.ny), z = (int)(n / ((int64_t)g.nx * g.ny));
    const Nbr nb = neighbours(g, x, y, z);
    const int64_t N = g.N;
    const double *G = work + FS_G * N;
    double div = 0.0;
    static_for<27>([&](auto Ic) {
      constexpr int I = decltype(Ic)::value;
      constexpr int cx = cx_of(I), cy = cy_of(I), cz = cz_of(I);
      if constexpr (I != 13) {
        const int64_t nn = ((int64_t)nb.zs[cz + 1] * g.ny + nb.ys[cy + 1]) * g.nx + nb.xs[cx + 1];
        constexpr double w = 3.0 * wgt(I);
        if constexpr (cx != 0) div += (cx * w) * (nb.sg[0][cx + 1] * G[nn]);
        if constexpr (cy != 0) div += (cy * w) * (nb.sg[1][cy + 1] * G[N + nn]);
        if constexpr (cz != 0) div += (cz * w) * (nb.sg[2][cz + 1] * G[2 * N + nn]);
      }
    });
    double gt[3], flux = 0.0, g2 = 0.0, ug = 0.0;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      gt[d] = work[(FS_GT + d) * N + n];
      flux += work[(FS_V + d) * N + n] * gt[d];
      g2 += gt[d] * gt[d];
      ug += work[(FS_U + d) * N + n] * gt[d];
    }
    const double mag = sqrt(g2), rho = work[FS_RHO * N + n], T = work[FS_T * N + n];
    double Sd = 0.0, Sa = 0.0, wt = 0.0;
    if (mag > 0.0) {
      Sd = (work[FS_HRR * N + n] + div - rho * flux) / (work[FS_RHOCP * N + n] * mag);
      Sa = Sd - ug / mag;
      wt = fmax(0.0, 1.0 - fabs(T - T_iso) / mag);
    }
    if (out) {
      out[n] = Sd;
      out[N + n] = Sa;
      out[2 * N + n] = wt;
    }
    const double dx = x - cx0, dy = y - cy0, dz = z - cz0;
    v[0] = wt;
    v[1] = wt * Sd;
    v[2] = wt * Sa;
    v[3] = wt * rho * Sd;
    v[4] = wt * sqrt(dx * dx + dy * dy + dz * dz);
  }
#pragma unroll
  for (int k = 0; k < LBM_FLAME_TOTALS; ++k) red[k][threadIdx.x] = v[k];
  __syncthreads();
  for (int w = DIAG_BLOCK / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w)
#pragma unroll
      for (int k = 0; k < LBM_FLAME_TOTALS; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0)
#pragma unroll
    for (int k = 0; k < LBM_FLAME_TOTALS; ++k) part[(int64_t)k * gridDim.x + blockIdx.x] = red[k][0];
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

inline bool any_symmetry(const Geom &g) {
  for (int k = 0; k < 6; ++k)
    if (g.bc[k] == LBM_BC_SYMMETRY) return true;
  return false;
}
template <int M, typename ST, typename RT>
struct RunStep {
  static hipError_t run(const Geom &g, const Buffers &b, const CollideConsts &kc, int cur, hipStream_t st) {
    (void)kc;   // k_step reads the device copy of the constants (Buffers::kc)
    if (!g.vt) {
      hipLaunchKernelGGL((k_step<M, ST, false>), dim3(blocks_for(g.N, ISL_BLOCK)), dim3(ISL_BLOCK), 0, st, g, b,
                         cur);
    } else if constexpr (sizeof(ST) >= 4) {
      hipLaunchKernelGGL((k_step<M, ST, true>), dim3(blocks_for(g.N, ISL_BLOCK)), dim3(ISL_BLOCK), 0, st, g, b,
                         cur);
    } else {
      return hipErrorInvalidValue;   // rejected by the descriptor check: FP64 and FP32 storage only
    }
    return hipGetLastError();
  }
};
template <int M, typename ST, typename RT>
struct RunCorr {
  static hipError_t run(const Geom &g, const Buffers &b, hipStream_t st) {
    switch (g.corr_tile) {
#define LBM_CORR_CASE(K)                                                                              \
  case K:                                                                                             \
    hipLaunchKernelGGL((k_corr<M, RT, RT, K>), dim3((unsigned)corr_tiles<K>(g)), dim3(CorrTile<K>::THREADS), 0, \
                       st, g, b);                                                                     \
    break;
      LBM_CORR_CASE(0) LBM_CORR_CASE(1) LBM_CORR_CASE(2) LBM_CORR_CASE(3) LBM_CORR_CASE(4) LBM_CORR_CASE(5)
      LBM_CORR_CASE(9)
#undef LBM_CORR_CASE
#define LBM_MARCH_CASE(K)                                                                              \
  case K:                                                                                              \
    if (any_symmetry(g))                                                                               \
      hipLaunchKernelGGL((k_corr_march<M, RT, RT, K, true>), dim3((unsigned)march_tiles<K, RT>(g)),     \
                         dim3(MarchTile<K, RT>::THREADS), 0, st, g, b);                                \
    else                                                                                               \
      hipLaunchKernelGGL((k_corr_march<M, RT, RT, K, false>), dim3((unsigned)march_tiles<K, RT>(g)),    \
                         dim3(MarchTile<K, RT>::THREADS), 0, st, g, b);                                \
    break;
      LBM_MARCH_CASE(6)
#undef LBM_MARCH_CASE
      default: return hipErrorInvalidValue;
    }
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
    const int64_t sx = g.xg ? 2LL * g.nseg * g.NY * g.NZ : 0;
    const int64_t sy = g.py ? 2LL * g.nx * g.NZ : 0;
    const int64_t sz = g.pz ? 2LL * g.nx * g.ny : 0;
    const int64_t tot = sx + sy + sz;
    if (tot == 0) return hipSuccess;
    // below 32768 ghost cells (quasi-1D flames and their batches, small lattices) a
    // thread per cell and direction; above, a thread per cell
    if (tot < 32768)
      hipLaunchKernelGGL((k_ghost<M, ST, RT, true>), dim3(blocks_for(tot, 128), 27), dim3(128), 0, st, g, b, kc, cur,
                         sx, sy, sz);
    else
      hipLaunchKernelGGL((k_ghost<M, ST, RT, false>), dim3(blocks_for(tot, 128)), dim3(128), 0, st, g, b, kc, cur,
                         sx, sy, sz);
    return hipGetLastError();
  }
};
template <int M, typename ST, typename RT>
struct RunDiag {
  static hipError_t run(const Geom &g, const Buffers &b, const CollideConsts &kc, int cur, double T_iso,
                        double *hrr, double *totals, hipStream_t st) {
    const unsigned nb = blocks_for(g.N, DIAG_BLOCK);
    hipLaunchKernelGGL((k_diag<M, ST, RT>), dim3(nb), dim3(DIAG_BLOCK), 0, st, g, b, kc, cur, T_iso, hrr);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess && totals) {
      hipLaunchKernelGGL(k_diag_sum, dim3(LBM_DIAG_TOTALS), dim3(DIAG_SUM_BLOCK), 0, st, b.diag, (int64_t)nb,
                         totals);
      e = hipGetLastError();
    }
    return e;
  }
};
template <int M, typename ST, typename RT>
struct RunFlame {
  static hipError_t run(const Geom &g, const Buffers &b, const CollideConsts &kc, int cur, double T_iso,
                        const double *centre, double *work, double *part, double *out, double *totals,
                        hipStream_t st) {
    hipLaunchKernelGGL((k_fs_local<M, ST, RT>), dim3(blocks_for(g.N, 128)), dim3(128), 0, st, g, b, kc, cur, work);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_fs_grad, dim3(blocks_for(g.N, 256)), dim3(256), 0, st, g, work);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    const unsigned nb = blocks_for(g.N, DIAG_BLOCK);
    hipLaunchKernelGGL(k_fs_final, dim3(nb), dim3(DIAG_BLOCK), 0, st, g, (const double *)work, T_iso, centre[0],
                       centre[1], centre[2], out, part);
    e = hipGetLastError();
    if (e == hipSuccess && totals) {
      hipLaunchKernelGGL(k_diag_sum, dim3(LBM_FLAME_TOTALS), dim3(DIAG_SUM_BLOCK), 0, st, (const double *)part,
                         (int64_t)nb, totals);
      e = hipGetLastError();
    }
    return e;
  }
};
template <int M, typename ST, typename RT>
struct RunGhostCorr {
  static hipError_t run(const Geom &g, const Buffers &b, hipStream_t st) {
    if (!any_symmetry(g)) return hipSuccess;
    const int64_t sx = g.xg ? 2LL * g.nseg * g.NY * g.NZ : 0;
    const int64_t sy = g.py ? 2LL * g.nx * g.NZ : 0;
    const int64_t sz = g.pz ? 2LL * g.nx * g.ny : 0;
    const int64_t tot = sx + sy + sz;
    if (tot == 0) return hipSuccess;
    hipLaunchKernelGGL((k_ghost_corr<RT>), dim3(blocks_for(tot, 128)), dim3(128), 0, st, g, b, sx, sy, sz);
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
    hipLaunchKernelGGL((k_export<M, ST, RT>), dim3(blocks_for(nn, 64), 27), dim3(64), 0, st, g, b, kc, cur, nodes,
                       nn, out, T_out);
    return hipGetLastError();
  }
};

}  // namespace

hipError_t launch_step(const Geom &g, const Buffers &b, const CollideConsts &kc, int store, int cur,
                       hipStream_t st) {
  return dispatch<RunStep>(g.M, store, g, b, kc, cur, st);
}

template <typename RT>
void launch_psi_rt(const Geom &g, const Buffers &b, hipStream_t st) {
  if (any_symmetry(g))
    hipLaunchKernelGGL((k_psi<RT, true>), dim3(blocks_for(g.N, 256)), dim3(256), 0, st, g, b);
  else
    hipLaunchKernelGGL((k_psi<RT, false>), dim3(blocks_for(g.N, 256)), dim3(256), 0, st, g, b);
}

hipError_t launch_psi(const Geom &g, const Buffers &b, int store, hipStream_t st) {
  if (store == LBM_STORE_F64)
    launch_psi_rt<Fmt<double>::Side>(g, b, st);
  else if (store == LBM_STORE_F32)
    launch_psi_rt<Fmt<float>::Side>(g, b, st);
  else
    launch_psi_rt<float>(g, b, st);
  return hipGetLastError();
}

int corr_tile_candidates(const Geom &g, int *out) {
  // the thin tiles take the node's own row for every y and z neighbour: one node thick only
  const bool thin = g.ny == 1 && g.nz == 1;
  if (thin) {
    for (int k = 0; k < 3; ++k) out[k] = 3 + k;
    return 3;
  }
  // the tiles of k_corr after k_psi, then the z-marching shape that forms psi itself,
  // and on a lattice one node thick in z the flat tile
  for (int k = 0; k < 3; ++k) out[k] = k;
  out[3] = 6;
  if (g.nz == 1) {
    out[4] = 9;
    return 5;
  }
  return 4;
}

bool corr_forms_psi(int tile) { return tile == 6; }

hipError_t launch_corr_only(const Geom &g, const Buffers &b, int store, hipStream_t st) {
  return dispatch<RunCorr>(g.M, store, g, b, st);
}

hipError_t launch_corr(const Geom &g, const Buffers &b, int store, hipStream_t st) {
  hipError_t e = dispatch<RunCorr>(g.M, store, g, b, st);
  if (e == hipSuccess) e = dispatch<RunGhostCorr>(g.M, store, g, b, st);
  return e;
}

hipError_t launch_init(const Geom &g, const Buffers &b, const CollideConsts &kc, int store, const double *rho,
                       const double *u, const double *T, const double *Y, int cur, hipStream_t st) {
  return dispatch<RunInit>(g.M, store, g, b, kc, rho, u, T, Y, cur, st);
}

hipError_t launch_ghost(const Geom &g, const Buffers &b, const CollideConsts &kc, int store, int cur,
                        hipStream_t st) {
  return dispatch<RunGhost>(g.M, store, g, b, kc, cur, st);
}

hipError_t launch_diag(const Geom &g, const Buffers &b, const CollideConsts &kc, int store, int cur, double T_iso,
                       double *hrr, double *totals, hipStream_t st) {
  return dispatch<RunDiag>(g.M, store, g, b, kc, cur, T_iso, hrr, totals, st);
}

hipError_t launch_flame(const Geom &g, const Buffers &b, const CollideConsts &kc, int store, int cur, double T_iso,
                        const double *centre, double *work, double *out, double *totals, hipStream_t st) {
  return dispatch<RunFlame>(g.M, store, g, b, kc, cur, T_iso, centre, work, b.diag, out, totals, st);
}

// ---- scratch of the allocation-free flame speeds ----------------------------------------
// The work fields (LBM_FLAME_WORK per node) and the per-workgroup partial sums of
// lbm_flame_speeds_static, for lattices of up to LBM_FLAME_STATIC_MAX_NODES nodes.  Each
// device holds its own copy for the life of the process.  Host code never passes the
// name `scratch` to a kernel: it stands for the host shadow of the symbol, not a device
// address.  The address on each device is resolved once, with that device current, and
// kept in flame_scratch_ptr.
constexpr int64_t FLAME_STATIC_PARTS = (LBM_FLAME_STATIC_MAX_NODES + DIAG_BLOCK - 1) / DIAG_BLOCK;
constexpr int64_t FLAME_STATIC_WORDS =
    (int64_t)LBM_FLAME_WORK * LBM_FLAME_STATIC_MAX_NODES + (int64_t)LBM_FLAME_TOTALS * FLAME_STATIC_PARTS;
static __device__ __align__(256) double scratch[FLAME_STATIC_WORDS];

constexpr int MAX_DEVICES = 64;
static std::mutex flame_scratch_mu;
static double *flame_scratch_ptr[MAX_DEVICES];

hipError_t flame_scratch_resolve(int device) {
  if (device < 0 || device >= MAX_DEVICES) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(flame_scratch_mu);
  if (flame_scratch_ptr[device]) return hipSuccess;
  void *p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  if (!p) return hipErrorInvalidSymbol;
  flame_scratch_ptr[device] = static_cast<double *>(p);
  return hipSuccess;
}

hipError_t launch_flame_static(const Geom &g, const Buffers &b, const CollideConsts &kc, int store, int cur,
                               int device, double T_iso, const double *centre, double *out, double *totals,
                               hipStream_t st) {
  if (g.N > LBM_FLAME_STATIC_MAX_NODES) return hipErrorInvalidValue;
  double *base = nullptr;
  {
    std::lock_guard<std::mutex> lock(flame_scratch_mu);
    if (device >= 0 && device < MAX_DEVICES) base = flame_scratch_ptr[device];
  }
  if (!base) return hipErrorInvalidSymbol;   // not resolved by lbm_create on this device
  double *work = base;
  double *part = base + (int64_t)LBM_FLAME_WORK * LBM_FLAME_STATIC_MAX_NODES;
  return dispatch<RunFlame>(g.M, store, g, b, kc, cur, T_iso, centre, work, part, out, totals, st);
}

hipError_t launch_macros(const Geom &g, const Buffers &b, const CollideConsts &kc, int store, int cur,
                         double *rho, double *u, double *T, double *P, double *Y, hipStream_t st) {
  return dispatch<RunMacros>(g.M, store, g, b, kc, cur, rho, u, T, P, Y, st);
}

hipError_t launch_export(const Geom &g, const Buffers &b, const CollideConsts &kc, int store, int cur,
                         const int64_t *nodes, int64_t n_nodes, double *out, double *T_out, hipStream_t st) {
  return dispatch<RunExport>(g.M, store, g, b, kc, cur, nodes, n_nodes, out, T_out, st);
}

// Streaming copy with 16-byte loads and stores, four per lane in flight, grid-stride
// over the buffer: the read + write bandwidth a streaming kernel reaches on the chip.
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
__global__ __launch_bounds__(256) void k_stream_copy(const u32x4 *__restrict__ src, u32x4 *__restrict__ dst,
                                                     int64_t n16) {
  const int64_t stride = (int64_t)gridDim.x * 256 * 4;
  for (int64_t base = (int64_t)blockIdx.x * 256 * 4 + threadIdx.x; base < n16; base += stride) {
    u32x4 v[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int64_t i = base + (int64_t)k * 256;
      if (i < n16) v[k] = src[i];
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int64_t i = base + (int64_t)k * 256;
      if (i < n16) dst[i] = v[k];
    }
  }
}

hipError_t launch_stream_copy(const void *src, void *dst, int64_t bytes, hipStream_t st) {
  const int64_t n16 = bytes / 16;
  if (n16 <= 0) return hipSuccess;
  // 8 workgroups of 256 lanes per CU on the 256 CUs, each lane 4 x 16 bytes per round
  const int64_t want = (n16 + 1023) / 1024;
  const unsigned grid = (unsigned)(want < 2048 ? want : 2048);
  hipLaunchKernelGGL(k_stream_copy, dim3(grid), dim3(256), 0, st, static_cast<const u32x4 *>(src),
                     static_cast<u32x4 *>(dst), n16);
  return hipGetLastError();
}

hipError_t launch_zero(void *p, int64_t n_words32, hipStream_t st) {
  if (n_words32 <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_zero, dim3(blocks_for(n_words32, 256)), dim3(256), 0, st, static_cast<uint32_t *>(p),
                     n_words32);
  return hipGetLastError();
}

}  // namespace lbm
