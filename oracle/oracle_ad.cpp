/*
 * Reverse sweep of the FP64 CPU oracle (test infrastructure only).
 *
 * TEST INFRASTRUCTURE ONLY: the reference the discrete adjoint of the HIP path is
 * checked against.  Only the tests may load it.
 *
 * The oracle's own source (oracle.c) is compiled here a second time with its
 * arithmetic type replaced by a recording type: every operation on a value that
 * depends on the state or on the Arrhenius parameters appends one entry (its operands
 * and the partial derivatives with respect to them) to a tape.  A reverse pass over
 * the tape then gives the vector-Jacobian product of whatever was recorded: one step
 * of the method (Sec. 2-4), the macroscopic fields of a state, or the equilibrium
 * initial state.  No derivative of the method is written by hand here; they follow
 * from the forward steps of the oracle, in the paper's order, through the chain rule.
 * The temperature comes from Newton's iterations on the energy (eq. temperature), and
 * the tape differentiates the iterations as taken: once converged to |dT| <= 1e-12 T
 * their derivative is that of the implicit function to the same order.
 */
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

namespace ad {

// one recorded operation: result = f(x, y), with d result / d x = dx, d / d y = dy;
// operand id 0 is a constant (no entry), so unary operations leave y = 0
struct Entry {
  int32_t x, y;
  double dx, dy;
};

struct Tape {
  std::vector<Entry> e;   // entry k records variable k + 1
  bool on = false;
  int32_t next_id() const { return (int32_t)e.size() + 1; }
};

inline Tape &tape() {
  static Tape t;
  return t;
}

}  // namespace ad

struct adouble {
  double v;
  int32_t id;   // 0: a constant; otherwise the tape variable holding this value
  adouble() = default;
  adouble(double x) : v(x), id(0) {}
  adouble(double x, int32_t i) : v(x), id(i) {}
};

namespace ad {

inline adouble rec1(double v, const adouble &x, double dx) {
  Tape &t = tape();
  if (!t.on || x.id == 0) return adouble(v);
  t.e.push_back(Entry{x.id, 0, dx, 0.0});
  return adouble(v, (int32_t)t.e.size());
}

inline adouble rec2(double v, const adouble &x, double dx, const adouble &y, double dy) {
  Tape &t = tape();
  if (!t.on || (x.id == 0 && y.id == 0)) return adouble(v);
  if (x.id == 0) return rec1(v, y, dy);
  if (y.id == 0) return rec1(v, x, dx);
  t.e.push_back(Entry{x.id, y.id, dx, dy});
  return adouble(v, (int32_t)t.e.size());
}

// a new independent variable of the given value
inline adouble input(double v) {
  Tape &t = tape();
  t.e.push_back(Entry{0, 0, 0.0, 0.0});
  return adouble(v, (int32_t)t.e.size());
}

// adjoints of all variables from seeds already placed in adj (indexed by id)
inline void reverse(std::vector<double> &adj) {
  const std::vector<Entry> &e = tape().e;
  for (int64_t k = (int64_t)e.size(); k >= 1; --k) {
    const double a = adj[k];
    if (a == 0.0) continue;
    const Entry &en = e[k - 1];
    if (en.x) adj[en.x] += en.dx * a;
    if (en.y) adj[en.y] += en.dy * a;
  }
}

}  // namespace ad

inline adouble operator+(const adouble &a, const adouble &b) { return ad::rec2(a.v + b.v, a, 1.0, b, 1.0); }
inline adouble operator-(const adouble &a, const adouble &b) { return ad::rec2(a.v - b.v, a, 1.0, b, -1.0); }
inline adouble operator*(const adouble &a, const adouble &b) { return ad::rec2(a.v * b.v, a, b.v, b, a.v); }
inline adouble operator/(const adouble &a, const adouble &b) {
  const double r = a.v / b.v;
  return ad::rec2(r, a, 1.0 / b.v, b, -r / b.v);
}
inline adouble operator+(const adouble &a, double b) { return ad::rec1(a.v + b, a, 1.0); }
inline adouble operator+(double a, const adouble &b) { return ad::rec1(a + b.v, b, 1.0); }
inline adouble operator-(const adouble &a, double b) { return ad::rec1(a.v - b, a, 1.0); }
inline adouble operator-(double a, const adouble &b) { return ad::rec1(a - b.v, b, -1.0); }
inline adouble operator*(const adouble &a, double b) { return ad::rec1(a.v * b, a, b); }
inline adouble operator*(double a, const adouble &b) { return ad::rec1(a * b.v, b, a); }
inline adouble operator/(const adouble &a, double b) { return ad::rec1(a.v / b, a, 1.0 / b); }
inline adouble operator/(double a, const adouble &b) {
  const double r = a / b.v;
  return ad::rec1(r, b, -r / b.v);
}
inline adouble operator-(const adouble &a) { return ad::rec1(-a.v, a, -1.0); }
inline adouble &operator+=(adouble &a, const adouble &b) { return a = a + b; }
inline adouble &operator-=(adouble &a, const adouble &b) { return a = a - b; }
inline adouble &operator*=(adouble &a, const adouble &b) { return a = a * b; }
inline adouble &operator/=(adouble &a, const adouble &b) { return a = a / b; }
inline bool operator<(const adouble &a, const adouble &b) { return a.v < b.v; }
inline bool operator>(const adouble &a, const adouble &b) { return a.v > b.v; }
inline bool operator<=(const adouble &a, const adouble &b) { return a.v <= b.v; }
inline bool operator>=(const adouble &a, const adouble &b) { return a.v >= b.v; }
inline bool operator<(const adouble &a, double b) { return a.v < b; }
inline bool operator>(const adouble &a, double b) { return a.v > b; }
inline bool operator<=(const adouble &a, double b) { return a.v <= b; }
inline bool operator>=(const adouble &a, double b) { return a.v >= b; }
inline bool operator<(double a, const adouble &b) { return a < b.v; }
inline bool operator>(double a, const adouble &b) { return a > b.v; }
inline adouble exp(const adouble &a) {
  const double r = std::exp(a.v);
  return ad::rec1(r, a, r);
}
inline adouble log(const adouble &a) { return ad::rec1(std::log(a.v), a, 1.0 / a.v); }
inline adouble sqrt(const adouble &a) {
  const double r = std::sqrt(a.v);
  return ad::rec1(r, a, 0.5 / r);
}
inline adouble fabs(const adouble &a) { return ad::rec1(std::fabs(a.v), a, a.v < 0.0 ? -1.0 : 1.0); }
inline adouble pow(const adouble &a, double b) {
  const double r = std::pow(a.v, b);
  return ad::rec1(r, a, b * std::pow(a.v, b - 1.0));
}
inline adouble pow(const adouble &a, const adouble &b) {
  const double r = std::pow(a.v, b.v);
  return ad::rec2(r, a, b.v * std::pow(a.v, b.v - 1.0), b, r * std::log(a.v));
}
inline bool isfinite(const adouble &a) { return std::isfinite(a.v); }

#define ORC_REAL 1
typedef adouble real;
#define ORC_VAL(x) ((x).v)
#include "oracle.c"

namespace {

int64_t last_entries = 0;

// state and parameters back to constants (values kept), tape cleared
void settle(orc_sim *s) {
  last_entries = (int64_t)ad::tape().e.size();
  const int64_t n = (int64_t)s->S * Q * s->N;
  for (int64_t k = 0; k < n; ++k) s->pop[k].id = 0;
  for (int k = 0; k < s->p.R; ++k)
    for (int c = 0; c < 3; ++c) s->arrh[k][c].id = 0;
  ad::tape().e.clear();
  ad::tape().on = false;
}

void start(orc_sim *s) {
  ad::tape().e.clear();
  ad::tape().on = true;
  (void)s;
}

}  // namespace

extern "C" {

/* One step of the method from the current state, recorded, then reversed:
 *   lam_prev[S][27][N] = (d pop_{n+1} / d pop_n)^T lam_next,
 *   grad[R][3] += (d pop_{n+1} / d (ln A_k, b_k, Ta_k))^T lam_next.
 * The state advances by the step, as orc_step does.  Returns the anomaly bits. */
uint32_t orc_ad_step_vjp(orc_sim *s, const double *lam_next, double *lam_prev, double *grad) {
  const int64_t n = (int64_t)s->S * Q * s->N;
  const int R = s->p.R;
  start(s);
  std::vector<int32_t> in_id((size_t)n);
  for (int64_t k = 0; k < n; ++k) {
    s->pop[k] = ad::input(s->pop[k].v);
    in_id[(size_t)k] = s->pop[k].id;
  }
  std::vector<int32_t> par_id((size_t)3 * R);
  for (int k = 0; k < R; ++k) {
    const adouble lnA = ad::input(std::log(s->arrh[k][0].v));
    par_id[(size_t)3 * k] = lnA.id;
    const double A0 = s->arrh[k][0].v;
    s->arrh[k][0] = exp(lnA);
    s->arrh[k][0].v = A0;   // the exact value the plain oracle uses; derivative d A / d ln A = A
    for (int c = 1; c < 3; ++c) {
      s->arrh[k][c] = ad::input(s->arrh[k][c].v);
      par_id[(size_t)3 * k + c] = s->arrh[k][c].id;
    }
  }
  const uint32_t anom = orc_step(s, 1, 1);
  std::vector<double> adj((size_t)ad::tape().next_id(), 0.0);
  for (int64_t k = 0; k < n; ++k)
    if (s->pop[k].id) adj[(size_t)s->pop[k].id] += lam_next[k];
  ad::reverse(adj);
  for (int64_t k = 0; k < n; ++k) lam_prev[k] = adj[(size_t)in_id[(size_t)k]];
  if (grad)
    for (int k = 0; k < 3 * R; ++k) grad[k] += adj[(size_t)par_id[(size_t)k]];
  settle(s);
  return anom;
}

/* Adjoint of the macroscopic fields of the current state: lam[S][27][N] =
 * sum over nodes of w_rho rho + w_u . u + w_T T + w_P P + w_Y . Y differentiated with
 * respect to the populations (any weight array may be NULL: zero).  The state is
 * unchanged. */
uint32_t orc_ad_macros_vjp(orc_sim *s, const double *w_rho, const double *w_u, const double *w_T,
                           const double *w_P, const double *w_Y, double *lam) {
  const int64_t n = (int64_t)s->S * Q * s->N, N = s->N;
  const int M = s->p.M;
  start(s);
  std::vector<int32_t> in_id((size_t)n);
  for (int64_t k = 0; k < n; ++k) {
    s->pop[k] = ad::input(s->pop[k].v);
    in_id[(size_t)k] = s->pop[k].id;
  }
  std::vector<adouble> rho((size_t)N), u((size_t)3 * N), T((size_t)N), P((size_t)N), Y((size_t)M * N);
  const uint32_t anom = macros_fields(s, rho.data(), u.data(), T.data(), P.data(), Y.data());
  std::vector<double> adj((size_t)ad::tape().next_id(), 0.0);
  auto seed = [&](const std::vector<adouble> &f, const double *w) {
    if (!w) return;
    for (size_t k = 0; k < f.size(); ++k)
      if (f[k].id) adj[(size_t)f[k].id] += w[k];
  };
  seed(rho, w_rho);
  seed(u, w_u);
  seed(T, w_T);
  seed(P, w_P);
  seed(Y, w_Y);
  ad::reverse(adj);
  for (int64_t k = 0; k < n; ++k) lam[k] = adj[(size_t)in_id[(size_t)k]];
  settle(s);
  return anom;
}

/* Equilibrium initial state from the fields (as orc_init), recorded, then reversed:
 * g_rho[N], g_u[3][N], g_T[N], g_Y[M][N] = (d pop_0 / d field)^T lam0 (any output may be
 * NULL).  Leaves the initial state in the simulation. */
void orc_ad_init_vjp(orc_sim *s, const double *rho, const double *u, const double *T, const double *Y,
                     const double *lam0, double *g_rho, double *g_u, double *g_T, double *g_Y) {
  const int64_t n = (int64_t)s->S * Q * s->N, N = s->N;
  const int M = s->p.M;
  start(s);
  auto inputs = [&](const double *v, int64_t len) {
    std::vector<adouble> a((size_t)len);
    for (int64_t k = 0; k < len; ++k) a[(size_t)k] = ad::input(v[k]);
    return a;
  };
  std::vector<adouble> r = inputs(rho, N), uu = inputs(u, 3 * N), TT = inputs(T, N), YY = inputs(Y, M * N);
  init_fields(s, r.data(), uu.data(), TT.data(), YY.data());
  std::vector<double> adj((size_t)ad::tape().next_id(), 0.0);
  for (int64_t k = 0; k < n; ++k)
    if (s->pop[k].id) adj[(size_t)s->pop[k].id] += lam0[k];
  ad::reverse(adj);
  auto out = [&](const std::vector<adouble> &a, double *g) {
    if (!g) return;
    for (size_t k = 0; k < a.size(); ++k) g[k] = adj[(size_t)a[k].id];
  };
  out(r, g_rho);
  out(uu, g_u);
  out(TT, g_T);
  out(YY, g_Y);
  settle(s);
}

/* Entries recorded by the last reversed call (its tape length). */
int64_t orc_ad_tape_entries(void) { return last_entries; }

}  // extern "C"
