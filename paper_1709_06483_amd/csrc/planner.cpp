// Host planning of Leja interpolation (see planner.h for the readings).
#include "planner.h"

#include <algorithm>
#include <cmath>
#include <limits>
#include <mutex>

namespace magnus {
namespace {

// ---------------------------------------------------------------------------
// Leja points of [-2, 2]
// ---------------------------------------------------------------------------
double log_prod(double x, const std::vector<double>& pts, size_t k) {
  double s = 0.0;
  for (size_t j = 0; j < k; ++j) s += std::log(std::fabs(x - pts[j]));
  return s;
}

// Maximise sum_j log|x - xi_j| near x0 by Newton's method on its derivative,
// staying inside [lo, hi].
double refine_max(double x0, double lo, double hi, const std::vector<double>& pts) {
  double x = x0;
  for (int it = 0; it < 60; ++it) {
    double g = 0.0, h = 0.0;
    for (double p : pts) {
      const double r = 1.0 / (x - p);
      g += r;
      h -= r * r;
    }
    if (h >= 0.0) break;
    double xn = x - g / h;
    if (!(xn > lo && xn < hi)) break;
    if (std::fabs(xn - x) <= 1e-16 * std::max(1.0, std::fabs(x))) { x = xn; break; }
    x = xn;
  }
  return x;
}

std::vector<double> compute_leja_points() {
  const int G = 40001;
  std::vector<double> xs(G), lp(G);
  for (int g = 0; g < G; ++g) xs[g] = -2.0 + 4.0 * g / (G - 1);
  std::vector<double> pts;
  pts.reserve(kNumPoints);
  pts.push_back(2.0);
  for (int g = 0; g < G; ++g) lp[g] = std::log(std::fabs(xs[g] - 2.0));
  const double h = 4.0 / (G - 1);
  for (int k = 1; k < kNumPoints; ++k) {
    double best = -std::numeric_limits<double>::infinity();
    for (int g = 0; g < G; ++g) best = std::max(best, lp[g]);
    // every grid local maximum close to the best is refined; the largest
    // refined value wins, ties (to 1e-13 relative) going to the leftmost
    const double near = 1e-4 * std::max(1.0, std::fabs(best));
    double bx = 0.0, bv = -std::numeric_limits<double>::infinity();
    for (int g = 0; g < G; ++g) {
      if (lp[g] < best - near) continue;
      const bool left_ok = (g == 0) || lp[g] >= lp[g - 1];
      const bool right_ok = (g == G - 1) || lp[g] >= lp[g + 1];
      if (!(left_ok && right_ok)) continue;
      double x = xs[g];
      if (g != 0 && g != G - 1) x = refine_max(xs[g], xs[g] - h, xs[g] + h, pts);
      const double v = log_prod(x, pts, pts.size());
      if (v > bv + 1e-13 * std::max(1.0, std::fabs(v))) { bv = v; bx = x; }
    }
    if (std::fabs(bx) < 1e-15) bx = 0.0;
    pts.push_back(bx);
    for (int g = 0; g < G; ++g) lp[g] += std::log(std::fabs(xs[g] - bx));
  }
  return pts;
}

// ---------------------------------------------------------------------------
// h_j(xi_0..xi_k): complete homogeneous symmetric polynomials, the divided
// differences of x^(j+k) at xi_0..xi_k.
// ---------------------------------------------------------------------------
constexpr int kTaylorTerms = 64;

struct HTable {
  std::vector<long double> h;  // [k][j], k < kNumPoints, j <= kTaylorTerms
  long double at(int k, int j) const { return h[(size_t)k * (kTaylorTerms + 1) + j]; }
};

HTable compute_h_table(const std::vector<double>& xi) {
  HTable t;
  t.h.assign((size_t)kNumPoints * (kTaylorTerms + 1), 0.0L);
  auto H = [&](int k, int j) -> long double& { return t.h[(size_t)k * (kTaylorTerms + 1) + j]; };
  for (int j = 0; j <= kTaylorTerms; ++j) H(0, j) = (j == 0) ? 1.0L : H(0, j - 1) * (long double)xi[0];
  for (int k = 1; k < kNumPoints; ++k) {
    H(k, 0) = 1.0L;
    for (int j = 1; j <= kTaylorTerms; ++j) H(k, j) = H(k - 1, j) + (long double)xi[k] * H(k, j - 1);
  }
  return t;
}

// ---------------------------------------------------------------------------
// Error table: eps_m(theta) on a geometric theta grid, running max over theta.
// ---------------------------------------------------------------------------
constexpr double kThetaMin = 1e-6;
constexpr double kThetaRatio = 1.02;
constexpr int kXGrid = 2001;

struct Tables {
  std::vector<double> xi;
  HTable H;
  std::vector<double> basis;      // [k][x]: prod_{j<k} (x - xi_j) on the x grid
  std::vector<double> basis_max;  // [k]: max_x |basis[k][x]|
  std::vector<double> basis_der;  // [k][x]: d/dx prod_{j<k} (x - xi_j)
  std::vector<double> thetas;     // grid
  std::vector<double> epsmax;     // [g][m], running max over theta_g' <= theta_g
  std::vector<double> epsder;     // [g][m], same for the derivative of the error
};

void dd_long(const Tables& T, double theta, int m, std::complex<long double>* d) {
  // c_n = (-i theta)^n / n!, n = 0..m + kTaylorTerms
  const int nmax = m + kTaylorTerms;
  std::vector<std::complex<long double>> c(nmax + 1);
  c[0] = 1.0L;
  const std::complex<long double> mit(0.0L, -(long double)theta);
  for (int n = 1; n <= nmax; ++n) c[n] = c[n - 1] * mit / (long double)n;
  for (int k = 0; k <= m; ++k) {
    std::complex<long double> acc = 0.0L;
    // sum small terms first
    for (int j = kTaylorTerms; j >= 0; --j) acc += c[k + j] * T.H.at(k, j);
    d[k] = acc;
  }
}

double tail_error(const Tables& T, double theta, int m, std::vector<double>* eps_all,
                  std::vector<double>* der_all = nullptr) {
  // eps_all[m'] (and der_all[m'], the sup of the derivative of the error) for
  // every m' <= kMaxDegree when requested
  const int K = kNumPoints - 1;
  std::vector<std::complex<long double>> dl(K + 1);
  dd_long(T, theta, K, dl.data());
  std::vector<double> tr(kXGrid, 0.0), ti(kXGrid, 0.0), ur(kXGrid, 0.0), ui(kXGrid, 0.0);
  if (der_all) der_all->assign(kMaxDegree + 1, 0.0);
  double result = 0.0;
  if (eps_all) eps_all->assign(kMaxDegree + 1, 0.0);
  // terms whose size is far below any representable error contribute nothing
  int ktop = K;
  while (ktop > 1 && std::abs(dl[ktop]) * (long double)T.basis_max[ktop] < 1e-40L) --ktop;
  for (int k = ktop; k >= 1; --k) {
    const double dr = (double)dl[k].real(), di = (double)dl[k].imag();
    const double* b = &T.basis[(size_t)k * kXGrid];
    double mx = 0.0;
    for (int x = 0; x < kXGrid; ++x) {
      tr[x] += dr * b[x];
      ti[x] += di * b[x];
      const double a = tr[x] * tr[x] + ti[x] * ti[x];
      if (a > mx) mx = a;
    }
    const int mm = k - 1;  // the tail k..K is the error of degree k-1
    if (mm == m) result = std::sqrt(mx);
    if (eps_all && mm <= kMaxDegree) (*eps_all)[mm] = std::sqrt(mx);
    if (der_all) {
      const double* bd = &T.basis_der[(size_t)k * kXGrid];
      double md = 0.0;
      for (int x = 0; x < kXGrid; ++x) {
        ur[x] += dr * bd[x];
        ui[x] += di * bd[x];
        md = std::max(md, ur[x] * ur[x] + ui[x] * ui[x]);
      }
      if (mm <= kMaxDegree) (*der_all)[mm] = std::sqrt(md);
    }
  }
  return result;
}

Tables* build_tables() {
  Tables* T = new Tables();
  T->xi = compute_leja_points();
  T->H = compute_h_table(T->xi);
  T->basis.assign((size_t)kNumPoints * kXGrid, 0.0);
  for (int x = 0; x < kXGrid; ++x) {
    const double xv = -2.0 + 4.0 * x / (kXGrid - 1);
    double p = 1.0;
    for (int k = 0; k < kNumPoints; ++k) {
      T->basis[(size_t)k * kXGrid + x] = p;
      p *= (xv - T->xi[k]);
    }
  }
  T->basis_der.assign((size_t)kNumPoints * kXGrid, 0.0);
  for (int x = 0; x < kXGrid; ++x) {
    const double xv = -2.0 + 4.0 * x / (kXGrid - 1);
    // (P_{k+1})' = (P_k)' (x - xi_k) + P_k
    for (int k = 0; k + 1 < kNumPoints; ++k)
      T->basis_der[(size_t)(k + 1) * kXGrid + x] =
          T->basis_der[(size_t)k * kXGrid + x] * (xv - T->xi[k]) + T->basis[(size_t)k * kXGrid + x];
  }
  T->basis_max.assign(kNumPoints, 0.0);
  for (int k = 0; k < kNumPoints; ++k)
    for (int x = 0; x < kXGrid; ++x)
      T->basis_max[k] = std::max(T->basis_max[k], std::fabs(T->basis[(size_t)k * kXGrid + x]));
  for (double th = kThetaMin; th < kThetaCap * kThetaRatio; th *= kThetaRatio)
    T->thetas.push_back(std::min(th, kThetaCap));
  if (T->thetas.back() < kThetaCap) T->thetas.push_back(kThetaCap);
  const size_t G = T->thetas.size();
  T->epsmax.assign(G * (kMaxDegree + 1), 0.0);
  T->epsder.assign(G * (kMaxDegree + 1), 0.0);
  std::vector<double> e, ed;
  for (size_t g = 0; g < G; ++g) {
    tail_error(*T, T->thetas[g], -1, &e, &ed);
    for (int m = 0; m <= kMaxDegree; ++m) {
      double v = e[m], w = ed[m];
      if (g > 0) {
        v = std::max(v, T->epsmax[(g - 1) * (kMaxDegree + 1) + m]);
        w = std::max(w, T->epsder[(g - 1) * (kMaxDegree + 1) + m]);
      }
      T->epsmax[g * (kMaxDegree + 1) + m] = v;
      T->epsder[g * (kMaxDegree + 1) + m] = w;
    }
  }
  return T;
}

const Tables& tables() {
  static std::once_flag once;
  static Tables* T = nullptr;
  std::call_once(once, [] { T = build_tables(); });
  return *T;
}

}  // namespace

const std::vector<double>& leja_points() { return tables().xi; }

void divided_differences(double theta, int m, std::complex<double>* d) {
  const Tables& T = tables();
  std::vector<std::complex<long double>> dl(m + 1);
  dd_long(T, theta, m, dl.data());
  for (int k = 0; k <= m; ++k) d[k] = std::complex<double>((double)dl[k].real(), (double)dl[k].imag());
}

double leja_error(double theta, int m) {
  if (m < 0 || m > kMaxDegree) return std::numeric_limits<double>::infinity();
  return tail_error(tables(), std::fabs(theta), m, nullptr);
}

bool plan_degree(double theta, double tol, int max_degree, int max_substeps, LejaPlan* out) {
  const Tables& T = tables();
  theta = std::fabs(theta);
  max_degree = std::min(max_degree, kMaxDegree);
  if (theta == 0.0) { *out = LejaPlan{1, 1, 0.0}; return true; }
  const int s_min = std::max(1, (int)std::ceil(theta / kThetaCap - 1e-12));
  bool found = false;
  LejaPlan best;
  long best_cost = 0;
  for (int s = s_min; s <= std::min(max_substeps, s_min + 8); ++s) {
    const double ths = theta / s;
    // smallest grid theta >= ths
    size_t g = std::lower_bound(T.thetas.begin(), T.thetas.end(), ths * (1.0 - 1e-13)) - T.thetas.begin();
    if (g >= T.thetas.size()) continue;
    const double target = tol / (2.0 * s);
    for (int m = 1; m <= max_degree; ++m) {
      const double e = T.epsmax[g * (kMaxDegree + 1) + m];
      if (e <= target) {
        const long cost = (long)m * s;
        if (!found || cost < best_cost) {
          found = true;
          best_cost = cost;
          best = LejaPlan{m, s, s * e};
        }
        break;
      }
    }
  }
  if (found) *out = best;
  return found;
}

int degree_for_substeps(double theta, double tol, int s, int max_degree, double* bound, double der_weight) {
  const Tables& T = tables();
  theta = std::fabs(theta);
  max_degree = std::min(max_degree, kMaxDegree);
  if (s < 1) return -1;
  if (theta == 0.0) { if (bound) *bound = 0.0; return 1; }
  const double ths = theta / s;
  if (ths > kThetaCap * (1.0 + 1e-12)) return -1;
  size_t g = std::lower_bound(T.thetas.begin(), T.thetas.end(), ths * (1.0 - 1e-13)) - T.thetas.begin();
  if (g >= T.thetas.size()) g = T.thetas.size() - 1;
  const double target = tol / (2.0 * s);
  for (int m = 1; m <= max_degree; ++m) {
    const double e = T.epsmax[g * (kMaxDegree + 1) + m] + der_weight * T.epsder[g * (kMaxDegree + 1) + m];
    if (e <= target) {
      if (bound) *bound = s * e;
      return m;
    }
  }
  return -1;
}

double leja_derivative_error(double theta, int m) {
  if (m < 0 || m > kMaxDegree) return std::numeric_limits<double>::infinity();
  std::vector<double> e, ed;
  tail_error(tables(), std::fabs(theta), -1, &e, &ed);
  return ed[m];
}

void weyl_interval(double a, double l1, double u1, double b, double l2, double u2, double k,
                   double l3, double u3, double* lo, double* hi) {
  auto lo_of = [](double c, double l, double u) { return c >= 0 ? c * l : c * u; };
  auto hi_of = [](double c, double l, double u) { return c >= 0 ? c * u : c * l; };
  *lo = lo_of(a, l1, u1) + lo_of(b, l2, u2) + (k != 0.0 ? lo_of(k, l3, u3) : 0.0);
  *hi = hi_of(a, l1, u1) + hi_of(b, l2, u2) + (k != 0.0 ? hi_of(k, l3, u3) : 0.0);
}

namespace {
void finish_plan(double tau, ExpPlan* p) {
  p->tau_sub = tau / p->lp.s;
  const double theta_s = p->theta / p->lp.s;
  std::vector<std::complex<double>> d(p->lp.m + 1);
  divided_differences(theta_s, p->lp.m, d.data());
  const std::complex<double> phase = std::polar(1.0, -p->tau_sub * p->c);
  p->d.resize(p->lp.m + 1);
  for (int k = 0; k <= p->lp.m; ++k) p->d[k] = phase * d[k];
}

void centre_and_radius(double tau, double lo, double hi, ExpPlan* p) {
  p->c = 0.5 * (lo + hi);
  // widening an enclosure is always safe; keep r away from zero
  p->r = std::max(0.5 * (hi - lo), 1e-8 * std::max(1.0, std::fabs(p->c)));
  p->scale = 2.0 / p->r;
  p->theta = 0.5 * tau * p->r;
}
}  // namespace

bool plan_exponential_fixed_s(double tau, double lo, double hi, double tol, int s, int max_degree,
                              ExpPlan* out, double coupling_norm) {
  ExpPlan p;
  centre_and_radius(tau, lo, hi, &p);
  double bound = 0.0;
  const int m = degree_for_substeps(p.theta, tol, s, max_degree, &bound, p.scale * coupling_norm);
  if (m < 0) return false;
  p.lp = LejaPlan{m, s, bound};
  finish_plan(tau, &p);
  *out = std::move(p);
  return true;
}

bool plan_exponential(double tau, double lo, double hi, double tol, int max_degree,
                      int max_substeps, ExpPlan* out) {
  ExpPlan p;
  centre_and_radius(tau, lo, hi, &p);
  if (!plan_degree(p.theta, tol, max_degree, max_substeps, &p.lp)) return false;
  finish_plan(tau, &p);
  *out = std::move(p);
  return true;
}

bool method_scheme(int method, Scheme* out) {
  Scheme S;
  switch (method) {
    case 0: {  // Cf4: exp(tau(a1 A1 + a2 A2)) exp(tau(a2 A1 + a1 A2)), the second factor acting first
      S.q = 2;
      S.nexp = 2;
      S.c[0] = kC1;
      S.c[1] = kC2;
      S.rho[0] = S.rho[1] = 0.5;
      S.w[0][0] = kAlpha2;
      S.w[0][1] = kAlpha1;
      S.w[1][0] = kAlpha1;
      S.w[1][1] = kAlpha2;
      break;
    }
    case 1: {  // M4: one exponential with the averaged field and the commutator
      S.q = 2;
      S.nexp = 1;
      S.commutator = true;
      S.c[0] = kC1;
      S.c[1] = kC2;
      S.rho[0] = 1.0;
      S.w[0][0] = S.w[0][1] = 0.5;
      break;
    }
    case 2: {  // M2: exponential midpoint rule
      S.q = 1;
      S.nexp = 1;
      S.c[0] = 0.5;
      S.rho[0] = 1.0;
      S.w[0][0] = 1.0;
      break;
    }
    case 3: {  // Cf4:3 on the three Gauss nodes; rows of the printed alpha matrix, last row first
      const double r15 = 3.8729833462074168852;  // sqrt(15)
      const double p = 37.0 / 240.0, q = 10.0 * r15 / 261.0;
      const double rows[3][3] = {{p - q, -1.0 / 30.0, p + q},
                                 {-11.0 / 360.0, 23.0 / 45.0, -11.0 / 360.0},
                                 {p + q, -1.0 / 30.0, p - q}};
      S.q = 3;
      S.nexp = 3;
      S.c[0] = 0.5 - r15 / 10.0;
      S.c[1] = 0.5;
      S.c[2] = 0.5 + r15 / 10.0;
      for (int k = 0; k < 3; ++k) {
        const double* row = rows[2 - k];
        S.rho[k] = row[0] + row[1] + row[2];  // A_j = -i(H1 + f_j H2)
        for (int j = 0; j < 3; ++j) S.w[k][j] = row[j];
      }
      break;
    }
    case 4: {  // M6 on the three Gauss nodes (one exponential; coefficients built by the caller)
      const double r15 = 3.8729833462074168852;
      S.q = 3;
      S.nexp = 1;
      S.commutator = true;
      S.sixth = true;
      S.c[0] = 0.5 - r15 / 10.0;
      S.c[1] = 0.5;
      S.c[2] = 0.5 + r15 / 10.0;
      break;
    }
    default:
      return false;
  }
  *out = S;
  return true;
}

namespace {
// Eigenvalues of the tridiagonal matrix below x (signs of the LDL^T pivots).
int sturm_count(const std::vector<double>& a, const std::vector<double>& b, double x) {
  int count = 0;
  double q = 1.0;
  for (size_t i = 0; i < a.size(); ++i) {
    const double off = i ? b[i - 1] * b[i - 1] : 0.0;
    q = a[i] - x - (i ? off / q : 0.0);
    if (q == 0.0) q = -1e-300;
    if (q < 0.0) ++count;
  }
  return count;
}
}  // namespace

void tridiag_extremes(const std::vector<double>& a, const std::vector<double>& b, double* lo, double* hi) {
  const size_t k = a.size();
  double g_lo = INFINITY, g_hi = -INFINITY;  // Gershgorin interval of the tridiagonal
  for (size_t i = 0; i < k; ++i) {
    const double r = (i ? std::fabs(b[i - 1]) : 0.0) + (i + 1 < k ? std::fabs(b[i]) : 0.0);
    g_lo = std::min(g_lo, a[i] - r);
    g_hi = std::max(g_hi, a[i] + r);
  }
  auto bisect = [&](int target) {  // smallest x with count(x) >= target
    double l = g_lo - 1.0, h = g_hi + 1.0;
    for (int it = 0; it < 200 && h - l > 1e-15 * std::max(1.0, std::fabs(h)); ++it) {
      const double m = 0.5 * (l + h);
      if (sturm_count(a, b, m) >= target) h = m;
      else l = m;
    }
    return h;
  };
  *lo = bisect(1);
  *hi = bisect((int)k);
}

}  // namespace magnus
