// Host-side planning of Leja interpolation for exp(-i tau H_hat) v.
//
// Section 3 of the paper approximates exp(A) v by the Newton form of the
// interpolation polynomial at Leja points, sum_i d_i prod_{j<i} (A - xi_j I) v,
// with divided differences d_i, a degree chosen so the error stays below a
// tolerance, early termination, and parameters that need an estimate of the
// spectrum.  The concrete choices made here (the reading of that section):
//
//  * H_hat is Hermitian with spectrum in [c - r, c + r] (Weyl combination of
//    per-term enclosures).  X = (2/r)(H_hat - c I) has spectrum in [-2, 2] and
//    exp(-i tau H_hat) = exp(-i tau c) exp(-i theta X), theta = tau r / 2.
//  * Real Leja points on [-2, 2]: xi_0 = 2, then greedy maximisers of the
//    product of distances (ties broken to the left).
//  * s substeps of theta/s and degree m chosen so that
//    s * sup_{[-2,2]} |exp(-i theta/s x) - p_m(x)| <= tol / 2 at least cost m s.
//    Because X is Hermitian (normal) that sup bounds the 2-norm error.
//  * Divided differences of exp(-i theta x) by the Taylor expansion
//    sum_n (-i theta)^n / n! x^n, whose monomials have divided differences
//    h_{n-k}(xi_0..xi_k) (complete homogeneous symmetric polynomials); summed
//    in long double with |theta| <= THETA_CAP so the relative accuracy of every
//    d_k is close to FP64 rounding.
#pragma once

#include <complex>
#include <cstdint>
#include <vector>

namespace magnus {

constexpr int kMaxDegree = 64;          // degree cap per substep
constexpr int kTail = 40;               // extra Newton terms used for error tails
constexpr int kNumPoints = kMaxDegree + kTail + 1;
constexpr double kThetaCap = 4.0;       // |theta| per substep handled by the d_k sum

// Leja points xi_0..xi_{kNumPoints-1} (computed once, thread-safe).
const std::vector<double>& leja_points();

// d_0..d_m of exp(-i theta x) at the Leja points, |theta| <= kThetaCap.
void divided_differences(double theta, int m, std::complex<double>* d);

// sup_{x in [-2,2]} |exp(-i theta x) - p_m(x)| from the Newton tail (grid sup).
double leja_error(double theta, int m);

struct LejaPlan {
  int m = 0;          // degree per substep
  int s = 1;          // substeps
  double bound = 0;   // s * err(theta/s, m) from the conservative table
};

// Plan for |theta| with caps; returns false if the caps cannot reach tol.
bool plan_degree(double theta, double tol, int max_degree, int max_substeps, LejaPlan* out);

// Smallest degree m <= max_degree with
//   s * (err(|theta|/s, m) + der_weight * derr(|theta|/s, m)) <= tol / 2
// for a given substep count s; returns -1 if none (or if |theta|/s > kThetaCap).
// derr is the sup over [-2, 2] of the derivative of exp(-i theta x) - p_m(x):
// for the block operator [[X, E], [0, X]] with Hermitian X its upper-right
// block carries D(f - p_m)(X)[E], which we bound by derr * |E| (der_weight = |E|).
int degree_for_substeps(double theta, double tol, int s, int max_degree, double* bound,
                        double der_weight = 0.0);

// sup over x in [-2, 2] of |d/dx (exp(-i theta x) - p_m(x))| (grid sup of the Newton tail).
double leja_derivative_error(double theta, int m);

// Weyl enclosure of a*[l1,u1] + b*[l2,u2] + k*[l3,u3].
void weyl_interval(double a, double l1, double u1, double b, double l2, double u2, double k,
                   double l3, double u3, double* lo, double* hi);

// Everything one exponential needs on the device.
struct ExpPlan {
  double c = 0, r = 0;         // centre, half-width of the enclosure
  double scale = 0;            // 2 / r
  double theta = 0;            // tau r / 2 (signed)
  double tau_sub = 0;          // tau / s
  LejaPlan lp;
  std::vector<std::complex<double>> d;   // d_0..d_m times exp(-i tau_sub c)
};

// tau: signed step of the exponential; [lo, hi] encloses spec(H_hat).
bool plan_exponential(double tau, double lo, double hi, double tol, int max_degree,
                      int max_substeps, ExpPlan* out);

// As plan_exponential with the substep count fixed to s (used when several
// states share one iteration sequence); false if no degree reaches tol.
// coupling_norm > 0 plans the block exponential of [[H, E], [0, H]] with
// |E| <= coupling_norm (error of the upper-right block included).
bool plan_exponential_fixed_s(double tau, double lo, double hi, double tol, int s, int max_degree,
                              ExpPlan* out, double coupling_norm = 0.0);

// Gauss nodes c_1, c_2 of Methods M4 / Cf4 and the Cf4 weights.
constexpr double kSqrt3 = 1.7320508075688772935;
constexpr double kC1 = 0.5 - kSqrt3 / 6.0;
constexpr double kC2 = 0.5 + kSqrt3 / 6.0;
constexpr double kAlpha1 = (3.0 - 2.0 * kSqrt3) / 12.0;
constexpr double kAlpha2 = (3.0 + 2.0 * kSqrt3) / 12.0;

// One step of a Magnus-type method for H(t) = H1 + f(t) H2, from the samples
// f_j = f(t_n + c_j tau), j < q.  Commutator-free methods (Cf4, Cf4:3) and
// the exponential midpoint rule (M2) are products of exponentials
// exp(-i tau (rho_k H1 + b_k H2)) with b_k = sum_j w[k][j] f_j, listed in the
// order they act on the state (the rightmost factor of Section 2 first).
// M4 has one exponential with the commutator term (commutator = true).
struct Scheme {
  int q = 0;
  int nexp = 0;
  bool commutator = false;  // M4, M6: one exponential with commutator terms
  bool sixth = false;       // M6 (its exponent is assembled from precomputed commutators)
  double c[3] = {0, 0, 0};
  double rho[3] = {0, 0, 0};
  double w[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
};

// Method ids as in the public header: 0 Cf4, 1 M4, 2 M2, 3 Cf4:3, 4 M6.
bool method_scheme(int method, Scheme* out);

// Smallest and largest eigenvalue of the symmetric tridiagonal matrix with
// diagonal a[0..k) and off-diagonal b[0..k-1) (Sturm-sequence bisection).
void tridiag_extremes(const std::vector<double>& a, const std::vector<double>& b, double* lo, double* hi);

}  // namespace magnus
