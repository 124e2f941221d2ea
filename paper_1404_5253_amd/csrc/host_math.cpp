// Host FP64 numerics of the WPCD pipeline: lattice, NN potentials in the WP basis, symmetric
// eigenproblem, recoupling coefficients and Wynn's epsilon table. These are the "negligible"
// step 1 of the paper's Sec. V.A and the scalar Pade step, kept on the CPU in FP64.
#include <algorithm>
#include <cmath>
#include <functional>
#include <map>
#include <queue>
#include <stdexcept>
#include <thread>
#include <tuple>
#include <vector>

#include "wpcd_internal.h"

namespace wpcd {

// ------------------------------------------------------------------ quadrature nodes

void gauss_legendre(int n, double* x, double* w) {
  // Roots of P_n by Newton's method from the Tricomi-type initial guess; weights
  // 2 / ((1 - x^2) P_n'(x)^2). Nodes ascending.
  for (int i = 0; i < (n + 1) / 2; ++i) {
    double z = std::cos(M_PI * (i + 0.75) / (n + 0.5));
    double pp = 0.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;
      if (n == 0) break;
      for (int k = 2; k <= n; ++k) {
        double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      double pn = (n == 1) ? z : p1;
      double pnm1 = (n == 1) ? 1.0 : p0;
      pp = n * (z * pn - pnm1) / (z * z - 1.0);
      double dz = pn / pp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) {
        // one more evaluation of the derivative at the converged root
        p0 = 1.0;
        p1 = z;
        for (int k = 2; k <= n; ++k) {
          double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
          p0 = p1;
          p1 = p2;
        }
        pn = (n == 1) ? z : p1;
        pnm1 = (n == 1) ? 1.0 : p0;
        pp = n * (z * pn - pnm1) / (z * z - 1.0);
        break;
      }
    }
    double wt = 2.0 / ((1.0 - z * z) * pp * pp);
    x[i] = -z;
    x[n - 1 - i] = z;
    w[i] = wt;
    w[n - 1 - i] = wt;
  }
  if (n % 2 == 1) x[n / 2] = 0.0;
}

// ------------------------------------------------------------------ lattice

std::vector<double> tangent_edges(int n, double alpha, double pmax) {
  // p_i = alpha tan(i theta_max / n), theta_max = atan(pmax / alpha): dense bins near 0.
  std::vector<double> e(n + 1);
  double th = std::atan(pmax / alpha);
  for (int i = 0; i <= n; ++i) e[i] = alpha * std::tan(i * th / n);
  e[0] = 0.0;
  e[n] = pmax;
  return e;
}

std::vector<double> h0_diagonal(const std::vector<double>& e, double h2m) {
  // <p_i | h2m p^2 | p_i> for unit-weight packets: (h2m / d_i) int_{D_i} p^2 dp.
  size_t M = e.size() - 1;
  std::vector<double> h(M);
  for (size_t i = 0; i < M; ++i) {
    double a = e[i], b = e[i + 1];
    h[i] = h2m * (a * a + a * b + b * b) / 3.0;
  }
  return h;
}

// ------------------------------------------------------------------ potentials

std::vector<double> yamaguchi_form(const std::vector<double>& e, double beta) {
  // G_i = d_i^{-1/2} int_{D_i} p / (p^2 + beta^2) dp; v_ii' = -lambda G_i G_i'.
  size_t M = e.size() - 1;
  std::vector<double> G(M);
  double b2 = beta * beta;
  for (size_t i = 0; i < M; ++i) {
    double a = e[i], b = e[i + 1];
    G[i] = 0.5 * std::log((b * b + b2) / (a * a + b2)) / std::sqrt(b - a);
  }
  return G;
}

static double legendre_q(int l, double z) {
  // Q_l(z), z > 1. For z >= 2 the hypergeometric series in 1/z^2; below, upward recurrence
  // from Q_0 = atanh(1/z), Q_1 = z Q_0 - 1.
  if (z < 2.0) {
    double q0 = 0.5 * std::log((z + 1.0) / (z - 1.0));
    if (l == 0) return q0;
    double qm = q0, qc = z * q0 - 1.0;
    for (int n = 1; n < l; ++n) {
      double qn = ((2.0 * n + 1.0) * z * qc - n * qm) / (n + 1.0);
      qm = qc;
      qc = qn;
    }
    return qc;
  }
  // sqrt(pi) l! / Gamma(l + 3/2) = l! / prod_{m=0}^{l} (m + 1/2)
  double pref = 1.0;
  for (int m = 1; m <= l; ++m) pref *= m;
  for (int m = 0; m <= l; ++m) pref /= (m + 0.5);
  double x = 1.0 / (z * z);
  double a = 0.5 * (l + 1), b = 0.5 * (l + 2), c = l + 1.5;
  double term = 1.0, sum = 1.0;
  for (int n = 0; n < 200; ++n) {
    term *= (a + n) * (b + n) / ((c + n) * (n + 1.0)) * x;
    sum += term;
    if (std::fabs(term) < 1e-18 * std::fabs(sum)) break;
  }
  return pref * sum / std::pow(2.0 * z, l + 1);
}

// Rows i = 0 .. M-1 on up to 16 host threads, interleaved (row i has M - i bin pairs); each row
// writes only its own pairs (i, k >= i) and their mirror images, so the rows do not race.
static void rows_parallel(size_t M, const std::function<void(size_t)>& row) {
  const unsigned hw = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  const size_t T = std::min<size_t>(hw, M);
  if (T <= 1) {
    for (size_t i = 0; i < M; ++i) row(i);
    return;
  }
  std::vector<std::thread> th;
  for (size_t t = 0; t < T; ++t)
    th.emplace_back([&, t] {
      for (size_t i = t; i < M; i += T) row(i);
    });
  for (auto& x : th) x.join();
}

std::vector<double> yukawa_wp(const std::vector<double>& e, int l, double mu) {
  // Unit-strength Yukawa e^{-mu r}/r in partial wave l, free WP basis:
  // v_ii' = (d_i d_i')^{-1/2} int int p p' v_l(p,p') dp dp',  p p' v_l = Q_l(z) / pi,
  // z = (p^2 + p'^2 + mu^2) / (2 p p').
  size_t M = e.size() - 1;
  std::vector<double> v(M * M);
  if (l == 0) {
    // closed form from the second antiderivative of ln(u^2 + mu^2)
    auto L2 = [mu](double u) {
      return 0.5 * (u * u - mu * mu) * std::log(u * u + mu * mu) - 1.5 * u * u + 2.0 * mu * u * std::atan(u / mu);
    };
    for (size_t i = 0; i < M; ++i)
      for (size_t k = 0; k < M; ++k) {
        double A = e[i], B = e[i + 1], C = e[k], D = e[k + 1];
        double plus = L2(B + D) - L2(B + C) - L2(A + D) + L2(A + C);
        double minus = L2(B - C) - L2(B - D) - L2(A - C) + L2(A - D);
        v[i * M + k] = (plus - minus) / (2.0 * M_PI) / std::sqrt((B - A) * (D - C));
      }
    return v;
  }
  const int ng = 32;
  double gx[ng], gw[ng];
  gauss_legendre(ng, gx, gw);
  std::vector<double> P(M * ng), W(M * ng);
  for (size_t i = 0; i < M; ++i) {
    double h = 0.5 * (e[i + 1] - e[i]), m = 0.5 * (e[i + 1] + e[i]);
    for (int a = 0; a < ng; ++a) {
      P[i * ng + a] = m + h * gx[a];
      W[i * ng + a] = h * gw[a];
    }
  }
  rows_parallel(M, [&](size_t i) {
    for (size_t k = i; k < M; ++k) {
      double s = 0.0;
      for (int a = 0; a < ng; ++a) {
        double p = P[i * ng + a];
        double acc = 0.0;
        for (int b = 0; b < ng; ++b) {
          double pp = P[k * ng + b];
          double z = (p * p + pp * pp + mu * mu) / (2.0 * p * pp);
          acc += W[k * ng + b] * legendre_q(l, z);
        }
        s += W[i * ng + a] * acc;
      }
      s /= M_PI * std::sqrt((e[i + 1] - e[i]) * (e[k + 1] - e[k]));
      v[i * M + k] = s;
      v[k * M + i] = s;
    }
  });
  return v;
}

// Energy-weight packets (weight w(p) = sqrt(2 h2m p), |w|^2 = d eps/dp; norm C_i = h2m dp2_i,
// dp2_i = p_i^2 - p_{i-1}^2; Sec. III.B, footnote). Integrals over a bin are taken in t = sqrt(p)
// (p = t^2, sqrt(p) dp = 2 t^2 dt), where the integrands are smooth at p = 0.

std::vector<double> h0_diagonal_energy(const std::vector<double>& e, double h2m) {
  // (1/C_i) int eps d eps over the bin: its mean energy
  size_t M = e.size() - 1;
  std::vector<double> h(M);
  for (size_t i = 0; i < M; ++i) h[i] = 0.5 * h2m * (e[i] * e[i] + e[i + 1] * e[i + 1]);
  return h;
}

static void sqrt_nodes(const std::vector<double>& e, int ng, std::vector<double>& P, std::vector<double>& W) {
  // per bin: nodes p = t^2 and weights of int sqrt(p) f(p) dp = int 2 t^2 f(t^2) dt
  std::vector<double> gx(ng), gw(ng);
  gauss_legendre(ng, gx.data(), gw.data());
  size_t M = e.size() - 1;
  P.assign(M * ng, 0.0);
  W.assign(M * ng, 0.0);
  for (size_t i = 0; i < M; ++i) {
    const double ta = std::sqrt(e[i]), tb = std::sqrt(e[i + 1]);
    const double h = 0.5 * (tb - ta), m = 0.5 * (tb + ta);
    for (int a = 0; a < ng; ++a) {
      const double t = m + h * gx[a];
      P[i * ng + a] = t * t;
      W[i * ng + a] = h * gw[a] * 2.0 * t * t;
    }
  }
}

std::vector<double> yamaguchi_form_energy(const std::vector<double>& e, double beta) {
  // G_i = C_i^{-1/2} int w(p) p / (p^2 + beta^2) dp = sqrt(2 / dp2_i) int p^{3/2} / (p^2 + beta^2) dp
  const int ng = 32;
  std::vector<double> P, W;
  sqrt_nodes(e, ng, P, W);
  size_t M = e.size() - 1;
  std::vector<double> G(M);
  for (size_t i = 0; i < M; ++i) {
    double s = 0.0;
    for (int a = 0; a < ng; ++a) {
      const double p = P[i * ng + a];
      s += W[i * ng + a] * p / (p * p + beta * beta);
    }
    G[i] = s * std::sqrt(2.0 / (e[i + 1] * e[i + 1] - e[i] * e[i]));
  }
  return G;
}

std::vector<double> yukawa_wp_energy(const std::vector<double>& e, int l, double mu) {
  // v_ii' = 2 (dp2_i dp2_i')^{-1/2} int int sqrt(p p') Q_l(z) / pi dp dp'
  const int ng = 32;
  std::vector<double> P, W;
  sqrt_nodes(e, ng, P, W);
  size_t M = e.size() - 1;
  std::vector<double> v(M * M);
  rows_parallel(M, [&](size_t i) {
    for (size_t k = i; k < M; ++k) {
      double s = 0.0;
      for (int a = 0; a < ng; ++a) {
        const double p = P[i * ng + a];
        double acc = 0.0;
        for (int b = 0; b < ng; ++b) {
          const double pp = P[k * ng + b];
          const double z = (p * p + pp * pp + mu * mu) / (2.0 * p * pp);
          acc += W[k * ng + b] * legendre_q(l, z);
        }
        s += W[i * ng + a] * acc;
      }
      const double d2i = e[i + 1] * e[i + 1] - e[i] * e[i], d2k = e[k + 1] * e[k + 1] - e[k] * e[k];
      s *= 2.0 / (M_PI * std::sqrt(d2i * d2k));
      v[i * M + k] = s;
      v[k * M + i] = s;
    }
  });
  return v;
}

// ------------------------------------------------------------------ symmetric eigenproblem

void sym_eigen(int n, std::vector<double>& A, std::vector<double>& d, std::vector<double>* Zout) {
  // Householder reduction to tridiagonal form T = Q^T A Q, then implicit QR steps with the
  // Wilkinson shift (bulge chasing with Givens rotations) accumulated into Q.
  const bool vec = Zout != nullptr;
  std::vector<double> Q;
  if (vec) {
    Q.assign((size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i) Q[(size_t)i * n + i] = 1.0;
  }
  std::vector<double> v(n), p(n), w(n);
  for (int k = 0; k + 2 < n; ++k) {
    int m = n - k - 1;  // length of x = A[k+1.., k]
    double alpha = 0.0;
    for (int r = 0; r < m; ++r) alpha += A[(size_t)(k + 1 + r) * n + k] * A[(size_t)(k + 1 + r) * n + k];
    alpha = std::sqrt(alpha);
    if (alpha == 0.0) continue;
    double x0 = A[(size_t)(k + 1) * n + k];
    double sgn = x0 >= 0.0 ? 1.0 : -1.0;
    for (int r = 0; r < m; ++r) v[r] = A[(size_t)(k + 1 + r) * n + k];
    v[0] += sgn * alpha;
    double vv = 0.0;
    for (int r = 0; r < m; ++r) vv += v[r] * v[r];
    if (vv == 0.0) continue;
    double beta = 2.0 / vv;
    // p = beta A22 v
    for (int r = 0; r < m; ++r) {
      double s = 0.0;
      const double* row = &A[(size_t)(k + 1 + r) * n + (k + 1)];
      for (int c = 0; c < m; ++c) s += row[c] * v[c];
      p[r] = beta * s;
    }
    double pv = 0.0;
    for (int r = 0; r < m; ++r) pv += p[r] * v[r];
    double K = 0.5 * beta * pv;
    for (int r = 0; r < m; ++r) w[r] = p[r] - K * v[r];
    for (int r = 0; r < m; ++r) {
      double* row = &A[(size_t)(k + 1 + r) * n + (k + 1)];
      for (int c = 0; c < m; ++c) row[c] -= v[r] * w[c] + w[r] * v[c];
    }
    A[(size_t)(k + 1) * n + k] = -sgn * alpha;
    A[(size_t)k * n + (k + 1)] = -sgn * alpha;
    for (int r = 1; r < m; ++r) {
      A[(size_t)(k + 1 + r) * n + k] = 0.0;
      A[(size_t)k * n + (k + 1 + r)] = 0.0;
    }
    if (vec) {
      // Q <- Q (I - beta v v^T) on columns k+1..n-1
      for (int r = 0; r < n; ++r) {
        double* row = &Q[(size_t)r * n + (k + 1)];
        double s = 0.0;
        for (int c = 0; c < m; ++c) s += row[c] * v[c];
        s *= beta;
        for (int c = 0; c < m; ++c) row[c] -= s * v[c];
      }
    }
  }
  d.assign(n, 0.0);
  std::vector<double> e(n, 0.0);
  for (int i = 0; i < n; ++i) d[i] = A[(size_t)i * n + i];
  for (int i = 0; i + 1 < n; ++i) e[i] = A[(size_t)(i + 1) * n + i];

  const double eps = 2.2e-16;
  int m = n - 1;
  int guard = 0;
  while (m > 0) {
    if (std::fabs(e[m - 1]) <= eps * (std::fabs(d[m - 1]) + std::fabs(d[m]))) {
      e[m - 1] = 0.0;
      --m;
      continue;
    }
    int l = m - 1;
    while (l > 0 && std::fabs(e[l - 1]) > eps * (std::fabs(d[l - 1]) + std::fabs(d[l]))) --l;
    if (++guard > 60 * n) throw std::runtime_error("symmetric eigensolver did not converge");
    // Wilkinson shift from the trailing 2x2 block
    double delta = 0.5 * (d[m - 1] - d[m]);
    double em = e[m - 1];
    double den = delta + (delta >= 0.0 ? 1.0 : -1.0) * std::hypot(delta, em);
    double mu = d[m] - em * em / den;
    double x = d[l] - mu, z = e[l];
    for (int k = l; k < m; ++k) {
      double r = std::hypot(x, z);
      double c = x / r, s = z / r;
      if (k > l) e[k - 1] = r;
      double a = d[k], b = e[k], cc = d[k + 1];
      d[k] = c * c * a + 2.0 * c * s * b + s * s * cc;
      d[k + 1] = s * s * a - 2.0 * c * s * b + c * c * cc;
      e[k] = c * s * (cc - a) + (c * c - s * s) * b;
      if (k + 1 < m) {
        x = e[k];
        z = s * e[k + 1];
        e[k + 1] = c * e[k + 1];
      }
      if (vec) {
        for (int r2 = 0; r2 < n; ++r2) {
          double qk = Q[(size_t)r2 * n + k], qk1 = Q[(size_t)r2 * n + k + 1];
          Q[(size_t)r2 * n + k] = c * qk + s * qk1;
          Q[(size_t)r2 * n + k + 1] = -s * qk + c * qk1;
        }
      }
    }
  }
  std::vector<int> idx(n);
  for (int i = 0; i < n; ++i) idx[i] = i;
  std::sort(idx.begin(), idx.end(), [&](int a, int b) { return d[a] < d[b]; });
  std::vector<double> ds(n);
  for (int i = 0; i < n; ++i) ds[i] = d[idx[i]];
  if (vec) {
    Zout->assign((size_t)n * n, 0.0);
    for (int r = 0; r < n; ++r)
      for (int i = 0; i < n; ++i) (*Zout)[(size_t)r * n + i] = Q[(size_t)i * n + idx[r]];
  }
  d = ds;
}

// ------------------------------------------------------------------ angular momentum algebra
// All arguments are doubled (2j) integers.

static long double fact(int n) {
  static std::vector<long double> f;
  if (f.empty()) {
    f.resize(171);
    f[0] = 1.0L;
    for (int i = 1; i < 171; ++i) f[i] = f[i - 1] * i;
  }
  return f.at(n);
}

static bool tri2(int a, int b, int c) {
  return c >= std::abs(a - b) && c <= a + b && ((a + b + c) % 2 == 0);
}

static long double delta2(int a, int b, int c) {
  return std::sqrt(fact((a + b - c) / 2) * fact((a - b + c) / 2) * fact((-a + b + c) / 2) / fact((a + b + c) / 2 + 1));
}

static double cg2(int j1, int m1, int j2, int m2, int J, int M) {
  // <j1 m1 j2 m2 | J M> by the Racah formula.
  if (m1 + m2 != M || !tri2(j1, j2, J)) return 0.0;
  if (std::abs(m1) > j1 || std::abs(m2) > j2 || std::abs(M) > J) return 0.0;
  if ((j1 + m1) % 2 || (j2 + m2) % 2 || (J + M) % 2) return 0.0;
  long double pre = std::sqrt((J + 1) * fact((J + j1 - j2) / 2) * fact((J - j1 + j2) / 2) * fact((j1 + j2 - J) / 2) /
                              fact((j1 + j2 + J) / 2 + 1));
  pre *= std::sqrt(fact((J + M) / 2) * fact((J - M) / 2) * fact((j1 - m1) / 2) * fact((j1 + m1) / 2) *
                   fact((j2 - m2) / 2) * fact((j2 + m2) / 2));
  long double s = 0.0L;
  for (int k = 0; k <= 200; ++k) {
    int a1 = (j1 + j2 - J) / 2 - k, a2 = (j1 - m1) / 2 - k, a3 = (j2 + m2) / 2 - k;
    int a4 = (J - j2 + m1) / 2 + k, a5 = (J - j1 - m2) / 2 + k;
    if (a1 < 0 || a2 < 0 || a3 < 0) break;
    if (a4 < 0 || a5 < 0) continue;
    long double t = 1.0L / (fact(k) * fact(a1) * fact(a2) * fact(a3) * fact(a4) * fact(a5));
    s += (k % 2 ? -t : t);
  }
  return (double)(pre * s);
}

double sixj2(int a, int b, int c, int d, int e, int f) {
  // {a b c; d e f} by the Racah formula.
  if (!tri2(a, b, c) || !tri2(a, e, f) || !tri2(d, b, f) || !tri2(d, e, c)) return 0.0;
  long double pre = delta2(a, b, c) * delta2(a, e, f) * delta2(d, b, f) * delta2(d, e, c);
  int t1 = (a + b + c) / 2, t2 = (a + e + f) / 2, t3 = (d + b + f) / 2, t4 = (d + e + c) / 2;
  int u1 = (a + b + d + e) / 2, u2 = (b + c + e + f) / 2, u3 = (c + a + f + d) / 2;
  int tmin = std::max(std::max(t1, t2), std::max(t3, t4));
  int tmax = std::min(u1, std::min(u2, u3));
  long double s = 0.0L;
  for (int t = tmin; t <= tmax; ++t) {
    long double v = fact(t + 1) / (fact(t - t1) * fact(t - t2) * fact(t - t3) * fact(t - t4) * fact(u1 - t) *
                                   fact(u2 - t) * fact(u3 - t));
    s += (t % 2 ? -v : v);
  }
  return (double)(pre * s);
}

static double ninej2(int j1, int j2, int j3, int j4, int j5, int j6, int j7, int j8, int j9) {
  // {j1 j2 j3; j4 j5 j6; j7 j8 j9} = sum_x (-1)^{2x} (2x+1) {j1 j4 j7; j8 j9 x}{j2 j5 j8; j4 x j6}{j3 j6 j9; x j1 j2}
  int xmin = std::max(std::max(std::abs(j1 - j9), std::abs(j4 - j8)), std::abs(j2 - j6));
  int xmax = std::min(std::min(j1 + j9, j4 + j8), j2 + j6);
  double s = 0.0;
  for (int x = xmin; x <= xmax; x += 2) {
    double v = sixj2(j1, j4, j7, j8, j9, x) * sixj2(j2, j5, j8, j4, x, j6) * sixj2(j3, j6, j9, x, j1, j2);
    s += (x % 2 ? -1.0 : 1.0) * (x + 1) * v;
  }
  return s;
}

std::vector<Chan> enumerate_channels(int two_J, int parity, int j_max, bool swave_only) {
  std::vector<Chan> out;
  for (int j = 0; j <= j_max; ++j)
    for (int s = 0; s <= 1; ++s)
      for (int l = std::abs(j - s); l <= j + s; ++l) {
        int t = (l + s + 1) % 2;
        for (int two_I = 1; two_I <= 2 * j + two_J + 1; two_I += 2) {
          if (!(std::abs(2 * j - two_I) <= two_J && two_J <= 2 * j + two_I)) continue;
          for (int lam : {(two_I - 1) / 2, (two_I + 1) / 2}) {
            if (((l + lam) % 2 == 0 ? 1 : -1) != parity) continue;
            if (swave_only && (l != 0 || lam != 0)) continue;
            out.push_back({l, s, j, lam, two_I, t});
          }
        }
      }
  std::sort(out.begin(), out.end(), [](const Chan& a, const Chan& b) {
    return std::make_tuple(a.j, a.l, a.s, a.lam, a.two_I) < std::make_tuple(b.j, b.l, b.s, b.lam, b.two_I);
  });
  out.erase(std::unique(out.begin(), out.end(),
                        [](const Chan& a, const Chan& b) {
                          return a.l == b.l && a.s == b.s && a.j == b.j && a.lam == b.lam && a.two_I == b.two_I;
                        }),
            out.end());
  return out;
}

std::vector<GTerm> g_table(const Chan& c, const Chan& cp, int two_J) {
  // Eq. gal with the factor (1/2)^{l2' + l1}; all angular momenta doubled internally.
  auto hat = [](int two_x) { return (double)(two_x + 1); };
  const int H = 1;  // 2 * (1/2)
  int l = 2 * c.l, s = 2 * c.s, j = 2 * c.j, lam = 2 * c.lam, I = c.two_I, t = 2 * c.t;
  int lp = 2 * cp.l, sp = 2 * cp.s, jp = 2 * cp.j, lamp = 2 * cp.lam, Ip = cp.two_I, tp = 2 * cp.t;
  int J = two_J, T = 1;
  double pref = -std::sqrt(hat(l) * hat(s) * hat(j) * hat(t) * hat(lam) * hat(I) * hat(lp) * hat(sp) * hat(jp) *
                           hat(tp) * hat(lamp) * hat(Ip));
  pref *= sixj2(H, H, tp, H, T, t);
  std::map<std::tuple<int, int, int>, double> acc;
  if (pref == 0.0) return {};
  auto fct = [](int n) { return (double)fact(n); };
  for (int L = 0; L <= 2 * std::max(c.l + c.lam, cp.l + cp.lam); L += 2) {
    if (!tri2(l, lam, L) || !tri2(lp, lamp, L)) continue;
    for (int S : {1, 3}) {
      double a = hat(L) * hat(S) * sixj2(H, H, sp, H, S, s);
      if (a == 0.0) continue;
      a *= ninej2(l, s, j, lam, H, I, L, S, J) * ninej2(lp, sp, jp, lamp, H, Ip, L, S, J);
      if (a == 0.0) continue;
      for (int l1 = 0; l1 <= c.l; ++l1) {
        int l2 = c.l - l1;
        for (int l1p = 0; l1p <= cp.l; ++l1p) {
          int l2p = cp.l - l1p;
          double cc = std::pow(0.5, l2p + l1) *
                      std::sqrt(fct(2 * c.l + 1) / (fct(2 * l1) * fct(2 * l2))) *
                      std::sqrt(fct(2 * cp.l + 1) / (fct(2 * l1p) * fct(2 * l2p)));
          int kmax = l1p + l2 + c.lam + cp.lam + L / 2 + 2;
          for (int k = 0; k <= kmax; ++k) {
            double sum = 0.0;
            for (int f = std::abs(l1 - c.lam); f <= l1 + c.lam; ++f) {
              double cf = cg2(2 * l1, 0, lam, 0, 2 * f, 0);
              if (cf == 0.0) continue;
              double ck = cg2(2 * k, 0, 2 * l1p, 0, 2 * f, 0);
              if (ck == 0.0) continue;
              double w6b = sixj2(2 * l2, 2 * l1, l, lam, L, 2 * f);
              if (w6b == 0.0) continue;
              for (int fp = std::abs(l2p - cp.lam); fp <= l2p + cp.lam; ++fp) {
                double cfp = cg2(2 * l2p, 0, lamp, 0, 2 * fp, 0);
                if (cfp == 0.0) continue;
                double ck2 = cg2(2 * k, 0, 2 * l2, 0, 2 * fp, 0);
                if (ck2 == 0.0) continue;
                sum += sixj2(2 * l1p, 2 * l2p, lp, lamp, L, 2 * fp) * w6b * cfp * cf *
                       sixj2(2 * fp, 2 * l1p, L, 2 * f, 2 * l2, 2 * k) * ck * ck2;
              }
            }
            if (sum != 0.0) acc[{l1, l1p, k}] += pref * a * (2 * k + 1) * cc * sum;
          }
        }
      }
    }
  }
  std::vector<GTerm> out;
  for (auto& kv : acc)
    if (std::fabs(kv.second) > 1e-15) out.push_back({std::get<0>(kv.first), std::get<1>(kv.first), std::get<2>(kv.first), kv.second});
  return out;
}

// ------------------------------------------------------------------ Wynn epsilon

cplx Wynn::push(cplx S) {
  // New anti-diagonal eps_k^{(n-k)}, k = 0..n, from the previous one:
  // eps_{k+1}^{(n-1-k)} = eps_{k-1}^{(n-k)} + 1 / (eps_k^{(n-k)} - eps_k^{(n-1-k)}).
  std::vector<cplx> nw;
  nw.reserve(diag.size() + 1);
  nw.push_back(S);
  for (size_t k = 0; k < diag.size(); ++k) {
    cplx d = nw[k] - diag[k];
    cplx inv = (std::abs(d) < 1e-300) ? cplx(1e300, 0.0) : 1.0 / d;
    cplx lower = k >= 1 ? diag[k - 1] : cplx(0.0, 0.0);
    nw.push_back(lower + inv);
  }
  diag.swap(nw);
  for (long k = (long)(diag.size() - 1) / 2 * 2; k >= 0; k -= 2)
    if (std::abs(diag[k]) < 1e200) return diag[k];
  return diag[0];
}

}  // namespace wpcd

namespace wpcd {

PackDesc make_pack(int nc, const std::vector<char>& nz) {
  // groups of channels with equal rows of the pattern (canonical order within a group)
  std::vector<std::vector<int>> groups;
  for (int g = 0; g < nc; ++g) {
    bool placed = false;
    for (auto& grp : groups) {
      const int h = grp[0];
      bool same = true;
      for (int gp = 0; gp < nc && same; ++gp) same = nz[g * nc + gp] == nz[h * nc + gp];
      if (same) {
        grp.push_back(g);
        placed = true;
        break;
      }
    }
    if (!placed) groups.push_back({g});
  }
  const int align = (nc % 2 == 0) ? 2 : 1;
  auto evaluate = [&](const std::vector<int>& perm, PackDesc* out) {
    PackDesc d;
    d.nc = nc;
    int total = 0;
    for (int u = 0; u < nc; ++u) {
      const int cu = perm[u];
      int lo = nc, hi = 0;
      for (int r = 0; r < nc; ++r)
        if (nz[perm[r] * nc + cu]) {
          lo = std::min(lo, r);
          hi = std::max(hi, r + 1);
        }
      if (hi <= lo) lo = hi = 0;   // an all-zero column stores nothing
      lo = lo / align * align;
      hi = std::min(nc, (hi + align - 1) / align * align);
      d.perm[u] = cu;
      d.lo[u] = lo;
      d.hi[u] = hi;
      d.off[u] = total;
      total += hi - lo;
    }
    d.npk = total;
    if (out) *out = d;
    return total;
  };
  std::vector<int> gorder(groups.size());
  for (size_t k = 0; k < gorder.size(); ++k) gorder[k] = (int)k;
  auto perm_of = [&](const std::vector<int>& go) {
    std::vector<int> perm;
    for (int k : go) perm.insert(perm.end(), groups[k].begin(), groups[k].end());
    return perm;
  };
  PackDesc best;
  int best_n = evaluate(perm_of(gorder), &best);
  if (groups.size() <= 8) {
    while (std::next_permutation(gorder.begin(), gorder.end())) {
      PackDesc d;
      const int n = evaluate(perm_of(gorder), &d);
      if (n < best_n) {
        best_n = n;
        best = d;
      }
    }
  }
  return best;
}

}  // namespace wpcd
