// Elastic nd observables from the S matrices of several J^pi blocks (Sec. IV): the transformation
// of a block's S from the representation of the third nucleon's total angular momentum I to the
// channel-spin (Sigma) representation, eigenphases, and the differential cross section and the
// neutron vector analysing power summed over the blocks. Host FP64; the S matrices come from the
// solves (amplitude()).
//
// Conventions. A channel couples J = j (x) I, I = lam (x) 1/2 (the deuteron j = 1 as pair state).
// The transformation printed in Sec. IV, T[(lam, Sigma), (lam, I)] = sqrt((2I+1)(2Sigma+1))
// (-1)^(J-I) {lam 1/2 I; j J Sigma}, is the overlap with the channel-spin states
// |Sigma nu, lam m; J M> = sum <Sigma nu lam m | J M> <j m_d 1/2 sigma | Sigma nu> |m_d>|sigma>|lam m>,
// and the amplitude below is written in that basis. For a beam along z and the outgoing
// direction (theta, phi = 0):
//   M[(Sigma' nu'), (Sigma nu)] = (sqrt(pi) / (i k)) sum sqrt(2 lam + 1) <Sigma nu lam 0 | J nu>
//       <Sigma' nu' lam' (nu - nu') | J nu> (S - 1)^J[(lam' Sigma'), (lam Sigma)] Y_lam'^(nu - nu')(theta, 0),
// dsigma/dOmega = Tr(M M^+) / 6 and A_y = Tr(M sigma_y(n) M^+) / Tr(M M^+), with sigma_y acting on
// the incoming neutron's spin and y along k_in x k_out.
#include <algorithm>
#include <cmath>
#include <complex>
#include <vector>

#include "wpcd_objects.h"

using wpcd::cplx;
using wpcd::fail;

namespace {

long double lfact(int n) {
  long double r = 1.0L;
  for (int i = 2; i <= n; ++i) r *= i;
  return r;
}

// Clebsch-Gordan <j1 m1 j2 m2 | J M> with doubled arguments (Racah's closed form).
double cg2(int j1, int m1, int j2, int m2, int J, int M) {
  if (m1 + m2 != M || std::abs(m1) > j1 || std::abs(m2) > j2 || std::abs(M) > J) return 0.0;
  if (J < std::abs(j1 - j2) || J > j1 + j2 || ((j1 + j2 + J) & 1)) return 0.0;
  if (((j1 + m1) & 1) || ((j2 + m2) & 1) || ((J + M) & 1)) return 0.0;
  const int a = (j1 + j2 - J) / 2, b = (j1 - j2 + J) / 2, c = (-j1 + j2 + J) / 2;
  long double pre = (J + 1) * lfact(a) * lfact(b) * lfact(c) / lfact((j1 + j2 + J) / 2 + 1);
  pre *= lfact((j1 + m1) / 2) * lfact((j1 - m1) / 2) * lfact((j2 + m2) / 2) * lfact((j2 - m2) / 2) *
         lfact((J + M) / 2) * lfact((J - M) / 2);
  long double s = 0.0L;
  for (int k = 0; k <= a; ++k) {
    const int d1 = (j1 - m1) / 2 - k, d2 = (j2 + m2) / 2 - k, d3 = (J - j2 + m1) / 2 + k,
              d4 = (J - j1 - m2) / 2 + k;
    const int e1 = a - k;
    if (d1 < 0 || d2 < 0 || d3 < 0 || d4 < 0 || e1 < 0) continue;
    const long double t = 1.0L / (lfact(k) * lfact(e1) * lfact(d1) * lfact(d2) * lfact(d3) * lfact(d4));
    s += (k & 1) ? -t : t;
  }
  return (double)(std::sqrt(pre) * s);
}

// Y_l^m(theta, 0) with the Condon-Shortley phase (real at phi = 0).
double ylm0(int l, int m, double theta) {
  const int am = std::abs(m);
  if (am > l) return 0.0;
  const double x = std::cos(theta), sx = std::sin(theta);
  // P_am^am = (-1)^am (2am - 1)!! sin^am, then upward in l
  double pmm = 1.0;
  for (int i = 1; i <= am; ++i) pmm *= -(2.0 * i - 1.0) * sx;
  double p = pmm;
  if (l > am) {
    double pm1 = x * (2.0 * am + 1.0) * pmm;
    double pm0 = pmm;
    for (int ll = am + 2; ll <= l; ++ll) {
      const double pn = ((2.0 * ll - 1.0) * x * pm1 - (ll + am - 1.0) * pm0) / (ll - am);
      pm0 = pm1;
      pm1 = pn;
    }
    p = pm1;
  }
  long double ratio = lfact(l - am) / lfact(l + am);
  double y = std::sqrt((2.0 * l + 1.0) / (4.0 * M_PI) * (double)ratio) * p;
  if (m < 0 && (am & 1)) y = -y;   // Y_l^-m = (-1)^m conj(Y_l^m)
  return y;
}

// The channel-spin channels (lam, 2 Sigma) of a block's open channels: for every lam present (in
// ascending order) the Sigma in {1/2, 3/2} with |lam - Sigma| <= J <= lam + Sigma.
void sigma_channels(int two_J, int n, const int* lam, std::vector<int>& ls, std::vector<int>& ts) {
  std::vector<int> lams(lam, lam + n);
  std::sort(lams.begin(), lams.end());
  lams.erase(std::unique(lams.begin(), lams.end()), lams.end());
  ls.clear();
  ts.clear();
  for (int l : lams)
    for (int two_S : {1, 3})
      if (std::abs(2 * l - two_S) <= two_J && two_J <= 2 * l + two_S) {
        ls.push_back(l);
        ts.push_back(two_S);
      }
}

wp_status sigma_rep(int two_J, int n, const int* lam, const int* two_I, const cplx* S, std::vector<int>& ls,
                    std::vector<int>& ts, std::vector<cplx>& Ss) {
  for (int b = 0; b < n; ++b) {   // (lam, I) must be an open channel of J: I = lam +- 1/2, |I - j| <= J <= I + j
    if (lam[b] < 0 || std::abs(2 * lam[b] - two_I[b]) != 1 || two_J < std::abs(two_I[b] - 2) || two_J > two_I[b] + 2)
      return fail(WP_EINVAL, "nd_sigma_rep: (lam, I) is not an open channel of this J");
    for (int c = 0; c < b; ++c)
      if (lam[c] == lam[b] && two_I[c] == two_I[b]) return fail(WP_EINVAL, "nd_sigma_rep: repeated channel");
  }
  sigma_channels(two_J, n, lam, ls, ts);
  if ((int)ls.size() != n) return fail(WP_EINVAL, "nd_sigma_rep: the open channels do not span whole lam shells");
  std::vector<double> T((size_t)n * n, 0.0);
  for (int a = 0; a < n; ++a)
    for (int b = 0; b < n; ++b) {
      if (ls[a] != lam[b]) continue;
      const int tI = two_I[b], tS = ts[a];
      const int ph = ((two_J - tI) / 2) & 1;
      T[(size_t)a * n + b] = std::sqrt((tI + 1.0) * (tS + 1.0)) * (ph ? -1.0 : 1.0) *
                             wpcd::sixj2(2 * lam[b], 1, tI, 2, two_J, tS);
    }
  Ss.assign((size_t)n * n, cplx(0, 0));
  for (int a = 0; a < n; ++a)
    for (int b = 0; b < n; ++b) {
      cplx s = 0.0;
      for (int c = 0; c < n; ++c)
        for (int d = 0; d < n; ++d) s += T[(size_t)a * n + c] * S[(size_t)c * n + d] * T[(size_t)b * n + d];
      Ss[(size_t)a * n + b] = s;
    }
  return WP_OK;
}

}  // namespace

extern "C" wp_status nd_sigma_rep(int two_J, int n, const int* lam, const int* two_I, const double* S, int* lam_s,
                                  int* two_Sigma, double* S_sigma) {
  if (n < 1 || n > 8 || !lam || !two_I || !S || two_J < 1 || !(two_J & 1)) return fail(WP_EINVAL, "nd_sigma_rep: bad argument");
  std::vector<int> ls, ts;
  std::vector<cplx> Ss;
  if (wp_status st = sigma_rep(two_J, n, lam, two_I, reinterpret_cast<const cplx*>(S), ls, ts, Ss)) return st;
  for (int a = 0; a < n; ++a) {
    if (lam_s) lam_s[a] = ls[a];
    if (two_Sigma) two_Sigma[a] = ts[a];
  }
  if (S_sigma)
    for (int e = 0; e < n * n; ++e) {
      S_sigma[2 * e] = Ss[e].real();
      S_sigma[2 * e + 1] = Ss[e].imag();
    }
  return WP_OK;
}

extern "C" wp_status nd_eigenphases(int n, const double* S, double* delta, double* O) {
  if (n < 1 || n > 8 || !S) return fail(WP_EINVAL, "nd_eigenphases: bad argument");
  const cplx* Sc = reinterpret_cast<const cplx*>(S);
  // O diagonalises the commuting real symmetric parts of S = O diag(exp(2 i delta)) O^T; one
  // generic combination of them has the same eigenvectors
  const double a = 0.6180339887498949;
  std::vector<double> A((size_t)n * n), d, Z;
  for (int i = 0; i < n * n; ++i) A[i] = Sc[i].real() + a * Sc[i].imag();
  wpcd::sym_eigen(n, A, d, &Z);   // rows of Z: eigenvectors
  for (int k = 0; k < n; ++k) {   // each eigenvector's largest component positive
    double* z = Z.data() + (size_t)k * n;
    int im = 0;
    for (int i = 1; i < n; ++i)
      if (std::fabs(z[i]) > std::fabs(z[im])) im = i;
    if (z[im] < 0.0)
      for (int i = 0; i < n; ++i) z[i] = -z[i];
    cplx dk = 0.0;
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) dk += z[i] * Sc[(size_t)i * n + j] * z[j];
    if (delta) delta[k] = 0.5 * std::arg(dk);
    if (O)
      for (int i = 0; i < n; ++i) O[(size_t)i * n + k] = z[i];
  }
  return WP_OK;
}

extern "C" wp_status nd_elastic_observables(int n_blocks, const int* two_J, const int* n_open, const int* lam,
                                            const int* two_I, const double* S, double k, int n_theta,
                                            const double* theta, double* dsdo, double* Ay) {
  if (n_blocks < 1 || !two_J || !n_open || !lam || !two_I || !S || !(k > 0) || n_theta < 1 || !theta)
    return fail(WP_EINVAL, "nd_elastic_observables: bad argument");
  struct Block {
    int two_J, n;
    std::vector<int> ls, ts;
    std::vector<cplx> D;   // S^Sigma - 1
  };
  std::vector<Block> blocks(n_blocks);
  size_t off_c = 0, off_s = 0;
  for (int b = 0; b < n_blocks; ++b) {
    Block& B = blocks[b];
    B.two_J = two_J[b];
    B.n = n_open[b];
    if (B.n < 1 || B.n > 8 || B.two_J < 1 || !(B.two_J & 1)) return fail(WP_EINVAL, "nd_elastic_observables: bad block");
    std::vector<cplx> Ss;
    if (wp_status st = sigma_rep(B.two_J, B.n, lam + off_c, two_I + off_c, reinterpret_cast<const cplx*>(S) + off_s,
                                 B.ls, B.ts, Ss))
      return st;
    B.D = Ss;
    for (int a = 0; a < B.n; ++a) B.D[(size_t)a * B.n + a] -= 1.0;
    off_c += B.n;
    off_s += (size_t)B.n * B.n;
  }
  // channel-spin states (2 Sigma, 2 nu) and the neutron's sigma_y among them
  const int st_S[6] = {1, 1, 3, 3, 3, 3}, st_n[6] = {-1, 1, -3, -1, 1, 3};
  cplx sy[6][6];
  for (int a = 0; a < 6; ++a)
    for (int b = 0; b < 6; ++b) {
      cplx v = 0.0;
      for (int md = -2; md <= 2; md += 2)
        for (int s1 = -1; s1 <= 1; s1 += 2)
          for (int s2 = -1; s2 <= 1; s2 += 2) {
            if (s1 == s2) continue;
            const cplx y = s1 == 1 ? cplx(0, -1) : cplx(0, 1);   // (sigma_y)_{s1 s2}
            v += cg2(2, md, 1, s1, st_S[a], st_n[a]) * y * cg2(2, md, 1, s2, st_S[b], st_n[b]);
          }
      sy[a][b] = v;
    }
  const cplx pref = std::sqrt(M_PI) / cplx(0.0, k);
  for (int t = 0; t < n_theta; ++t) {
    cplx M[6][6] = {};
    for (const Block& B : blocks)
      for (int b = 0; b < B.n; ++b)
        for (int in = 0; in < 6; ++in) {
          if (st_S[in] != B.ts[b]) continue;
          const double c1 = cg2(B.ts[b], st_n[in], 2 * B.ls[b], 0, B.two_J, st_n[in]);
          if (c1 == 0.0) continue;
          for (int a = 0; a < B.n; ++a) {
            const cplx dab = B.D[(size_t)a * B.n + b];
            if (dab == 0.0) continue;
            for (int out = 0; out < 6; ++out) {
              if (st_S[out] != B.ts[a]) continue;
              const int two_m = st_n[in] - st_n[out];
              if (std::abs(two_m) > 2 * B.ls[a]) continue;
              const double c2 = cg2(B.ts[a], st_n[out], 2 * B.ls[a], two_m, B.two_J, st_n[in]);
              if (c2 == 0.0) continue;
              M[out][in] += pref * std::sqrt(2.0 * B.ls[b] + 1.0) * c1 * c2 * dab * ylm0(B.ls[a], two_m / 2, theta[t]);
            }
          }
        }
    double den = 0.0;
    cplx num = 0.0;
    for (int i = 0; i < 6; ++i)
      for (int j = 0; j < 6; ++j) {
        den += std::norm(M[i][j]);
        cplx msy = 0.0;   // (M sigma_y)_{ij}
        for (int l = 0; l < 6; ++l) msy += M[i][l] * sy[l][j];
        num += msy * std::conj(M[i][j]);
      }
    if (dsdo) dsdo[t] = den / 6.0;
    if (Ay) Ay[t] = den > 0.0 ? num.real() / den : 0.0;
  }
  return WP_OK;
}
