// Host construction of the 1D bases (Sec. 2.1, eqs. 2.1-2.6).
//
// Level 0: orthonormal Legendre sqrt(2q+1) P_q(2x-1) on [0,1].
// Level n >= 1, cell j: 2^((n-1)/2) psi_p(2^(n-1) x - j), psi_p the Alpert
// multiwavelets on [0,1], each piecewise P^k on the halves, orthonormal,
// orthogonal to all polynomials of degree <= k + p (0-based p), with the sign
// fixed so the highest nonzero Legendre coefficient on the right half is > 0.
//
// Construction here: the 2(k+1)-dimensional space of piecewise polynomials is
// written in the orthonormal half-interval Legendre bases; for p = k .. 0 the
// constraint vectors (moments against Legendre polynomials of degree
// 0..k+p, and the already-found psi_{p+1..k}) are orthonormalised by modified
// Gram-Schmidt and psi_p is the normalised residual of the unit vector that
// leaves the largest residual (the complement is one-dimensional).
#include <algorithm>
#include <cmath>
#include <map>
#include <mutex>

#include "internal.h"

namespace sgdg {

static void legendre_pair(int n, long double t, long double& pn, long double& pn1) {
  // P_n(t) and P_{n-1}(t) by the three-term recurrence
  long double p0 = 1.0L, p1 = t;
  if (n == 0) { pn = 1.0L; pn1 = 0.0L; return; }
  for (int m = 2; m <= n; ++m) {
    long double p2 = ((2 * m - 1) * t * p1 - (m - 1) * p0) / m;
    p0 = p1;
    p1 = p2;
  }
  pn = p1;
  pn1 = p0;
}

void gauss01(int n, std::vector<double>& x, std::vector<double>& w) {
  // Newton iteration for the roots of P_n, then w = 2 / ((1 - t^2) P_n'(t)^2); mapped to [0,1].
  x.assign(n, 0.0);
  w.assign(n, 0.0);
  for (int i = 0; i < n; ++i) {
    long double t = std::cos(M_PI * (i + 0.75L) / (n + 0.5L));
    long double pn, pn1, dp;
    for (int it = 0; it < 100; ++it) {
      legendre_pair(n, t, pn, pn1);
      dp = n * (t * pn - pn1) / (t * t - 1.0L);
      long double dt = pn / dp;
      t -= dt;
      if (std::fabs((double)dt) < 1e-18) break;
    }
    legendre_pair(n, t, pn, pn1);
    dp = n * (t * pn - pn1) / (t * t - 1.0L);
    x[n - 1 - i] = (double)(0.5L * (t + 1.0L));
    w[n - 1 - i] = (double)(1.0L / ((1.0L - t * t) * dp * dp));
  }
}

void legendre01_all(int n, double x, double* val, double* der) {
  // P_q(t), t = 2x-1, by the three-term recurrence; derivative by
  // P'_q = q P_{q-1} + t P'_{q-1}; orthonormal scaling sqrt(2q+1), d/dx = 2 d/dt.
  double t = 2.0 * x - 1.0;
  double P[16], dP[16];
  P[0] = 1.0;
  dP[0] = 0.0;
  if (n >= 1) {
    P[1] = t;
    dP[1] = 1.0;
  }
  for (int q = 2; q <= n; ++q) {
    P[q] = ((2 * q - 1) * t * P[q - 1] - (q - 1) * P[q - 2]) / q;
    dP[q] = q * P[q - 1] + t * dP[q - 1];
  }
  for (int q = 0; q <= n; ++q) {
    double s = std::sqrt(2.0 * q + 1.0);
    if (val) val[q] = s * P[q];
    if (der) der[q] = 2.0 * s * dP[q];
  }
}

static Basis1D make_basis(int k) {
  Basis1D b;
  b.k = k;
  const int K1 = k + 1, nb = 2 * K1;
  std::vector<double> xg, wg;
  gauss01(3 * k + 6, xg, wg);
  // constraint vectors: <phi_i, half-cell basis functions>, i = 0..2k
  std::vector<std::vector<long double>> cons(2 * k + 1, std::vector<long double>(nb, 0.0L));
  double vq[16], vi[16];
  for (int g = 0; g < (int)xg.size(); ++g) {
    for (int half = 0; half < 2; ++half) {
      double t = 0.5 * (xg[g] + half);  // point in [0,1]
      legendre01_all(k, xg[g], vq, nullptr);
      legendre01_all(2 * k, t, vi, nullptr);
      for (int i = 0; i <= 2 * k; ++i)
        for (int q = 0; q < K1; ++q)
          cons[i][half * K1 + q] += (long double)wg[g] * 0.5L * std::sqrt(2.0L) * vq[q] * vi[i];
    }
  }
  std::vector<std::vector<long double>> psi(K1);
  for (int p = k; p >= 0; --p) {
    std::vector<std::vector<long double>> set;
    for (int i = 0; i <= k + p; ++i) set.push_back(cons[i]);
    for (int q = p + 1; q <= k; ++q) set.push_back(psi[q]);
    // modified Gram-Schmidt, two passes
    std::vector<std::vector<long double>> ortho;
    for (auto v : set) {
      for (int pass = 0; pass < 2; ++pass)
        for (auto& o : ortho) {
          long double dot = 0;
          for (int c = 0; c < nb; ++c) dot += o[c] * v[c];
          for (int c = 0; c < nb; ++c) v[c] -= dot * o[c];
        }
      long double nrm = 0;
      for (int c = 0; c < nb; ++c) nrm += v[c] * v[c];
      nrm = std::sqrt(nrm);
      for (int c = 0; c < nb; ++c) v[c] /= nrm;
      ortho.push_back(v);
    }
    // complement: residual of the unit vector with the largest residual
    std::vector<long double> best;
    long double bestn = -1;
    for (int e = 0; e < nb; ++e) {
      std::vector<long double> r(nb, 0.0L);
      r[e] = 1.0L;
      for (int pass = 0; pass < 2; ++pass)
        for (auto& o : ortho) {
          long double dot = 0;
          for (int c = 0; c < nb; ++c) dot += o[c] * r[c];
          for (int c = 0; c < nb; ++c) r[c] -= dot * o[c];
        }
      long double nrm = 0;
      for (int c = 0; c < nb; ++c) nrm += r[c] * r[c];
      if (nrm > bestn) {
        bestn = nrm;
        best = r;
      }
    }
    long double nrm = std::sqrt(bestn);
    for (auto& v : best) v /= nrm;
    // sign rule on the right half
    int top = -1;
    for (int q = 0; q < K1; ++q)
      if (std::fabs((double)best[K1 + q]) > 1e-10) top = q;
    if (best[K1 + top] < 0)
      for (auto& v : best) v = -v;
    psi[p] = best;
  }
  b.cL.assign(K1 * K1, 0.0);
  b.cR.assign(K1 * K1, 0.0);
  for (int p = 0; p < K1; ++p)
    for (int q = 0; q < K1; ++q) {
      b.cL[p * K1 + q] = (double)psi[p][q];
      b.cR[p * K1 + q] = (double)psi[p][K1 + q];
    }
  // two-scale refinement: coefficient of child basis q in parent basis i
  b.ML.assign(K1 * K1, 0.0);
  b.MR.assign(K1 * K1, 0.0);
  for (int g = 0; g < (int)xg.size(); ++g) {
    for (int half = 0; half < 2; ++half) {
      double t = 0.5 * (xg[g] + half);
      legendre01_all(k, xg[g], vq, nullptr);
      legendre01_all(k, t, vi, nullptr);
      auto& M = half ? b.MR : b.ML;
      for (int q = 0; q < K1; ++q)
        for (int i = 0; i < K1; ++i) M[q * K1 + i] += wg[g] * 0.5 * std::sqrt(2.0) * vq[q] * vi[i];
    }
  }
  return b;
}

const Basis1D& basis1d(int k) {
  static std::mutex mu;
  static std::map<int, Basis1D> cache;
  std::lock_guard<std::mutex> lock(mu);
  auto it = cache.find(k);
  if (it == cache.end()) it = cache.emplace(k, make_basis(k)).first;
  return it->second;
}

double hier_value(const Basis1D& b, int level, int j, int p, double x, bool deriv) {
  const int k = b.k, K1 = k + 1;
  double v[16], dv[16];
  if (level == 0) {
    legendre01_all(k, x, v, dv);
    return deriv ? dv[p] : v[p];
  }
  double s = std::ldexp(1.0, level - 1);
  double t = s * x - j;
  if (t < 0.0 || t >= 1.0) return 0.0;
  int half = t >= 0.5 ? 1 : 0;
  double u = 2.0 * t - half;
  legendre01_all(k, u, v, dv);
  const double* c = half ? &b.cR[p * K1] : &b.cL[p * K1];
  double acc = 0.0;
  for (int q = 0; q < K1; ++q) acc += c[q] * (deriv ? dv[q] : v[q]);
  // psi(t) = sum c_q sqrt(2) phi_q(2t - half); d/dx brings 2 s
  return deriv ? std::sqrt(s) * std::sqrt(2.0) * 2.0 * s * acc : std::sqrt(s) * std::sqrt(2.0) * acc;
}

}  // namespace sgdg
