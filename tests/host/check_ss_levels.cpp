// Host check of build_ss_levels: for every level b the hierarchical 1D
// operator restricted to levels 0..b equals Q^T Bs_b Q, Q the synthesis from
// hierarchical coefficients to level-b cell-Legendre coefficients (two-scale
// relation), Bs_b the block-tridiagonal level-b matrix.  Degrees 1..3,
// periodic and zero Dirichlet, constant and variable k(x).  Prints the worst
// relative difference.
#include <cmath>
#include <cstdio>
#include <vector>
#include "internal.h"
using namespace sgdg;
std::string g_err;
namespace sgdg {
sgdg_status fail(sgdg_status st, const std::string& m) { g_err = m; return st; }
sgdg_status hip_fail(hipError_t, const char*) { return SGDG_ERR_HIP; }
}
int main() {
  double worst = 0;
  for (int k = 1; k <= 3; ++k)
    for (int bc = 0; bc <= 1; ++bc)
      for (int var = 0; var <= 1; ++var) {
        const int N = 5, K1 = k + 1, K2 = K1 * K1;
        sgdg_kdiag kd{1.0, var ? 0.5 : 0.0, 1.0, 0.3};
        Op1D op = build_op1d(N, k, 20.0, kd, bc);
        std::vector<int64_t> off;
        bool uni;
        std::vector<double> T = build_ss_levels(op, off, uni);
        const Basis1D& bs = basis1d(k);
        for (int b = 0; b <= N; ++b) {
          const int C = 1 << b, n = K1 * C;
          // hierarchical restricted (cells in hier order 0..C-1)
          std::vector<double> H(n * n, 0.0);
          for (int t = 0; t < C; ++t)
            for (int e = op.cptr[t]; e < op.cptr[t + 1]; ++e) {
              int sc = op.src[e];
              if (sc >= C) continue;
              for (int pt = 0; pt < K1; ++pt)
                for (int ps = 0; ps < K1; ++ps) H[(t * K1 + pt) * n + sc * K1 + ps] = op.val[(size_t)e * K2 + pt * K1 + ps];
            }
          // single-scale level-b matrix
          std::vector<double> Bs(n * n, 0.0);
          for (int c = 0; c < C; ++c) {
            const double* blk = &T[off[b] + (uni ? 0 : c) * 3 * K2];
            int nb[3] = {(c - 1 + C) % C, c, (c + 1) % C};
            for (int w = 0; w < 3; ++w)
              for (int q = 0; q < K1; ++q)
                for (int r = 0; r < K1; ++r) Bs[(c * K1 + q) * n + nb[w] * K1 + r] += blk[w * K2 + q * K1 + r];
          }
          // Q: columns = synthesis of hierarchical unit vectors
          std::vector<double> Q(n * n, 0.0);
          for (int col = 0; col < n; ++col) {
            std::vector<double> h(n, 0.0);
            h[col] = 1.0;
            std::vector<double> cur(h.begin(), h.begin() + K1);
            for (int l = 1; l <= b; ++l) {
              int np = 1 << (l - 1);
              std::vector<double> nx(2 * np * K1);
              for (int j = 0; j < np; ++j)
                for (int q = 0; q < K1; ++q) {
                  double lo = 0, hi = 0;
                  for (int i = 0; i < K1; ++i) {
                    lo += bs.ML[q * K1 + i] * cur[j * K1 + i] + bs.cL[i * K1 + q] * h[(np + j) * K1 + i];
                    hi += bs.MR[q * K1 + i] * cur[j * K1 + i] + bs.cR[i * K1 + q] * h[(np + j) * K1 + i];
                  }
                  nx[(2 * j) * K1 + q] = lo;
                  nx[(2 * j + 1) * K1 + q] = hi;
                }
              cur.swap(nx);
            }
            for (int i = 0; i < n; ++i) Q[i * n + col] = cur[i];
          }
          double mx = 0, err = 0;
          for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) {
              double a = 0;
              for (int u = 0; u < n; ++u)
                for (int v = 0; v < n; ++v) a += Q[u * n + i] * Bs[u * n + v] * Q[v * n + j];
              mx = std::max(mx, std::fabs(H[i * n + j]));
              err = std::max(err, std::fabs(a - H[i * n + j]));
            }
          worst = std::max(worst, err / mx);
          if (err / mx > 1e-12) printf("k=%d bc=%d var=%d b=%d err %.3e max %.3e uni %d\n", k, bc, var, b, err, mx, uni);
        }
      }
  printf("worst relative %.3e\n", worst);
}
