// Host build of the 1D interior-penalty operator in the hierarchical basis.
//
// Bilinear form (Sec. 2.1, eq. 2.10, jumps/averages eq. 2.11) of one axis:
//   B(u, v) = int k(x) u' v' dx
//             + sum over faces e of Omega_N: -{k u'}[v] - {k v'}[u] + (sigma/h_N)[u][v],
// periodic (the face at x = 0 joins the last and first cell) or zero
// Dirichlet (the face at x = 0 acts on the first cell with [u] = -u(0+),
// {k u'} = k u'(0+); the face at x = 1 on the last cell with [u] = u(1-),
// {k u'} = k u'(1-): trace times outward normal and one-sided flux, the
// boundary convention stated after eq. 2.11), h_N = 2^-N.
//
// Route: for every source hierarchical function, its restriction to the
// finest cells is obtained by two-scale refinement of the Alpert / Legendre
// coefficients; the full-grid SIPG operator is applied cell by cell (volume
// and face matrices); the result is analysed back to hierarchical
// coefficients by the fast multiwavelet transform restricted to the cells it
// touches.  Only cell blocks above the rounding floor are kept (vanishing
// moments make all others exactly zero), giving a cell-block CSR matrix.
#include <algorithm>
#include <cmath>
#include <map>
#include <tuple>

#include "internal.h"

namespace sgdg {

namespace {

struct Range {  // values at one level for extended cells a .. a+len-1 (len <= 2^n)
  int n = 0;
  long a = 0, len = 0;
  std::vector<double> s;  // len * K1
  bool full() const { return len == (1L << n); }
  // pointer to the coefficients of actual cell c (mod 2^n), or nullptr
  const double* at(long c, int K1) const {
    long m = 1L << n;
    long off = ((c - a) % m + m) % m;
    if (off >= len) return nullptr;
    return &s[off * K1];
  }
};

inline double kval(const sgdg_kdiag& kd, double x) { return kd.a0 + kd.a1 * std::sin(2.0 * M_PI * kd.freq * x + kd.phase); }

}  // namespace

// Full-grid SIPG matrices on the level-N cells: volume (per cell, or one when
// k(x) is constant), interior faces (2K1 x 2K1, rows/cols [left cell q |
// right cell q]; per face, or one) and the two zero-Dirichlet boundary faces
// (K1 x K1 on the end cells).  Every matrix is [target q][source r].
CellMats cell_mats(int N, int k, double sigma, const sgdg_kdiag& kd) {
  const int K1 = k + 1, K2 = K1 * K1;
  const long nc = 1L << N;
  const double h = std::ldexp(1.0, -N);
  CellMats cm;
  cm.constk = (kd.a1 == 0.0);
  const bool constk = cm.constk;

  // volume matrices per finest cell: (1/h^2) sum_g w_g k(x_g) phi'_q phi'_r
  std::vector<double> xg, wg;
  gauss01(12, xg, wg);
  std::vector<double> dphi(xg.size() * K1);
  for (size_t g = 0; g < xg.size(); ++g) legendre01_all(k, xg[g], nullptr, &dphi[g * K1]);
  cm.kvol.assign((constk ? 1 : nc) * K2, 0.0);
  for (long c = 0; c < (constk ? 1 : nc); ++c)
    for (size_t g = 0; g < xg.size(); ++g) {
      double kv = kval(kd, (c + xg[g]) * h);
      for (int q = 0; q < K1; ++q)
        for (int r = 0; r < K1; ++r)
          cm.kvol[c * K2 + q * K1 + r] += wg[g] * kv * dphi[g * K1 + q] * dphi[g * K1 + r] / (h * h);
    }
  // face matrices (2K1 x 2K1): rows/cols [left cell q | right cell q]
  double v0[16], v1[16], d0[16], d1[16];
  legendre01_all(k, 0.0, v0, d0);
  legendre01_all(k, 1.0, v1, d1);
  std::vector<double> jump(2 * K1), mder(2 * K1);
  for (int q = 0; q < K1; ++q) {
    jump[q] = v1[q] / std::sqrt(h);
    jump[K1 + q] = -v0[q] / std::sqrt(h);
    mder[q] = 0.5 * d1[q] / (h * std::sqrt(h));
    mder[K1 + q] = 0.5 * d0[q] / (h * std::sqrt(h));
  }
  const long nf = constk ? 1 : nc;
  cm.face.assign(nf * 4 * K2, 0.0);
  for (long e = 0; e < nf; ++e) {
    const double ke = kval(kd, e * h);
    double* F = &cm.face[e * 4 * K2];
    for (int a = 0; a < 2 * K1; ++a)
      for (int b = 0; b < 2 * K1; ++b)
        F[a * 2 * K1 + b] = -ke * jump[a] * mder[b] - ke * mder[a] * jump[b] + sigma / h * jump[a] * jump[b];
  }

  // zero-Dirichlet boundary face matrices (K1 x K1, on one cell): x = 0 acts on
  // cell 0 (jump -v0/sqrt(h), flux d0/h^1.5), x = 1 on cell nc-1 (v1, d1)
  cm.FB0.assign(K2, 0.0);
  cm.FB1.assign(K2, 0.0);
  {
    const double k0 = kval(kd, 0.0), k1 = kval(kd, 1.0), sh = std::sqrt(h), h15 = h * sh;
    for (int a = 0; a < K1; ++a)
      for (int b = 0; b < K1; ++b) {
        const double ja0 = -v0[a] / sh, jb0 = -v0[b] / sh, da0 = d0[a] / h15, db0 = d0[b] / h15;
        const double ja1 = v1[a] / sh, jb1 = v1[b] / sh, da1 = d1[a] / h15, db1 = d1[b] / h15;
        cm.FB0[a * K1 + b] = -k0 * ja0 * db0 - k0 * da0 * jb0 + sigma / h * ja0 * jb0;
        cm.FB1[a * K1 + b] = -k1 * ja1 * db1 - k1 * da1 * jb1 + sigma / h * ja1 * jb1;
      }
  }
  return cm;
}

Op1D build_op1d(int N, int k, double sigma, const sgdg_kdiag& kd, int bc) {
  const Basis1D& bs = basis1d(k);
  const int K1 = k + 1, K2 = K1 * K1;
  const long nc = 1L << N;
  const CellMats cm = cell_mats(N, k, sigma, kd);
  const bool constk = cm.constk;
  const std::vector<double>& kvol = cm.kvol;
  const std::vector<double>& FB0 = cm.FB0;
  const std::vector<double>& FB1 = cm.FB1;
  const double scale_est = sigma * std::ldexp(1.0, 2 * N);
  std::map<std::pair<int32_t, int32_t>, std::vector<double>> blocks;  // (target cell, source cell) -> [pt][ps]

  for (long cs = 0; cs < nc; ++cs) {
    // level and translate of source cell index cs
    int ls = 0;
    long js = 0;
    if (cs > 0) {
      ls = 1;
      while ((1L << ls) <= cs) ++ls;  // 2^(ls-1) <= cs < 2^ls
      js = cs - (1L << (ls - 1));
    }
    // finest-level restriction of the K1 functions (source index ps) by refinement
    long a0, len0;
    int lev;
    std::vector<double> cur;  // [cell][ps][q]
    if (ls == 0) {
      lev = 0;
      a0 = 0;
      len0 = 1;
      cur.assign(K1 * K1, 0.0);
      for (int p = 0; p < K1; ++p) cur[p * K1 + p] = 1.0;
    } else {
      lev = ls;
      a0 = 2 * js;
      len0 = 2;
      cur.assign(2 * K2, 0.0);
      for (int p = 0; p < K1; ++p)
        for (int q = 0; q < K1; ++q) {
          cur[0 * K2 + p * K1 + q] = bs.cL[p * K1 + q];
          cur[1 * K2 + p * K1 + q] = bs.cR[p * K1 + q];
        }
    }
    for (; lev < N; ++lev) {
      std::vector<double> nxt(2 * len0 * K2, 0.0);
      for (long c = 0; c < len0; ++c)
        for (int p = 0; p < K1; ++p)
          for (int q = 0; q < K1; ++q) {
            double sl = 0, sr = 0;
            for (int i = 0; i < K1; ++i) {
              double s = cur[c * K2 + p * K1 + i];
              sl += bs.ML[q * K1 + i] * s;
              sr += bs.MR[q * K1 + i] * s;
            }
            nxt[(2 * c) * K2 + p * K1 + q] = sl;
            nxt[(2 * c + 1) * K2 + p * K1 + q] = sr;
          }
      cur.swap(nxt);
      a0 *= 2;
      len0 *= 2;
    }
    // apply the full-grid operator: result over [a0-1, a0+len0+1) (or all cells)
    bool full = (len0 >= nc - 1);
    long ra = full ? 0 : a0 - 1;
    long rlen = full ? nc : len0 + 2;
    // per source function ps we build one Range at level N
    std::vector<Range> res(K1);
    for (int p = 0; p < K1; ++p) {
      res[p].n = N;
      res[p].a = ra;
      res[p].len = rlen;
      res[p].s.assign(rlen * K1, 0.0);
    }
    auto gval = [&](long c, int p, int q) -> double {  // source restriction at actual cell c
      long off = ((c - a0) % nc + nc) % nc;
      if (off >= len0) return 0.0;
      return cur[off * K2 + p * K1 + q];
    };
    auto addres = [&](long c, int p, int q, double v) {
      long off = ((c - ra) % nc + nc) % nc;
      if (off < rlen) res[p].s[off * K1 + q] += v;
    };
    // volume terms
    for (long o = 0; o < len0; ++o) {
      long c = ((a0 + o) % nc + nc) % nc;
      const double* K = &kvol[(constk ? 0 : c) * K2];
      for (int p = 0; p < K1; ++p)
        for (int q = 0; q < K1; ++q) {
          double acc = 0;
          for (int r = 0; r < K1; ++r) acc += K[q * K1 + r] * cur[o * K2 + p * K1 + r];
          addres(c, p, q, acc);
        }
    }
    // face terms: faces e touching the source cells a0 .. a0+len0 (face e between e-1 and e)
    long nf = full ? nc : len0 + 1;
    for (long f = 0; f < nf; ++f) {
      long e = full ? f : a0 + f;
      long em = ((e % nc) + nc) % nc;
      if (bc == 1 && em == 0) {
        // the two boundary faces: each couples one end cell with itself
        for (int p = 0; p < K1; ++p)
          for (int side = 0; side < 2; ++side) {
            const long c = side == 0 ? 0 : nc - 1;
            const double* FB = side == 0 ? FB0.data() : FB1.data();
            double u[16];
            for (int q = 0; q < K1; ++q) u[q] = gval(c, p, q);
            for (int a = 0; a < K1; ++a) {
              double acc = 0;
              for (int b = 0; b < K1; ++b) acc += FB[a * K1 + b] * u[b];
              if (acc != 0.0) addres(c, p, a, acc);
            }
          }
        continue;
      }
      const double* Fp = &cm.face[(constk ? 0 : em) * 4 * K2];
      long L = em - 1, R = em;
      for (int p = 0; p < K1; ++p) {
        double u[32];
        for (int q = 0; q < K1; ++q) {
          u[q] = gval(L, p, q);
          u[K1 + q] = gval(R, p, q);
        }
        for (int a = 0; a < 2 * K1; ++a) {
          double acc = 0;
          for (int b = 0; b < 2 * K1; ++b) acc += Fp[a * 2 * K1 + b] * u[b];
          if (acc != 0.0) addres(a < K1 ? L : R, p, a % K1, acc);
        }
      }
    }
    // analysis: finest cell-Legendre -> hierarchical, level by level
    std::vector<Range> level = res;
    for (int n = N; n >= 1; --n) {
      const Range& r0 = level[0];
      long pa, plen;
      long half = 1L << (n - 1);
      if (r0.full()) {
        pa = 0;
        plen = half;
      } else {
        pa = (long)std::floor(r0.a / 2.0);
        long last = (long)std::floor((r0.a + r0.len - 1) / 2.0);
        plen = last - pa + 1;
        if (plen >= half) {
          pa = 0;
          plen = half;
        }
      }
      std::vector<Range> parent(K1);
      for (int p = 0; p < K1; ++p) {
        parent[p].n = n - 1;
        parent[p].a = pa;
        parent[p].len = plen;
        parent[p].s.assign(plen * K1, 0.0);
        const Range& ch = level[p];
        for (long o = 0; o < plen; ++o) {
          long P = pa + o;
          const double* sl = ch.at(2 * P, K1);
          const double* sr = ch.at(2 * P + 1, K1);
          double* sp = &parent[p].s[o * K1];
          double dcoef[16] = {0};
          for (int i = 0; i < K1; ++i) {
            double acc = 0, dacc = 0;
            for (int q = 0; q < K1; ++q) {
              double vl = sl ? sl[q] : 0.0, vr = sr ? sr[q] : 0.0;
              acc += bs.ML[q * K1 + i] * vl + bs.MR[q * K1 + i] * vr;
              dacc += bs.cL[i * K1 + q] * vl + bs.cR[i * K1 + q] * vr;
            }
            sp[i] = acc;
            dcoef[i] = dacc;
          }
          long Pm = ((P % half) + half) % half;
          int32_t ct = (int32_t)(half + Pm);  // level-n cell index of target
          double mx = 0;
          for (int i = 0; i < K1; ++i) mx = std::max(mx, std::fabs(dcoef[i]));
          if (mx > 1e-14 * scale_est) {
            auto& blk = blocks[{ct, (int32_t)cs}];
            if (blk.empty()) blk.assign(K2, 0.0);
            for (int i = 0; i < K1; ++i) blk[i * K1 + p] = dcoef[i];
          }
        }
      }
      level.swap(parent);
    }
    // level 0 coefficients
    for (int p = 0; p < K1; ++p) {
      const double* s0 = level[p].at(0, K1);
      double mx = 0;
      for (int i = 0; i < K1; ++i) mx = std::max(mx, std::fabs(s0 ? s0[i] : 0.0));
      if (s0 && mx > 1e-14 * scale_est) {
        auto& blk = blocks[{0, (int32_t)cs}];
        if (blk.empty()) blk.assign(K2, 0.0);
        for (int i = 0; i < K1; ++i) blk[i * K1 + p] = s0[i];
      }
    }
  }
  double maxabs = 0;
  for (auto& kv : blocks)
    for (double v : kv.second) maxabs = std::max(maxabs, std::fabs(v));
  Op1D op;
  op.N = N;
  op.k = k;
  op.sigma = sigma;
  op.bc = bc;
  op.kd = {kd.a0, kd.a1, kd.freq, kd.phase};
  op.cptr.assign(nc + 1, 0);
  for (auto& kv : blocks) {
    double mx = 0;
    for (double v : kv.second) mx = std::max(mx, std::fabs(v));
    if (mx <= 1e-13 * maxabs) continue;
    op.cptr[kv.first.first + 1]++;
    op.src.push_back(kv.first.second);
    op.val.insert(op.val.end(), kv.second.begin(), kv.second.end());
  }
  for (long c = 0; c < nc; ++c) op.cptr[c + 1] += op.cptr[c];
  return op;
}

// The same operator restricted to the piecewise polynomials on the level-b
// cells, b = 0..N, in the cell-Legendre (single-scale) basis of level b.  On
// level N it is the full-grid SIPG form itself: block tridiagonal, cell c
// coupling to c-1 (block L), itself (D) and c+1 (R), indices taken mod 2^N
// (periodic) or with the end blocks absent (zero Dirichlet, whose boundary
// faces sit on the diagonal).  Each coarser level is the Galerkin restriction
// of the finer one through the two-scale relation (a level-b cell function
// is ML / MR times its coefficients on the left / right child), which keeps
// the block-tridiagonal shape: for parent P,
//   D'_P = ML^T D_2P ML + ML^T R_2P MR + MR^T L_2P+1 ML + MR^T D_2P+1 MR,
//   L'_P = ML^T L_2P MR,   R'_P = MR^T R_2P+1 ML.
// Since the hierarchical basis of levels 0..b is an orthonormal basis of the
// same space, the hierarchical operator restricted to levels 0..b equals
// this level-b matrix conjugated by the multiwavelet transform (Sec. 2.1,
// eq. 2.10 on the space of a fibre of the sparse grid).
// Layout: level b at off[b], cells c = 0..2^b - 1 (one cell when uniform),
// blocks L, D, R of K1 x K1 each, [target q][source r].
std::vector<double> build_ss_levels(const Op1D& op, std::vector<int64_t>& off, bool& uniform) {
  const int N = op.N, k = op.k, K1 = k + 1, K2 = K1 * K1, B3 = 3 * K2;
  const sgdg_kdiag kd{op.kd[0], op.kd[1], op.kd[2], op.kd[3]};
  const CellMats cm = cell_mats(N, k, op.sigma, kd);
  const Basis1D& bs = basis1d(k);
  uniform = cm.constk && op.bc == 0;
  auto ncell = [&](int b) -> long { return uniform ? 1L : (1L << b); };
  off.assign(N + 2, 0);
  for (int b = 0; b <= N; ++b) off[b + 1] = off[b] + ncell(b) * B3;
  std::vector<double> T(off[N + 1], 0.0);
  // level N
  {
    const long nc = 1L << N;
    double* lv = &T[off[N]];
    for (long c = 0; c < ncell(N); ++c)
      for (int i = 0; i < K2; ++i) lv[c * B3 + K2 + i] = cm.kvol[(cm.constk ? 0 : c) * K2 + i];
    for (long e = 0; e < (uniform ? 1 : nc); ++e) {
      if (op.bc == 1 && e == 0) {
        for (int i = 0; i < K2; ++i) {
          lv[0 * B3 + K2 + i] += cm.FB0[i];
          lv[(nc - 1) * B3 + K2 + i] += cm.FB1[i];
        }
        continue;
      }
      const double* F = &cm.face[(cm.constk ? 0 : e) * 4 * K2];
      const long cl = uniform ? 0 : (e - 1 + nc) % nc, cr = uniform ? 0 : e;
      for (int a = 0; a < K1; ++a)
        for (int b = 0; b < K1; ++b) {
          lv[cl * B3 + K2 + a * K1 + b] += F[a * 2 * K1 + b];                // D of the left cell
          lv[cl * B3 + 2 * K2 + a * K1 + b] += F[a * 2 * K1 + K1 + b];       // R of the left cell
          lv[cr * B3 + a * K1 + b] += F[(K1 + a) * 2 * K1 + b];              // L of the right cell
          lv[cr * B3 + K2 + a * K1 + b] += F[(K1 + a) * 2 * K1 + K1 + b];    // D of the right cell
        }
    }
  }
  // Galerkin restriction level by level: out += Mt^T B Ms
  auto rap = [&](double* out, const double* Bm, const double* Mt, const double* Ms) {
    for (int i = 0; i < K1; ++i)
      for (int j = 0; j < K1; ++j) {
        double acc = 0;
        for (int q = 0; q < K1; ++q)
          for (int r = 0; r < K1; ++r) acc += Mt[q * K1 + i] * Bm[q * K1 + r] * Ms[r * K1 + j];
        out[i * K1 + j] += acc;
      }
  };
  const double* ML = bs.ML.data();
  const double* MR = bs.MR.data();
  for (int b = N; b >= 1; --b) {
    const double* fine = &T[off[b]];
    double* crs = &T[off[b - 1]];
    for (long P = 0; P < ncell(b - 1); ++P) {
      const long c0 = uniform ? 0 : 2 * P, c1 = uniform ? 0 : 2 * P + 1;
      double* o = &crs[P * B3];
      rap(o + K2, fine + c0 * B3 + K2, ML, ML);
      rap(o + K2, fine + c0 * B3 + 2 * K2, ML, MR);
      rap(o + K2, fine + c1 * B3, MR, ML);
      rap(o + K2, fine + c1 * B3 + K2, MR, MR);
      rap(o, fine + c0 * B3, ML, MR);
      rap(o + 2 * K2, fine + c1 * B3 + 2 * K2, MR, ML);
    }
  }
  return T;
}

}  // namespace sgdg
