// Reaction term F(U) = P f(R U) at the Gauss points of the finest mesh.
//
// Sec. 5 of the paper: u_h is reconstructed at the Gaussian points of the
// finest-level mesh Omega_N and int f(u_h) v dx is done by that quadrature
// (k+1 Gauss-Legendre points per axis in every finest cell; with this rule
// P R = I on the sparse space).  R and P = R^T diag(W) are applied by sum
// factorisation over the axes:
//
//   expand stage m (m = 0..d-2): T_{m+1}[q_0..q_m][sparse grid of axes m+1..d-1]
//       = sum over l_m <= N - |l_{>m}|, p of T_m[..][(l_m, l_{>m}); j(q_m), p, ..] E[l_m][q_m][p]
//   line kernel (last axis): per line expand to its np1 points, apply f (or
//       the per-point species-Jacobian solve of the implicit stage), contract
//       back with the weights, all in LDS;
//   contract stage m (m = d-2..0): the transpose, summing each coefficient
//       over the points of its support; stage 0 writes plan vectors and fuses
//       the mode's post-processing (residual G, correction of U).
//
// Every stage covers all instances, species and right-hand sides of the plan
// in one launch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <functional>
#include <numeric>

#include "internal.h"
#include "kernels.h"
#include "reaction.h"

namespace sgdg {

sgdg_status plan_upload(sgdg_plan* p, const void* src, size_t bytes, void** out);
static sgdg_status line_lds_attr(const RHost* rh);

template <class T>
static sgdg_status up(sgdg_plan* p, const std::vector<T>& v, T** out) {
  return plan_upload(p, v.data(), v.size() * sizeof(T), (void**)out);
}

static std::vector<std::vector<int>> grid_blocks(int r, int N) {
  std::vector<std::vector<int>> out;
  std::vector<int> l(r, 0);
  std::function<void(int, int)> rec = [&](int m, int rem) {
    if (m == r) {
      out.push_back(l);
      return;
    }
    for (int v = 0; v <= rem; ++v) {
      l[m] = v;
      rec(m + 1, rem - v);
    }
  };
  rec(0, N);
  std::stable_sort(out.begin(), out.end(), [](const std::vector<int>& a, const std::vector<int>& b) {
    int sa = std::accumulate(a.begin(), a.end(), 0), sb = std::accumulate(b.begin(), b.end(), 0);
    if (sa != sb) return sa < sb;
    return a < b;
  });
  return out;
}

sgdg_status reaction_build(sgdg_plan* plan) {
  RHost* rh = new RHost();
  plan->rdata = rh;
  const int d = plan->d;
  std::vector<RInst> ri;
  std::vector<RBlk> rblk;
  std::vector<int32_t> rid;
  std::vector<double> E, w1;
  int64_t ws = 0;
  rh->cum_x.assign(d, std::vector<int64_t>(1, 0));
  rh->cum_y.assign(d, std::vector<int64_t>(1, 0));
  rh->cum_line.assign(1, 0);
  for (int i = 0; i < plan->ninst; ++i) {
    const HostInstance& hi = plan->inst[i];
    const int N = hi.desc.n, K1 = hi.desc.k + 1, S = hi.desc.nspecies;
    RInst r{};
    r.N = N;
    r.K1 = K1;
    r.S = S;
    r.nq = K1;
    r.np1 = K1 << N;
    r.n1 = K1 << N;
    r.d = d;
    r.seg = hi.offset;
    r.ndof = hi.ndof;
    std::memcpy(r.rx, hi.desc.rx, sizeof(r.rx));
    rh->max_n1 = std::max(rh->max_n1, r.n1);
    rh->max_np1 = std::max(rh->max_np1, r.np1);
    // 1D Gauss points and basis values
    std::vector<double> xg, wg;
    gauss01(r.nq, xg, wg);
    const Basis1D& bs = basis1d(hi.desc.k);
    const double h = std::ldexp(1.0, -N);
    r.E_off = (int64_t)E.size();
    r.w_off = (int64_t)w1.size();
    for (int q = 0; q < r.np1; ++q) w1.push_back(wg[q % r.nq] * h);
    for (int l = 0; l <= N; ++l)
      for (int q = 0; q < r.np1; ++q) {
        const int cell = q / r.nq;
        const int j = l == 0 ? 0 : (cell >> (N - l + 1));
        const double x = (cell + xg[q % r.nq]) * h;
        for (int p = 0; p < K1; ++p) E.push_back(hier_value(bs, l, j, p, x, false));
      }
    // r-dimensional sparse grids, r = 1..d
    for (int rr = 1; rr <= d; ++rr) {
      auto blocks = grid_blocks(rr, N);
      r.blk_off[rr] = (int32_t)rblk.size();
      r.nblk[rr] = (int32_t)blocks.size();
      r.id_off[rr] = (int32_t)rid.size();
      int pw = 1;
      for (int m = 0; m < rr; ++m) pw *= (N + 1);
      std::vector<int32_t> tab(pw, -1);
      int64_t st = 0;
      for (size_t b = 0; b < blocks.size(); ++b) {
        RBlk B{};
        B.start = st;
        int64_t sz = 1;
        int lin = 0;
        for (int m = 0; m < rr; ++m) {
          B.lev[m] = blocks[b][m];
          sz *= (int64_t)level_count(blocks[b][m]) * K1;
          lin = lin * (N + 1) + blocks[b][m];
        }
        B.size = (int32_t)sz;
        B.lsum = std::accumulate(blocks[b].begin(), blocks[b].end(), 0);
        tab[lin] = (int32_t)b;
        rblk.push_back(B);
        st += sz;
      }
      r.gdof[rr] = st;
      rid.insert(rid.end(), tab.begin(), tab.end());
    }
    r.gdof[0] = 1;
    r.npre[0] = 1;
    for (int m = 1; m <= d; ++m) r.npre[m] = r.npre[m - 1] * r.np1;
    // workspace (doubles per right-hand side): expansion outputs hold two inputs
    for (int m = 1; m <= d - 1; ++m) {
      r.X_off[m] = ws;
      ws += 2 * (int64_t)S * r.npre[m] * r.gdof[d - m];
    }
    for (int m = 1; m <= d - 1; ++m) {
      r.Y_off[m] = ws;
      ws += (int64_t)S * r.npre[m] * r.gdof[d - m];
    }
    if (d == 1) {
      r.Y_off[0] = ws;
      ws += (int64_t)S * hi.ndof;
    }
    for (int m = 0; m + 1 <= d - 1; ++m)
      rh->cum_x[m].push_back(rh->cum_x[m].back() + (int64_t)S * r.npre[m + 1] * r.gdof[d - m - 1]);
    for (int m = 1; m <= d - 1; ++m)
      rh->cum_y[m].push_back(rh->cum_y[m].back() + (int64_t)S * r.npre[m] * r.gdof[d - m]);
    rh->cum_line.push_back(rh->cum_line.back() + r.npre[d - 1]);
    ri.push_back(r);
  }
  rh->rws = ws;
  if (rh->max_n1 > 2048) return fail(SGDG_ERR_UNSUPPORTED, "reaction: (k+1) 2^N above 2048 per axis");
  sgdg_status st;
  if ((st = up(plan, ri, &rh->dev.inst)) != SGDG_OK || (st = up(plan, rblk, &rh->dev.rblk)) != SGDG_OK ||
      (st = up(plan, rid, &rh->dev.rid)) != SGDG_OK || (st = up(plan, E, &rh->dev.E)) != SGDG_OK ||
      (st = up(plan, w1, &rh->dev.w1)) != SGDG_OK || (st = up(plan, rh->cum_line, &rh->dev.cum_line)) != SGDG_OK)
    return st;
  for (int m = 0; m < d; ++m) {
    if ((st = up(plan, rh->cum_x[m], &rh->dev.cum_x[m])) != SGDG_OK) return st;
    if ((st = up(plan, rh->cum_y[m], &rh->dev.cum_y[m])) != SGDG_OK) return st;
  }
  return line_lds_attr(rh);
}

void reaction_destroy(sgdg_plan* plan) {
  delete (RHost*)plan->rdata;
  plan->rdata = nullptr;
}

int64_t reaction_ws_doubles(const sgdg_plan* plan) { return ((const RHost*)plan->rdata)->rws; }

// ---------------------------------------------------------------- kernels

__device__ __forceinline__ int find_inst(const int64_t* __restrict__ cum, int ninst, int64_t e) {
  int lo = 0, hi = ninst - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (cum[mid] <= e)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

__device__ __forceinline__ int find_rblk(const RBlk* __restrict__ b, int n, int64_t e) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (b[mid].start <= e)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

__device__ __forceinline__ int cell_of_level(int q, int l, int N, int nq) { return l == 0 ? 0 : ((q / nq) >> (N - l + 1)); }

// input vector of expansion stage 0 / the line kernel when d = 1 (plan vectors), per input z
__device__ __forceinline__ const double* plan_in(const RxArgs& a, int z, int64_t rhs_total) {
  return (z == 0 ? (const double*)a.U : a.G) + rhs_total;
}

__global__ __launch_bounds__(256) void k_rx_expand(RTables R, int ninst, int m, int64_t total, RxArgs a,
                                                   int64_t rws) {
  const int z = blockIdx.z, rhs = blockIdx.y;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t* cum = R.cum_x[m];
  if (e >= cum[ninst]) return;
  const int inst = find_inst(cum, ninst, e);
  if (a.conv && a.conv[rhs * ninst + inst]) return;
  const RInst& I = R.inst[inst];
  const int d = I.d, r = d - m, N = I.N, K1 = I.K1, S = I.S, np1 = I.np1;
  int64_t le = e - cum[inst];
  const int64_t nout = I.npre[m + 1] * I.gdof[r - 1];
  const int s = (int)(le / nout);
  le -= (int64_t)s * nout;
  const int64_t pre1 = le / I.gdof[r - 1];
  const int64_t eo = le - pre1 * I.gdof[r - 1];
  const int qm = (int)(pre1 % np1);
  const int64_t pre0 = pre1 / np1;
  const RBlk* ob = R.rblk + I.blk_off[r - 1];
  const int bo = find_rblk(ob, I.nblk[r - 1], eo);
  const RBlk B = ob[bo];
  const int64_t rest = eo - B.start;
  const int64_t Sb = B.size;
  int lin = 0, pw = 1;
  for (int t = r - 2; t >= 0; --t) {
    lin += B.lev[t] * pw;
    pw *= (N + 1);
  }
  // pw = (N+1)^(r-1): weight of the leading axis (axis m) in the r-dim id table
  const int32_t* __restrict__ id = R.rid + I.id_off[r];
  const RBlk* ib = R.rblk + I.blk_off[r];
  const double* __restrict__ in;
  double* xr = a.rws + (int64_t)rhs * rws;
  if (m == 0)
    in = plan_in(a, z, (int64_t)rhs * total) + I.seg + (int64_t)s * I.ndof;
  else
    in = xr + I.X_off[m] + (((int64_t)z * S + s) * I.npre[m] + pre0) * I.gdof[r];
  const double* __restrict__ E = R.E + I.E_off;
  double acc = 0.0;
  for (int l = 0; l <= N - B.lsum; ++l) {
    const int bi = id[l * pw + lin];
    const int64_t base = ib[bi].start;
    const int j = cell_of_level(qm, l, N, I.nq);
    const double* ev = E + ((int64_t)l * np1 + qm) * K1;
    for (int p = 0; p < K1; ++p) acc += in[base + (int64_t)(j * K1 + p) * Sb + rest] * ev[p];
  }
  xr[I.X_off[m + 1] + (((int64_t)z * S + s) * I.npre[m + 1] + pre1) * I.gdof[r - 1] + eo] = acc;
}

__device__ __forceinline__ void rx_f(const double (*c)[4][4], int S, const double* u, double* f) {
  const double u0 = u[0], u1 = S > 1 ? u[1] : 0.0;
  double p0[4] = {1.0, u0, u0 * u0, u0 * u0 * u0};
  double p1[4] = {1.0, u1, u1 * u1, u1 * u1 * u1};
  for (int s = 0; s < S; ++s) {
    double acc = 0.0;
    for (int aa = 0; aa < 4; ++aa)
      for (int bb = 0; bb < 4; ++bb) acc += c[s][aa][bb] * p0[aa] * p1[bb];
    f[s] = acc;
  }
}

__device__ __forceinline__ void rx_jac(const double (*c)[4][4], int S, const double* u, double J[2][2]) {
  const double u0 = u[0], u1 = S > 1 ? u[1] : 0.0;
  double p0[4] = {1.0, u0, u0 * u0, u0 * u0 * u0};
  double p1[4] = {1.0, u1, u1 * u1, u1 * u1 * u1};
  for (int s = 0; s < S; ++s) {
    double j0 = 0.0, j1 = 0.0;
    for (int aa = 0; aa < 4; ++aa)
      for (int bb = 0; bb < 4; ++bb) {
        if (aa > 0) j0 += c[s][aa][bb] * aa * p0[aa - 1] * p1[bb];
        if (bb > 0) j1 += c[s][aa][bb] * bb * p0[aa] * p1[bb - 1];
      }
    J[s][0] = j0;
    J[s][1] = j1;
  }
}

// One workgroup per line along the last axis: expand, pointwise map, contract.
__global__ __launch_bounds__(256) void k_rx_line(RTables R, int ninst, int mode, int64_t total, RxArgs a, int64_t rws,
                                                 int max_n1, int max_np1) {
  extern __shared__ double lds[];
  const int rhs = blockIdx.y;
  const int64_t gl = blockIdx.x;
  if (gl >= R.cum_line[ninst]) return;
  const int inst = find_inst(R.cum_line, ninst, gl);
  if (a.conv && a.conv[rhs * ninst + inst]) return;
  const RInst& I = R.inst[inst];
  const int d = I.d, N = I.N, K1 = I.K1, S = I.S, np1 = I.np1, n1 = I.n1, nq = I.nq;
  const int64_t pre = gl - R.cum_line[inst];
  const int nin = mode == RX_CORR ? 2 : 1;
  double* coef = lds;                      // [z][s][max_n1]
  double* fq = lds + 4 * (int64_t)max_n1;  // [s][max_np1]
  double* xr = a.rws + (int64_t)rhs * rws;
  for (int z = 0; z < nin; ++z)
    for (int s = 0; s < S; ++s) {
      const double* in;
      if (d == 1)
        in = plan_in(a, z, (int64_t)rhs * total) + I.seg + (int64_t)s * I.ndof;
      else
        in = xr + I.X_off[d - 1] + (((int64_t)z * S + s) * I.npre[d - 1] + pre) * n1;
      for (int i = threadIdx.x; i < n1; i += blockDim.x) coef[(z * 2 + s) * max_n1 + i] = in[i];
    }
  __syncthreads();
  const double* __restrict__ E = R.E + I.E_off;
  const double* __restrict__ w1 = R.w1 + I.w_off;
  for (int q = threadIdx.x; q < np1; q += blockDim.x) {
    double u[2][2] = {{0.0, 0.0}, {0.0, 0.0}};
    for (int l = 0; l <= N; ++l) {
      const int j = cell_of_level(q, l, N, nq);
      const int o = (l == 0 ? 0 : (K1 << (l - 1))) + j * K1;
      const double* ev = E + ((int64_t)l * np1 + q) * K1;
      for (int p = 0; p < K1; ++p)
        for (int z = 0; z < nin; ++z)
          for (int s = 0; s < S; ++s) u[z][s] += coef[(z * 2 + s) * max_n1 + o + p] * ev[p];
    }
    double out[2];
    if (mode == RX_CORR) {
      double J[2][2];
      rx_jac(I.rx, S, u[0], J);
      if (S == 1) {
        out[0] = u[1][0] / (1.0 - a.dt2 * J[0][0]);
      } else {
        const double A = 1.0 - a.dt2 * J[0][0], B = -a.dt2 * J[0][1];
        const double C = -a.dt2 * J[1][0], D = 1.0 - a.dt2 * J[1][1];
        const double det = A * D - B * C;
        out[0] = (D * u[1][0] - B * u[1][1]) / det;
        out[1] = (A * u[1][1] - C * u[1][0]) / det;
      }
    } else {
      rx_f(I.rx, S, u[0], out);
    }
    for (int s = 0; s < S; ++s) fq[s * max_np1 + q] = w1[q] * out[s];
  }
  __syncthreads();
  for (int i = threadIdx.x; i < n1; i += blockDim.x) {
    const int c1 = i / K1, p = i - c1 * K1;
    const int l = c1 == 0 ? 0 : 32 - __clz(c1);
    const int j = c1 == 0 ? 0 : c1 - (1 << (l - 1));
    const int qs = l == 0 ? 0 : (j << (N - l + 1)) * nq;
    const int qe = l == 0 ? np1 : ((j + 1) << (N - l + 1)) * nq;
    double acc[2] = {0.0, 0.0};
    for (int q = qs; q < qe; ++q) {
      const double ev = E[((int64_t)l * np1 + q) * K1 + p];
      for (int s = 0; s < S; ++s) acc[s] += fq[s * max_np1 + q] * ev;
    }
    for (int s = 0; s < S; ++s) {
      if (d == 1)
        xr[I.Y_off[0] + (int64_t)s * I.ndof + i] = acc[s];
      else
        xr[I.Y_off[d - 1] + ((int64_t)s * I.npre[d - 1] + pre) * n1 + i] = acc[s];
    }
  }
}

// contraction stage m >= 1: Y_m from Y_{m+1}
__global__ __launch_bounds__(256) void k_rx_contract(RTables R, int ninst, int m, RxArgs a, int64_t rws) {
  const int rhs = blockIdx.y;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t* cum = R.cum_y[m];
  if (e >= cum[ninst]) return;
  const int inst = find_inst(cum, ninst, e);
  if (a.conv && a.conv[rhs * ninst + inst]) return;
  const RInst& I = R.inst[inst];
  const int d = I.d, r = d - m, N = I.N, K1 = I.K1, np1 = I.np1, nq = I.nq;
  int64_t le = e - cum[inst];
  const int64_t nout = I.npre[m] * I.gdof[r];
  const int s = (int)(le / nout);
  le -= (int64_t)s * nout;
  const int64_t pre0 = le / I.gdof[r];
  const int64_t eo = le - pre0 * I.gdof[r];
  const RBlk* bb = R.rblk + I.blk_off[r];
  const RBlk B = bb[find_rblk(bb, I.nblk[r], eo)];
  const int64_t L = eo - B.start;
  // sub-block of axes m+1.. in the (r-1)-dim grid
  int lin = 0;
  for (int t = 1; t < r; ++t) lin = lin * (N + 1) + B.lev[t];
  const RBlk Bs = R.rblk[I.blk_off[r - 1] + R.rid[I.id_off[r - 1] + lin]];
  const int64_t Ss = Bs.size;
  const int tm = (int)(L / Ss);
  const int64_t rest = L - (int64_t)tm * Ss;
  const int j = tm / K1, p = tm - j * K1, l = B.lev[0];
  const int qs = l == 0 ? 0 : (j << (N - l + 1)) * nq;
  const int qe = l == 0 ? np1 : ((j + 1) << (N - l + 1)) * nq;
  double* xr = a.rws + (int64_t)rhs * rws;
  const double* __restrict__ in = xr + I.Y_off[m + 1] + ((int64_t)s * I.npre[m + 1] + pre0 * np1) * I.gdof[r - 1] +
                                  Bs.start + rest;
  const double* __restrict__ E = R.E + I.E_off;
  const double* __restrict__ w1 = R.w1 + I.w_off;
  double acc = 0.0;
  for (int q = qs; q < qe; ++q) acc += w1[q] * E[((int64_t)l * np1 + q) * K1 + p] * in[(int64_t)q * I.gdof[r - 1]];
  xr[I.Y_off[m] + ((int64_t)s * I.npre[m] + pre0) * I.gdof[r] + eo] = acc;
}

// final stage over plan chunks: contraction of axis 0 (or pass-through for d = 1) and post-processing
__global__ __launch_bounds__(CHUNK) void k_rx_final(DevTables T, RTables R, int ninst, int nchunks, int mode,
                                                    int64_t total, RxArgs a, int64_t rws) {
  const int c = blockIdx.x, rhs = blockIdx.y, tid = threadIdx.x;
  const Chunk ch = T.chunks[c];
  const int inst = ch.inst, s = ch.species;
  if (a.conv && a.conv[rhs * ninst + inst]) return;
  const RInst& I = R.inst[inst];
  const int d = I.d, N = I.N, K1 = I.K1, np1 = I.np1, nq = I.nq;
  double* xr = a.rws + (int64_t)rhs * rws;
  double acc = 0.0;
  const int64_t g = ch.start + tid;
  if (tid < ch.count) {
    const int64_t eo = g - I.seg - (int64_t)s * I.ndof;
    if (d == 1) {
      acc = xr[I.Y_off[0] + (int64_t)s * I.ndof + eo];
    } else {
      const RBlk* bb = R.rblk + I.blk_off[d];
      const RBlk B = bb[find_rblk(bb, I.nblk[d], eo)];
      const int64_t L = eo - B.start;
      int lin = 0;
      for (int t = 1; t < d; ++t) lin = lin * (N + 1) + B.lev[t];
      const RBlk Bs = R.rblk[I.blk_off[d - 1] + R.rid[I.id_off[d - 1] + lin]];
      const int64_t Ss = Bs.size;
      const int tm = (int)(L / Ss);
      const int64_t rest = L - (int64_t)tm * Ss;
      const int j = tm / K1, p = tm - j * K1, l = B.lev[0];
      const int qs = l == 0 ? 0 : (j << (N - l + 1)) * nq;
      const int qe = l == 0 ? np1 : ((j + 1) << (N - l + 1)) * nq;
      const double* __restrict__ in = xr + I.Y_off[1] + (int64_t)s * I.npre[1] * I.gdof[d - 1] + Bs.start + rest;
      const double* __restrict__ E = R.E + I.E_off;
      const double* __restrict__ w1 = R.w1 + I.w_off;
      for (int q = qs; q < qe; ++q) acc += w1[q] * E[((int64_t)l * np1 + q) * K1 + p] * in[(int64_t)q * I.gdof[d - 1]];
    }
  }
  const int64_t gi = (int64_t)rhs * total + g;
  double g2 = 0.0;
  if (tid < ch.count) {
    if (mode == RX_F) {
      a.F[gi] = acc;
    } else if (mode == RX_RESID) {
      a.F[gi] = acc;
      const double G = a.U[gi] - a.dt2 * acc - a.W[gi];
      a.Gout[gi] = G;
      g2 = G * G;
    } else {
      a.U[gi] -= acc;
    }
  }
  if (mode == RX_RESID) {
    for (int off = 32; off > 0; off >>= 1) g2 += __shfl_xor(g2, off, 64);
    __shared__ double red[CHUNK / 64];
    if ((tid & 63) == 0) red[tid >> 6] = g2;
    __syncthreads();
    if (tid == 0) {
      double t = 0.0;
      for (int w = 0; w < CHUNK / 64; ++w) t += red[w];
      a.part[(int64_t)rhs * nchunks + c] = t;
    }
  }
}

static size_t line_lds_bytes(const RHost* rh) { return (4 * (size_t)rh->max_n1 + 2 * (size_t)rh->max_np1) * sizeof(double); }

static sgdg_status line_lds_attr(const RHost* rh) {
  hipError_t e = hipFuncSetAttribute((const void*)k_rx_line, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)line_lds_bytes(rh));
  if (e != hipSuccess) return hip_fail(e, "hipFuncSetAttribute(line kernel LDS)");
  return SGDG_OK;
}

void reaction_pass(const sgdg_plan* plan, int nrhs, RxMode mode, const RxArgs& a, hipStream_t s) {
  const RHost* rh = (const RHost*)plan->rdata;
  const int d = plan->d, ninst = plan->ninst;
  const int nin = mode == RX_CORR ? 2 : 1;
  for (int m = 0; m + 1 <= d - 1; ++m) {
    const int64_t n = rh->cum_x[m].back();
    if (n == 0) continue;
    hipLaunchKernelGGL(k_rx_expand, dim3((unsigned)((n + 255) / 256), (unsigned)nrhs, (unsigned)nin), dim3(256), 0, s,
                       rh->dev, ninst, m, plan->total, a, rh->rws);
  }
  const size_t lds = line_lds_bytes(rh);
  hipLaunchKernelGGL(k_rx_line, dim3((unsigned)rh->cum_line.back(), (unsigned)nrhs), dim3(256), lds, s, rh->dev, ninst,
                     (int)mode, plan->total, a, rh->rws, rh->max_n1, rh->max_np1);
  for (int m = d - 2; m >= 1; --m) {
    const int64_t n = rh->cum_y[m].back();
    hipLaunchKernelGGL(k_rx_contract, dim3((unsigned)((n + 255) / 256), (unsigned)nrhs), dim3(256), 0, s, rh->dev,
                       ninst, m, a, rh->rws);
  }
  hipLaunchKernelGGL(k_rx_final, dim3((unsigned)plan->nchunks, (unsigned)nrhs), dim3(CHUNK), 0, s, plan->dev, rh->dev,
                     ninst, plan->nchunks, (int)mode, plan->total, a, rh->rws);
}

}  // namespace sgdg
