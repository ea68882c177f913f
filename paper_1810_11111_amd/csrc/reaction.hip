// Reaction term F(U) = P f(R U) at the Gauss points of the finest mesh.
//
// Sec. 5 of the paper: u_h is reconstructed at the Gaussian points of the
// finest-level mesh Omega_N and int f(u_h) v dx is done by that quadrature
// (k+1 Gauss-Legendre points per axis in every finest cell; with this rule
// P R = I on the sparse space).  The paper names the cost of this step as the
// dominant one and points at the special structure of the basis as the way to
// cut it; here that structure is used directly.
//
// R and P = R^T diag(W) are applied axis by axis ("unidirectional"), each
// axis as a batch of independent 1D fibres.  A fibre along axis m with level
// budget L = N - (levels of the other, not yet transformed axes) holds a 1D
// hierarchical vector of levels 0..L:
//   expand  : inverse fast multiwavelet transform to the 2^L level-L cells
//             (two-scale relations), then (k+1)-term evaluation at each of the
//             np1 = (k+1) 2^N Gauss points of the axis;
//   contract: weights, projection of the np1 point values onto the 2^N finest
//             cells, forward fast multiwavelet transform, levels <= L kept.
// Both are O((k+1)^2 n) per fibre and uniform across lanes (a coefficient's
// support is never summed point by point).  Stages: expand axes 0..d-2,
// line kernel on the last axis (expand, pointwise f or per-point species
// Jacobian solve, contract), contract axes d-2..0; the last contraction
// writes plan vectors with the residual / correction post-processing fused.
// One workgroup per fibre (128 lanes; 256 for the lines of the last axis),
// all intermediate work in LDS, the polynomial degree a template constant; every stage
// covers all instances, species and right-hand sides in one launch.
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

constexpr int RX_THREADS_FIB = 128;   // expansion / contraction fibres
constexpr int RX_THREADS_LINE = 256;  // lines of the last axis
constexpr int RX_MAX_N1 = 2048;
constexpr int RX_TAIL = 64 + 16 + 16;  // two-scale matrices + per-wave partial sums + level starts of a fibre

// LDS per workgroup (doubles: buffers of the largest fibre, then the tail).
// The expansion keeps the hierarchical input and two transform buffers; the
// contraction's point values are dead once projected, so its second
// transform buffer takes their place; the line kernel has three buffers per
// transform group and one point buffer per (input, species) pair.
static size_t expand_lds_bytes(const RHost* rh) {
  return (3 * (size_t)rh->max_n1 + RX_TAIL) * sizeof(double);
}
static size_t contract_lds_bytes(const RHost* rh) {
  return (2 * (size_t)rh->max_n1 + RX_TAIL) * sizeof(double);
}
static size_t line_lds_bytes(const RHost* rh, int ngrp, int nin) {
  return (3 * (size_t)ngrp * rh->max_n1 + 2 * (size_t)nin * rh->max_np1 + RX_TAIL) * sizeof(double);
}
// Concurrent transform groups of the line kernel (4, 2 or 1).  More groups
// shorten each line's chain of barriers but take more LDS per workgroup; the
// most that fit the LDS and still let every line of the launch be resident at
// once (when a launch is larger than one wave of workgroups, throughput
// matters more than the length of a line's chain).
static int line_groups(const RHost* rh, int64_t nlines, int nin) {
  int g = 4;
  while (g > 1) {
    const size_t b = line_lds_bytes(rh, g, nin);
    const int64_t per_cu = b <= (size_t)APPLY_LDS_BYTES_HOST ? (int64_t)APPLY_LDS_BYTES_HOST / (int64_t)b : 0;
    if (per_cu > 0 && nlines <= per_cu * std::max(rh->ncu, 1)) break;
    g >>= 1;
  }
  return g;
}
static int line_groups_max(const RHost* rh, int nin) {
  int g = 4;
  while (g > 1 && line_lds_bytes(rh, g, nin) > (size_t)APPLY_LDS_BYTES_HOST) g >>= 1;
  return g;
}
static sgdg_status set_lds_attrs(const RHost* rh);

sgdg_status reaction_build(sgdg_plan* plan) {
  RHost* rh = new RHost();
  plan->rdata = rh;
  const int d = plan->d;
  // A fibre of a whole finest-grid line stays in LDS: (k+1) 2^N <= 2048.
  // Larger plans are still valid for the sweep and the Krylov exponential;
  // their reaction calls report SGDG_ERR_UNSUPPORTED.
  for (const HostInstance& hi : plan->inst)
    if (((hi.desc.k + 1) << hi.desc.n) > RX_MAX_N1) {
      rh->supported = false;
      return SGDG_OK;
    }
  std::vector<RInst> ri;
  std::vector<RBlk> rblk;
  std::vector<int32_t> rid;
  std::vector<double> EL, w1, mats;
  int64_t ws = 0;
  rh->cum_x.assign(d, std::vector<int64_t>(1, 0));
  rh->cum_y.assign(d, std::vector<int64_t>(1, 0));
  rh->cum_line.assign(1, 0);
  rh->cum_fin.assign(1, 0);
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
    std::vector<double> xg, wg;
    gauss01(r.nq, xg, wg);
    const Basis1D& bs = basis1d(hi.desc.k);
    const double h = std::ldexp(1.0, -N);
    r.EL_off = (int64_t)EL.size();
    r.w_off = (int64_t)w1.size();
    r.mats_off = (int64_t)mats.size();
    for (int q = 0; q < r.np1; ++q) w1.push_back(wg[q % r.nq] * h);
    // level-L cell basis 2^(L/2) phi_p(2^L x - c) at the finest Gauss points
    double phi[16];
    for (int L = 0; L <= N; ++L)
      for (int q = 0; q < r.np1; ++q) {
        const int cellN = q / r.nq;
        const int cL = cellN >> (N - L);
        const double xloc = ((cellN - ((int64_t)cL << (N - L))) + xg[q % r.nq]) * std::ldexp(1.0, L - N);
        legendre01_all(hi.desc.k, xloc, phi, nullptr);
        for (int p = 0; p < K1; ++p) EL.push_back(std::sqrt(std::ldexp(1.0, L)) * phi[p]);
      }
    // two-scale matrices, rows padded to 16 entries each
    const std::vector<double>* src[4] = {&bs.ML, &bs.MR, &bs.cL, &bs.cR};
    for (int t = 0; t < 4; ++t) {
      std::vector<double> pad(16, 0.0);
      std::copy(src[t]->begin(), src[t]->end(), pad.begin());
      mats.insert(mats.end(), pad.begin(), pad.end());
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
    // fibres: expansion/contraction stage m runs over (species, prefix, column of the (d-m-1)-dim grid)
    for (int m = 0; m + 1 <= d - 1; ++m)
      rh->cum_x[m].push_back(rh->cum_x[m].back() + (int64_t)S * r.npre[m] * r.gdof[d - m - 1]);
    for (int m = 1; m + 1 <= d - 1; ++m)
      rh->cum_y[m].push_back(rh->cum_y[m].back() + (int64_t)S * r.npre[m] * r.gdof[d - m - 1]);
    rh->cum_line.push_back(rh->cum_line.back() + r.npre[d - 1]);
    rh->cum_fin.push_back(rh->cum_fin.back() + (d >= 2 ? (int64_t)S * r.gdof[d - 1] : 1));
    ri.push_back(r);
  }
  rh->rws = ws;
  sgdg_status st;
  if ((st = up(plan, ri, &rh->dev.inst)) != SGDG_OK || (st = up(plan, rblk, &rh->dev.rblk)) != SGDG_OK ||
      (st = up(plan, rid, &rh->dev.rid)) != SGDG_OK || (st = up(plan, EL, &rh->dev.EL)) != SGDG_OK ||
      (st = up(plan, w1, &rh->dev.w1)) != SGDG_OK || (st = up(plan, mats, &rh->dev.mats)) != SGDG_OK ||
      (st = up(plan, rh->cum_line, &rh->dev.cum_line)) != SGDG_OK ||
      (st = up(plan, rh->cum_fin, &rh->dev.cum_fin)) != SGDG_OK)
    return st;
  for (int m = 0; m < d; ++m) {
    if ((st = up(plan, rh->cum_x[m], &rh->dev.cum_x[m])) != SGDG_OK) return st;
    if ((st = up(plan, rh->cum_y[m], &rh->dev.cum_y[m])) != SGDG_OK) return st;
  }
  if (hipDeviceGetAttribute(&rh->ncu, hipDeviceAttributeMultiprocessorCount, plan->device) != hipSuccess) {
    rh->ncu = 0;
    (void)hipGetLastError();
  }
  return set_lds_attrs(rh);
}

void reaction_destroy(sgdg_plan* plan) {
  delete (RHost*)plan->rdata;
  plan->rdata = nullptr;
}

int64_t reaction_ws_doubles(const sgdg_plan* plan) { return ((const RHost*)plan->rdata)->rws; }
bool reaction_supported(const sgdg_plan* plan) { return ((const RHost*)plan->rdata)->supported; }
int64_t reaction_final_fibres(const sgdg_plan* plan) {
  const RHost* rh = (const RHost*)plan->rdata;
  return rh->supported ? rh->cum_fin.back() : 0;
}

// ---------------------------------------------------------------- device helpers

// the instance of work item e from the ascending first items cum[0..ninst)
// (one round of loads per 64 instances, as in find_rblk)
__device__ __forceinline__ int find_inst(const int64_t* __restrict__ cum, int ninst, int64_t e) {
  if (ninst == 1) return 0;  // no table load for single-instance plans
  const int lane = threadIdx.x & 63;
  int best = 0;
  for (int t0 = 0; t0 < ninst; t0 += 64) {
    const int t = min(t0 + lane, ninst - 1);
    const bool ok = t0 + lane < ninst && cum[t] <= e;
    const unsigned long long mk = __ballot(ok);
    if (mk) best = t0 + 63 - __clzll(mk);
  }
  return best;
}

// the block of b[0..n) (ascending starts) holding element e: every lane of
// the wave tests one block per round of 64, so the search costs one round of
// loads (the starts at or below e are a prefix; the last of them wins)
__device__ __forceinline__ int find_rblk(const RBlk* __restrict__ b, int n, int64_t e) {
  const int lane = threadIdx.x & 63;
  int best = 0;
  for (int t0 = 0; t0 < n; t0 += 64) {
    const int t = min(t0 + lane, n - 1);
    const bool ok = t0 + lane < n && b[t].start <= e;
    const unsigned long long mk = __ballot(ok);
    if (mk) best = t0 + 63 - __clzll(mk);
  }
  return best;
}

// a[m] for a small kernel-argument array without a dynamic index (which would
// move the argument struct to scratch memory)
__device__ __forceinline__ const int64_t* pick(const int64_t* const (&a)[SGDG_MAX_D], int m) {
  const int64_t* r = a[0];
#pragma unroll
  for (int i = 1; i < SGDG_MAX_D; ++i)
    if (m == i) r = a[i];
  return r;
}

__device__ __forceinline__ int off1(int l, int K1) { return l == 0 ? 0 : (K1 << (l - 1)); }

// two-scale matrices in LDS: M[0..15] ML[q][i] (child q from parent i), M[16..] MR,
// M[32..] cL[p][q] (wavelet p on left child basis q), M[48..] cR; row length K1
__device__ __forceinline__ void load_mats(const RTables& R, const RInst& I, double* M) {
  for (int e = threadIdx.x; e < 64; e += blockDim.x) M[e] = R.mats[I.mats_off + e];
}

// inverse fast multiwavelet transform: hierarchical levels 0..L in h -> level-L
// cell-Legendre coefficients (returned pointer, one of b0 / b1)
// The transforms below are run by a group of nt threads with local index tid
// (by default the whole workgroup); every thread of the workgroup passes the
// same barriers, and a thread with tid >= any loop bound takes part in the
// barriers only.
template <int K1>
__device__ __forceinline__ double* ifwt(const double* h, double* b0, double* b1, int L, const double* M,
                                        int tid = threadIdx.x, int nt = blockDim.x) {
  for (int e = tid; e < K1; e += nt) b0[e] = h[e];
  __syncthreads();
  double* cur = b0;
  double* nxt = b1;
  int n = 1;
  // coarse levels two per barrier while level n+1 has at most one item per
  // thread: the thread forms the K1 level-n values of its item's parent cell
  // (the sums of the one-level pass, in the same order), then its item
  for (; n + 1 <= L && (K1 << (n + 1)) <= nt; n += 2) {
    const double* dw1 = h + (K1 << (n - 1));
    const double* dw2 = h + (K1 << n);
    const int e = tid;
    if (e < (K1 << (n + 1))) {
      const int c = e / K1, q = e - c * K1, c1 = c >> 1, j = c1 >> 1;
      const double* M1 = (c1 & 1) ? M + 16 : M;
      const double* W1 = (c1 & 1) ? M + 48 : M + 32;
      double pv[K1];
#pragma unroll
      for (int q1 = 0; q1 < K1; ++q1) {
        double a = 0.0;
#pragma unroll
        for (int i = 0; i < K1; ++i) a += M1[q1 * K1 + i] * cur[j * K1 + i];
#pragma unroll
        for (int p = 0; p < K1; ++p) a += W1[p * K1 + q1] * dw1[j * K1 + p];
        pv[q1] = a;
      }
      const double* M2 = (c & 1) ? M + 16 : M;
      const double* W2 = (c & 1) ? M + 48 : M + 32;
      double acc = 0.0;
#pragma unroll
      for (int i = 0; i < K1; ++i) acc += M2[q * K1 + i] * pv[i];
#pragma unroll
      for (int p = 0; p < K1; ++p) acc += W2[p * K1 + q] * dw2[c1 * K1 + p];
      nxt[e] = acc;
    }
    __syncthreads();
    double* t = cur;
    cur = nxt;
    nxt = t;
  }
  for (; n <= L; ++n) {
    const double* dw = h + (K1 << (n - 1));
    const int items = (K1 << n);
    for (int e = tid; e < items; e += nt) {
      const int c = e / K1, q = e - c * K1, j = c >> 1;
      const double* Mq = (c & 1) ? M + 16 : M;
      const double* Wq = (c & 1) ? M + 48 : M + 32;
      double acc = 0.0;
#pragma unroll
      for (int i = 0; i < K1; ++i) acc += Mq[q * K1 + i] * cur[j * K1 + i];
#pragma unroll
      for (int p = 0; p < K1; ++p) acc += Wq[p * K1 + q] * dw[j * K1 + p];
      nxt[e] = acc;
    }
    __syncthreads();
    double* t = cur;
    cur = nxt;
    nxt = t;
  }
  return cur;
}

// forward fast multiwavelet transform of level-N cell coefficients in s (s and
// tmp are overwritten); emit(level, j, p, value) receives every hierarchical
// coefficient (wavelets of levels N..1, then level 0).
template <int K1, class Emit>
__device__ __forceinline__ void ffwt(double* s, double* tmp, int N, const double* M, Emit emit, int tid = threadIdx.x,
                                     int nt = blockDim.x) {
  double* cur = s;
  double* nxt = tmp;
  for (int n = N; n >= 1; --n) {
    const int npar = 1 << (n - 1);
    const int half = npar * K1;
    for (int e = tid; e < 2 * half; e += nt) {
      const int w = e >= half;
      const int e2 = e - w * half;
      const int j = e2 / K1, i = e2 - j * K1;
      const double* sl = cur + (2 * j) * K1;
      const double* sr = sl + K1;
      double acc = 0.0;
      if (!w) {
#pragma unroll
        for (int q = 0; q < K1; ++q) acc += M[q * K1 + i] * sl[q] + M[16 + q * K1 + i] * sr[q];
        nxt[j * K1 + i] = acc;
      } else {
#pragma unroll
        for (int q = 0; q < K1; ++q) acc += M[32 + i * K1 + q] * sl[q] + M[48 + i * K1 + q] * sr[q];
        emit(n, j, i, acc);
      }
    }
    __syncthreads();
    double* t = cur;
    cur = nxt;
    nxt = t;
  }
  for (int e = tid; e < K1; e += nt) emit(0, 0, e, cur[e]);
  __syncthreads();
}

// value at finest point q of the level-L cell expansion s (K1 Gauss points per cell)
template <int K1>
__device__ __forceinline__ double eval_pt(const double* s, const double* __restrict__ EL, int L, int N, int np1, int q) {
  const int c = (q / K1) >> (N - L);
  const double* e = EL + ((int64_t)L * np1 + q) * K1;
  double u = 0.0;
#pragma unroll
  for (int p = 0; p < K1; ++p) u += s[c * K1 + p] * e[p];
  return u;
}

// weighted point values g (weights already applied) -> level-N cell coefficients in out
template <int K1>
__device__ __forceinline__ void project_cells(const double* g, const double* __restrict__ EL, int N, int np1,
                                              double* out, int tid = threadIdx.x, int nt = blockDim.x) {
  const int ncell = 1 << N;
  const double* e = EL + (int64_t)N * np1 * K1;
  for (int t = tid; t < ncell * K1; t += nt) {
    const int c = t / K1, p = t - c * K1;
    double acc = 0.0;
#pragma unroll
    for (int gq = 0; gq < K1; ++gq) acc += g[c * K1 + gq] * e[(c * K1 + gq) * K1 + p];
    out[t] = acc;
  }
  __syncthreads();
}

__device__ __forceinline__ const double* plan_in(const RxArgs& a, int z, int64_t rhs_total) {
  return (z == 0 ? (const double*)a.U : a.G) + rhs_total;
}

__device__ __forceinline__ void rx_f(const double (*c)[4][4], int S, const double* u, double* f) {
  const double u0 = u[0], u1 = S > 1 ? u[1] : 0.0;
  const double p0[4] = {1.0, u0, u0 * u0, u0 * u0 * u0};
  const double p1[4] = {1.0, u1, u1 * u1, u1 * u1 * u1};
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    double acc = 0.0;
    if (s < S)
#pragma unroll
      for (int aa = 0; aa < 4; ++aa)
#pragma unroll
        for (int bb = 0; bb < 4; ++bb) acc += c[s][aa][bb] * p0[aa] * p1[bb];
    f[s] = acc;
  }
}

__device__ __forceinline__ void rx_jac(const double (*c)[4][4], int S, const double* u, double J[2][2]) {
  const double u0 = u[0], u1 = S > 1 ? u[1] : 0.0;
  const double p0[4] = {1.0, u0, u0 * u0, u0 * u0 * u0};
  const double p1[4] = {1.0, u1, u1 * u1, u1 * u1 * u1};
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    double j0 = 0.0, j1 = 0.0;
    if (s < S)
#pragma unroll
      for (int aa = 0; aa < 4; ++aa)
#pragma unroll
        for (int bb = 0; bb < 4; ++bb) {
          if (aa > 0) j0 += c[s][aa][bb] * aa * p0[aa - 1] * p1[bb];
          if (bb > 0) j1 += c[s][aa][bb] * bb * p0[aa] * p1[bb - 1];
        }
    J[s][0] = j0;
    J[s][1] = j1;
  }
}

// post-processing of one output coefficient of the final stage; returns G^2 (RESID) or 0
__device__ __forceinline__ double finish(const RxArgs& a, int mode, int64_t gi, double v) {
  if (mode == RX_F) {
    a.F[gi] = v;
  } else if (mode == RX_RESID) {
    a.F[gi] = v;
    const double G = a.U[gi] - a.dt2 * v - a.W[gi];
    a.Gout[gi] = G;
    return G * G;
  } else if (mode == RX_LOCAL) {
    a.Gout[gi] = v;
  } else {
    a.U[gi] -= v;
  }
  return 0.0;
}

// Sum over the workgroup in a fixed order (wave sums, then waves in index
// order); the result is valid in thread 0.  wsum: LDS scratch of one double
// per wave.
__device__ __forceinline__ double block_sum(double v, double* wsum) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  const int w = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
  if ((threadIdx.x & 63) == 0) wsum[w] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0)
    for (int i = 0; i < nw; ++i) t += wsum[i];
  return t;
}

// ---------------------------------------------------------------- kernels

// expansion stage m: fibres along axis m, grid (fibres, rhs, input)
template <int K1>
__device__ void rx_expand_body(const RTables& R, int inst, int m, int64_t total, const RxArgs& a, int64_t rws,
                               int max_n1, double* lds) {
  const int z = blockIdx.z, rhs = blockIdx.y;
  const int64_t f = blockIdx.x;
  const int64_t* cum = pick(R.cum_x, m);
  const RInst& I = R.inst[inst];
  const int d = I.d, r = d - m, N = I.N, S = I.S, np1 = I.np1;
  int64_t le = f - cum[inst];
  const int64_t gd_in = I.gdof[r], gd_out = I.gdof[r - 1];
  const int64_t per_s = I.npre[m] * gd_out;
  const int s = (int)(le / per_s);
  le -= (int64_t)s * per_s;
  const int64_t pre0 = le / gd_out;
  const int64_t eo = le - pre0 * gd_out;
  const RBlk* ob = R.rblk + I.blk_off[r - 1];
  const RBlk& B = ob[find_rblk(ob, I.nblk[r - 1], eo)];
  const int64_t rest = eo - B.start, Sb = B.size;
  const int L = N - B.lsum;
  int lin = 0, pw = 1;
  for (int t = r - 2; t >= 0; --t) {
    lin += B.lev[t] * pw;
    pw *= (N + 1);
  }
  double* h = lds;
  double* b0 = lds + max_n1;
  double* b1 = lds + 2 * max_n1;
  double* M = lds + 3 * max_n1;
  const int32_t* __restrict__ id = R.rid + I.id_off[r];
  const RBlk* ib = R.rblk + I.blk_off[r];
  double* xr = a.rws + (int64_t)rhs * rws;
  const double* __restrict__ in =
      m == 0 ? plan_in(a, z, (int64_t)rhs * total) + I.seg + (int64_t)s * I.ndof
             : xr + I.X_off[m] + (((int64_t)z * S + s) * I.npre[m] + pre0) * gd_in;
  double* out = xr + I.X_off[m + 1] + (((int64_t)z * S + s) * I.npre[m + 1] + pre0 * np1) * gd_out + eo;
  const double* __restrict__ EL = R.EL + I.EL_off;
  // start of the fibre's level-l block (l <= L), one thread per level, then
  // every entry of every level is loaded in one round
  int64_t* lb = (int64_t*)(M + 80);
  if ((int)threadIdx.x <= L) lb[threadIdx.x] = ib[id[threadIdx.x * pw + lin]].start + rest;
  load_mats(R, I, M);
  __syncthreads();
  for (int e = threadIdx.x; e < (K1 << L); e += blockDim.x) {
    const int l = e < K1 ? 0 : 32 - __clz(e / K1);  // entry e of levels 0..L in hierarchical order
    h[e] = in[lb[l] + (int64_t)(e - off1(l, K1)) * Sb];
  }
  __syncthreads();
  const double* sc = ifwt<K1>(h, b0, b1, L, M);
  for (int q = threadIdx.x; q < np1; q += blockDim.x) out[(int64_t)q * gd_out] = eval_pt<K1>(sc, EL, L, N, np1, q);
}

__global__ __launch_bounds__(RX_THREADS_FIB) void k_rx_expand(RTables R, int ninst, int m, int64_t total, RxArgs a,
                                                              int64_t rws, int max_n1) {
  extern __shared__ double lds[];
  const int inst = find_inst(pick(R.cum_x, m), ninst, blockIdx.x);
  if (a.conv && a.conv[blockIdx.y * ninst + inst]) return;
  switch (R.inst[inst].K1) {
    case 2: rx_expand_body<2>(R, inst, m, total, a, rws, max_n1, lds); break;
    case 3: rx_expand_body<3>(R, inst, m, total, a, rws, max_n1, lds); break;
    default: rx_expand_body<4>(R, inst, m, total, a, rws, max_n1, lds); break;
  }
}

// one workgroup per line of the last axis: expand (all species and inputs),
// pointwise map, contract; for d = 1 the line is the whole instance and the
// plan vectors are read and finished directly
template <int K1>
__device__ void rx_line_body(const RTables& R, int inst, int mode, int64_t total, const RxArgs& a, int64_t rws,
                             int max_n1, int max_np1, int64_t nfin, int ngrp, double* lds) {
  const int rhs = blockIdx.y;
  const int64_t gl = blockIdx.x;
  const RInst& I = R.inst[inst];
  const int d = I.d, N = I.N, S = I.S, np1 = I.np1, n1 = I.n1;
  const int64_t pre = gl - R.cum_line[inst];
  const int nin = mode == RX_CORR ? 2 : 1;
  // up to ngrp groups of threads transform different (input, species) lines
  // at the same time, each in its own three buffers (no more groups than
  // lines, so that each group is as large as possible)
  const int npair = nin * S;
  const int ng = min(ngrp, npair);
  const int gs = blockDim.x / ng, gi = threadIdx.x / gs, gt = threadIdx.x - gi * gs;
  double* h = lds + (int64_t)gi * 3 * max_n1;
  double* b0 = h + max_n1;
  double* b1 = b0 + max_n1;
  double* pts = lds + (int64_t)ngrp * 3 * max_n1;  // [z*2+s][max_np1], z < nin
  double* M = pts + 2 * nin * max_np1;
  double* wsum = M + 64;
  double* xr = a.rws + (int64_t)rhs * rws;
  const double* __restrict__ EL = R.EL + I.EL_off;
  const double* __restrict__ w1 = R.w1 + I.w_off;
  const double dt2 = a.dt2;
  load_mats(R, I, M);
  for (int r0 = 0; r0 < npair; r0 += ng) {
    const int pi = r0 + gi;
    const bool act = pi < npair;
    const int z = act ? pi / S : 0, s = act ? pi - z * S : 0;
    const int lt = act ? gt : (1 << 30);  // an idle group passes the barriers only
    const double* in = d == 1 ? plan_in(a, z, (int64_t)rhs * total) + I.seg + (int64_t)s * I.ndof
                              : xr + I.X_off[d - 1] + (((int64_t)z * S + s) * I.npre[d - 1] + pre) * n1;
    for (int i = lt; i < n1; i += gs) h[i] = in[i];
    __syncthreads();
    const double* sc = ifwt<K1>(h, b0, b1, N, M, lt, gs);
    double* pz = pts + (z * 2 + s) * max_np1;
    for (int q = lt; q < np1; q += gs) pz[q] = eval_pt<K1>(sc, EL, N, N, np1, q);
    __syncthreads();
  }
  for (int q = threadIdx.x; q < np1; q += blockDim.x) {
    double u[2] = {pts[q], S > 1 ? pts[max_np1 + q] : 0.0};
    double out[2];
    if (mode == RX_CORR) {
      const double g0 = pts[2 * max_np1 + q], g1 = S > 1 ? pts[3 * max_np1 + q] : 0.0;
      double J[2][2];
      rx_jac(I.rx, S, u, J);
      if (S == 1) {
        out[0] = g0 / (1.0 - dt2 * J[0][0]);
      } else {
        const double A = 1.0 - dt2 * J[0][0], Bq = -dt2 * J[0][1];
        const double C = -dt2 * J[1][0], D = 1.0 - dt2 * J[1][1];
        const double det = A * D - Bq * C;
        out[0] = (D * g0 - Bq * g1) / det;
        out[1] = (A * g1 - C * g0) / det;
      }
    } else if (mode == RX_LOCAL) {
      // u - dt2 f(u) = w at this point, Newton from u = w (at most RX_LOCAL_MAX_ITER corrections)
      const double w0 = u[0], w1v = u[1];
      const double wmag = fmax(1.0, fmax(fabs(w0), fabs(w1v)));
      double x[2] = {w0, w1v};
      for (int it = 0; it <= RX_LOCAL_MAX_ITER; ++it) {
        double f[2];
        rx_f(I.rx, S, x, f);
        const double g0 = x[0] - dt2 * f[0] - w0, g1 = S > 1 ? x[1] - dt2 * f[1] - w1v : 0.0;
        if (fmax(fabs(g0), fabs(g1)) <= RX_LOCAL_TOL * wmag || it == RX_LOCAL_MAX_ITER) break;
        double J[2][2];
        rx_jac(I.rx, S, x, J);
        if (S == 1) {
          x[0] -= g0 / (1.0 - dt2 * J[0][0]);
        } else {
          const double A = 1.0 - dt2 * J[0][0], Bq = -dt2 * J[0][1];
          const double C = -dt2 * J[1][0], D = 1.0 - dt2 * J[1][1];
          const double det = A * D - Bq * C;
          x[0] -= (D * g0 - Bq * g1) / det;
          x[1] -= (A * g1 - C * g0) / det;
        }
      }
      out[0] = x[0];
      out[1] = x[1];
    } else {
      rx_f(I.rx, S, u, out);
    }
    pts[q] = w1[q] * out[0];
    if (S > 1) pts[max_np1 + q] = w1[q] * out[1];
  }
  __syncthreads();
  double g2 = 0.0;
  // contraction: the species at the same time when there are groups enough
  const int cg = min(ng, S);
  const int cgs = blockDim.x / cg, cgi = threadIdx.x / cgs, cgt = threadIdx.x - cgi * cgs;
  double* c0 = lds + (int64_t)cgi * 3 * max_n1;
  double* c1 = c0 + max_n1;
  for (int r0 = 0; r0 < S; r0 += cg) {
    const int s = r0 + cgi;
    const bool act = s < S;
    const int lt = act ? cgt : (1 << 30);
    const int sp = act ? s : 0;
    project_cells<K1>(pts + sp * max_np1, EL, N, np1, c0, lt, cgs);
    if (d == 1) {
      const int64_t base = (int64_t)rhs * total + I.seg + (int64_t)sp * I.ndof;
      ffwt<K1>(c0, c1, N, M, [&](int n, int j, int p, double v) {
        g2 += finish(a, mode, base + off1(n, K1) + j * K1 + p, v);
      }, lt, cgs);
    } else {
      double* out = xr + I.Y_off[d - 1] + ((int64_t)sp * I.npre[d - 1] + pre) * n1;
      ffwt<K1>(c0, c1, N, M, [&](int n, int j, int p, double v) { out[off1(n, K1) + j * K1 + p] = v; }, lt, cgs);
    }
  }
  if (d == 1 && mode == RX_RESID) {
    g2 = block_sum(g2, wsum);
    if (threadIdx.x == 0) a.part[(int64_t)rhs * nfin + R.cum_fin[inst]] = g2;
  }
}

__global__ __launch_bounds__(RX_THREADS_LINE) void k_rx_line(RTables R, int ninst, int mode, int64_t total, RxArgs a,
                                                             int64_t rws, int max_n1, int max_np1, int64_t nfin,
                                                             int ngrp) {
  extern __shared__ double lds[];
  const int inst = find_inst(R.cum_line, ninst, blockIdx.x);
  if (a.conv && a.conv[blockIdx.y * ninst + inst]) return;
  switch (R.inst[inst].K1) {
    case 2: rx_line_body<2>(R, inst, mode, total, a, rws, max_n1, max_np1, nfin, ngrp, lds); break;
    case 3: rx_line_body<3>(R, inst, mode, total, a, rws, max_n1, max_np1, nfin, ngrp, lds); break;
    default: rx_line_body<4>(R, inst, mode, total, a, rws, max_n1, max_np1, nfin, ngrp, lds); break;
  }
}

// contraction stage m (m >= 1 writes Y_m; m == 0 finishes plan vectors)
template <int K1>
__device__ void rx_contract_body(const RTables& R, int inst, int m, int mode, int64_t total, const RxArgs& a,
                                 int64_t rws, int max_n1, int64_t nfin, double* lds) {
  const int rhs = blockIdx.y;
  const int64_t f = blockIdx.x;
  const int64_t* cum = m == 0 ? R.cum_fin : pick(R.cum_y, m);
  const RInst& I = R.inst[inst];
  const int d = I.d, r = d - m, N = I.N, np1 = I.np1;
  int64_t le = f - cum[inst];
  const int64_t gd_in = I.gdof[r - 1], gd_out = I.gdof[r];
  const int64_t per_s = I.npre[m] * gd_in;
  const int s = (int)(le / per_s);
  le -= (int64_t)s * per_s;
  const int64_t pre0 = le / gd_in;
  const int64_t eo = le - pre0 * gd_in;
  const RBlk* ob = R.rblk + I.blk_off[r - 1];
  const RBlk& B = ob[find_rblk(ob, I.nblk[r - 1], eo)];
  const int64_t rest = eo - B.start, Sb = B.size;
  const int L = N - B.lsum;
  int lin = 0, pw = 1;
  for (int t = r - 2; t >= 0; --t) {
    lin += B.lev[t] * pw;
    pw *= (N + 1);
  }
  double* g = lds;
  double* b0 = lds + max_n1;
  double* b1 = lds;  // the point values are dead once projected into b0
  double* M = lds + 2 * max_n1;
  double* wsum = M + 64;
  double* xr = a.rws + (int64_t)rhs * rws;
  const double* __restrict__ EL = R.EL + I.EL_off;
  const double* __restrict__ w1 = R.w1 + I.w_off;
  // start of the output's level-n block (n <= L), one thread per level,
  // before the transform needs them
  const int32_t* __restrict__ id = R.rid + I.id_off[r];
  const RBlk* ib = R.rblk + I.blk_off[r];
  int64_t* lb = (int64_t*)(M + 80);
  if ((int)threadIdx.x <= L) lb[threadIdx.x] = ib[id[threadIdx.x * pw + lin]].start;
  load_mats(R, I, M);
  const double* __restrict__ in = xr + I.Y_off[m + 1] + ((int64_t)s * I.npre[m + 1] + pre0 * np1) * gd_in + eo;
  for (int q = threadIdx.x; q < np1; q += blockDim.x) g[q] = w1[q] * in[(int64_t)q * gd_in];
  __syncthreads();
  project_cells<K1>(g, EL, N, np1, b0);
  if (m > 0) {
    double* out = xr + I.Y_off[m] + ((int64_t)s * I.npre[m] + pre0) * gd_out + rest;
    ffwt<K1>(b0, b1, N, M, [&](int n, int j, int p, double v) {
      if (n <= L) out[lb[n] + (int64_t)(j * K1 + p) * Sb] = v;
    });
  } else {
    const int64_t base = (int64_t)rhs * total + I.seg + (int64_t)s * I.ndof + rest;
    double g2 = 0.0;
    ffwt<K1>(b0, b1, N, M, [&](int n, int j, int p, double v) {
      if (n <= L) g2 += finish(a, mode, base + lb[n] + (int64_t)(j * K1 + p) * Sb, v);
    });
    if (mode == RX_RESID) {
      g2 = block_sum(g2, wsum);
      if (threadIdx.x == 0) a.part[(int64_t)rhs * nfin + f] = g2;
    }
  }
}

__global__ __launch_bounds__(RX_THREADS_FIB) void k_rx_contract(RTables R, int ninst, int m, int mode, int64_t total,
                                                                RxArgs a, int64_t rws, int max_n1, int64_t nfin) {
  extern __shared__ double lds[];
  const int inst = find_inst(m == 0 ? R.cum_fin : pick(R.cum_y, m), ninst, blockIdx.x);
  if (a.conv && a.conv[blockIdx.y * ninst + inst]) return;
  switch (R.inst[inst].K1) {
    case 2: rx_contract_body<2>(R, inst, m, mode, total, a, rws, max_n1, nfin, lds); break;
    case 3: rx_contract_body<3>(R, inst, m, mode, total, a, rws, max_n1, nfin, lds); break;
    default: rx_contract_body<4>(R, inst, m, mode, total, a, rws, max_n1, nfin, lds); break;
  }
}

static sgdg_status set_lds_attrs(const RHost* rh) {
  size_t lmax = 0;
  for (int nin = 1; nin <= 2; ++nin) lmax = std::max(lmax, line_lds_bytes(rh, line_groups_max(rh, nin), nin));
  hipError_t e = hipFuncSetAttribute((const void*)k_rx_line, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lmax);
  if (e == hipSuccess)
    e = hipFuncSetAttribute((const void*)k_rx_expand, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)expand_lds_bytes(rh));
  if (e == hipSuccess)
    e = hipFuncSetAttribute((const void*)k_rx_contract, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)contract_lds_bytes(rh));
  if (e != hipSuccess) return hip_fail(e, "hipFuncSetAttribute(reaction kernels LDS)");
  return SGDG_OK;
}

void reaction_pass(const sgdg_plan* plan, int nrhs, RxMode mode, const RxArgs& a, hipStream_t s) {
  const RHost* rh = (const RHost*)plan->rdata;
  const int d = plan->d, ninst = plan->ninst;
  const int nin = mode == RX_CORR ? 2 : 1;
  const int ngrp = std::min(line_groups(rh, rh->cum_line.back() * nrhs, nin), line_groups_max(rh, nin));
  const size_t el = expand_lds_bytes(rh), cl = contract_lds_bytes(rh), ll = line_lds_bytes(rh, ngrp, nin);
  const int64_t nfin = rh->cum_fin.back();
  for (int m = 0; m + 1 <= d - 1; ++m)
    hipLaunchKernelGGL(k_rx_expand, dim3((unsigned)rh->cum_x[m].back(), (unsigned)nrhs, (unsigned)nin),
                       dim3(RX_THREADS_FIB), el, s, rh->dev, ninst, m, plan->total, a, rh->rws, rh->max_n1);
  hipLaunchKernelGGL(k_rx_line, dim3((unsigned)rh->cum_line.back(), (unsigned)nrhs), dim3(RX_THREADS_LINE), ll, s, rh->dev,
                     ninst, (int)mode, plan->total, a, rh->rws, rh->max_n1, rh->max_np1, nfin, ngrp);
  for (int m = d - 2; m >= 0; --m) {
    const int64_t nf = m == 0 ? nfin : rh->cum_y[m].back();
    hipLaunchKernelGGL(k_rx_contract, dim3((unsigned)nf, (unsigned)nrhs), dim3(RX_THREADS_FIB), cl, s, rh->dev, ninst, m,
                       (int)mode, plan->total, a, rh->rws, rh->max_n1, nfin);
  }
}

}  // namespace sgdg
