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
// hierarchical vector of levels 0..L.  Stages: expand axes 0..d-2, a line
// kernel on the last axis (expand, pointwise f or per-point species Jacobian
// solve, contract), contract axes d-2..0; the last contraction writes plan
// vectors with the residual / correction post-processing fused.  Every stage
// covers all instances, species and right-hand sides in one launch, and the
// polynomial degree is a template constant.
//
// Expansion and contraction stages (one thread per fibre, no LDS, no
// barriers).  A point q of the axis lies in exactly one cell of every level,
// so a fibre's value there is sum over levels l <= L and p of
// v_{l,j(q,l),p}(x_q) c_{l,j,p}: each thread walks the points of its fibre
// in order, holding the coefficients of the current cell of every level in
// registers (reloaded when a cell boundary is crossed) and reading the basis
// values from a per-instance table.  The contraction is the transpose: it
// accumulates w_q v(x_q) g_q into one running sum per level and emits a
// cell's coefficients when the walk leaves the cell.  Consecutive threads
// take consecutive fibres, which sit at consecutive addresses of both the
// hierarchical and the point-valued arrays, so every load and store is
// coalesced.  Small stages split each fibre's points into 2^lam chunks
// (threads of one fibre in one wave); the contraction then combines the
// partial sums of the coarse levels across the chunks with a fixed-order
// butterfly.
//
// Last axis (one workgroup per tile of whole lines, all inputs and species
// staged in LDS): inverse fast multiwavelet transform of every line in place
// (two-scale relations, all lines of the tile in the same barrier step), the
// pointwise map cell by cell (point values from the finest-level cell
// coefficients, map, projection back), and the forward transform in place.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <functional>
#include <numeric>
#include <type_traits>

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

constexpr int RX_THREADS = 256;        // every reaction kernel
constexpr int RX_MAX_N1 = 2048;        // (k+1) 2^N per axis
constexpr int RX_LMAX = 11;            // levels 0..10 (k >= 1, (k+1) 2^N <= 2048)
constexpr int RX_LINE_LDS = 32 * 1024; // LDS budget of a line tile (several tiles per compute unit)
constexpr int RX_ITEMS = 2;            // transform items per thread of a line tile at the finest level
constexpr int RX_TAIL = 64 + 32 + 8;   // two-scale matrices, reaction coefficients, per-wave partial sums
constexpr int64_t RX_THREADS_WANTED = 1 << 17;
constexpr int RX_WALK = 64;  // most points one thread of an expansion / contraction walks
constexpr int RX_XS_LDS = 32 * 1024;  // largest hierarchical block an expansion / contraction tile stages in LDS
constexpr int RX_WLINE_MAXN = 8;   // last-axis wave form: lines of at most 64 lanes (N <= 8 at k = 1)
constexpr int RX_WLINE_ROUNDS = 16;    // its default tiles: at most 16 rounds of one line per wave (more for N < 6)
constexpr int RX_WLINE_MAXROUNDS = 64; // the most rounds a tile may take (autotuning)

// LDS of the last-axis kernel: per line 2.5 npair n1 doubles (inputs, and the
// two scaling buffers of the transforms), plus the tail
static int64_t line_doubles(int npair, int n1) { return (int64_t)5 * npair * (n1 / 2); }
static size_t line_tile_doubles(int npair, int nl, int n1, int K1) {
  return (size_t)line_doubles(npair, n1) * nl + RX_TAIL + (size_t)n1 * (K1 + 1);
}
static sgdg_status set_line_lds(const RHost* rh);

// Tiles of the wave-form last-axis kernel: `rounds` rounds of each
// instance's lines per round, instance by instance.
static std::vector<LineTask> wave_tiles(const LineClass& lc, int rounds) {
  std::vector<LineTask> t;
  for (const WaveLines& il : lc.lines) {
    const int64_t nl = (int64_t)il.lpr * rounds;
    for (int64_t p0 = 0; p0 < il.lines; p0 += nl)
      t.push_back(LineTask{il.inst, (int32_t)std::min<int64_t>(nl, il.lines - p0), p0});
  }
  return t;
}

sgdg_status reaction_build(sgdg_plan* plan) {
  RHost* rh = new RHost();
  plan->rdata = rh;
  const int d = plan->d;
  // A whole finest-grid line stays in LDS: (k+1) 2^N <= 2048.  Larger plans
  // are still valid for the sweep and the Krylov exponential; their reaction
  // calls report SGDG_ERR_UNSUPPORTED.
  // Two-species instances keep four lines of inputs and their transform
  // buffers in LDS during the implicit-stage correction: (k+1) 2^N <= 1024.
  for (const HostInstance& hi : plan->inst) {
    const int n1 = (hi.desc.k + 1) << hi.desc.n;
    const size_t need = line_tile_doubles(2 * hi.desc.nspecies, 1, n1, hi.desc.k + 1) * sizeof(double);
    if (n1 > RX_MAX_N1 || need > (size_t)APPLY_LDS_BYTES_HOST) {
      rh->supported = false;
      return SGDG_OK;
    }
  }
  std::vector<RInst> ri;
  std::vector<RBlk> rblk;
  std::vector<int32_t> rid, rbe;
  std::vector<double> EL, EH, w1, mats;
  int64_t ws = 0;
  // chunking of every stage: enough threads to fill the device, and tiles no
  // wider than the smallest fibre set of the plan
  int nmin = 1 << 30;
  for (const HostInstance& hi : plan->inst) nmin = std::min(nmin, hi.desc.n);
  int maxnp1 = 0;
  for (const HostInstance& hi : plan->inst) maxnp1 = std::max(maxnp1, (hi.desc.k + 1) << hi.desc.n);
  for (int m = 0; m + 1 <= d - 1; ++m) {
    int64_t nf = 0, gmin = INT64_MAX;
    for (const HostInstance& hi : plan->inst) {
      const int N = hi.desc.n, K1 = hi.desc.k + 1;
      // fibres of stage m: species x np1^m prefixes x DOFs of the (d-m-1)-dim grid
      int64_t g = 0;
      for (const auto& b : grid_blocks(d - m - 1, N)) {
        int64_t sz = 1;
        for (int v : b) sz *= (int64_t)level_count(v) * K1;
        g += sz;
      }
      int64_t pre = 1;
      for (int t = 0; t < m; ++t) pre *= (int64_t)K1 << N;
      nf += hi.desc.nspecies * pre * g;
      gmin = std::min(gmin, g);
    }
    // 2^lam chunks per fibre: enough threads to fill the device, at most
    // RX_WALK points per thread, tiles no wider than the smallest fibre set;
    // the first two chunk bits go to waves (wave-uniform point index), the
    // rest to lanes
    int lam = 0;
    const int lmax = std::min(8, nmin);
    while (lam < lmax && ((nf << lam) < RX_THREADS_WANTED || (maxnp1 >> lam) > RX_WALK ||
                          (RX_THREADS >> lam) > gmin))
      ++lam;
    rh->lam[m] = lam;
    rh->llane[m] = std::max(0, lam - 2);
  }
  rh->cum_x.assign(d, std::vector<int64_t>(1, 0));
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
    rh->k1mask |= 1 << K1;
    rh->max_n1 = std::max(rh->max_n1, r.n1);
    rh->max_np1 = std::max(rh->max_np1, r.np1);
    std::vector<double> xg, wg;
    gauss01(r.nq, xg, wg);
    const Basis1D& bs = basis1d(hi.desc.k);
    const double h = std::ldexp(1.0, -N);
    r.EL_off = (int64_t)EL.size();
    r.EH_off = (int64_t)EH.size();
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
    // hierarchical basis (eq. 2.6) at the finest Gauss points, one row per
    // point: for every level l the one cell of level l that holds the point
    // (level 0: the Legendre basis)
    for (int q = 0; q < r.np1; ++q)
      for (int l = 0; l <= N; ++l) {
        const int cellN = q / r.nq;
        const double x = (cellN + xg[q % r.nq]) * h;
        const int j = l == 0 ? 0 : cellN >> (N - l + 1);
        for (int p = 0; p < K1; ++p) EH.push_back(hier_value(bs, l, j, p, x, false));
      }
    // two-scale matrices, rows padded to 16 entries each
    const std::vector<double>* src[4] = {&bs.ML, &bs.MR, &bs.cL, &bs.cR};
    for (int t = 0; t < 4; ++t) {
      std::vector<double> pad(16, 0.0);
      std::copy(src[t]->begin(), src[t]->end(), pad.begin());
      mats.insert(mats.end(), pad.begin(), pad.end());
    }
    // r-dimensional sparse grids, r = 1..d, and the block of every element
    for (int rr = 1; rr <= d; ++rr) {
      auto blocks = grid_blocks(rr, N);
      r.blk_off[rr] = (int32_t)rblk.size();
      r.nblk[rr] = (int32_t)blocks.size();
      r.id_off[rr] = (int32_t)rid.size();
      r.be_off[rr] = (int64_t)rbe.size();
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
        rbe.insert(rbe.end(), (size_t)sz, (int32_t)b);
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
    // fibre tiles of stage m: 256 >> lam fibres of one (species, prefix)
    for (int m = 0; m + 1 <= d - 1; ++m) {
      const int64_t tw = RX_THREADS >> rh->lam[m];
      r.ntile[m] = (int32_t)((r.gdof[d - m - 1] + tw - 1) / tw);
      rh->cum_x[m].push_back(rh->cum_x[m].back() + (int64_t)S * r.npre[m] * r.ntile[m]);
    }
    // line tiles: instances of the same degree and species count whose
    // lines run in the wave form form one class and one launch (a wave loads
    // a tile's instance state when the instance changes); the LDS-tile form
    // groups by (degree, level, species), one LDS layout each
    {
      const bool wave = d >= 2 && N <= RX_WLINE_MAXN;
      LineClass* lc = nullptr;
      for (LineClass& c : rh->lclass)
        if (c.wave == wave && c.K1 == K1 && c.S == S && (wave || c.N == N)) lc = &c;
      const bool first = !lc;
      if (!lc) {
        rh->lclass.emplace_back();
        lc = &rh->lclass.back();
        lc->K1 = K1;
        lc->N = N;
        lc->S = S;
        lc->wave = wave;
      }
      if (wave) {
        // tiles of whole rounds (4 waves, LPW lines each); the default shape
        // takes about 2048 tiles per instance, up to 16 rounds (the class's
        // smallest instance decides: small problems keep many workgroups),
        // and 16 workgroups per CU
        const int cplh = std::min(K1 == 2 ? 8 : 4, 1 << N);  // finest cells per lane (wl_cpl)
        const int hh = N - (cplh == 8 ? 3 : cplh == 4 ? 2 : cplh == 2 ? 1 : 0);
        const int lpr = (RX_THREADS / 64) * (64 >> std::min(hh, 6));
        int64_t most = 0;
        for (const WaveLines& wl : lc->lines) most = std::max(most, wl.lines);
        if (r.npre[d - 1] > most) lc->lpr = lpr;  // (the lines per round of the class's largest instance)
        lc->N = std::max(lc->N, N);
        lc->lines.push_back({i, lpr, r.npre[d - 1]});
        const int want = (int)std::min<int64_t>(std::max<int64_t>(1, r.npre[d - 1] / 2048 / lpr), RX_WLINE_ROUNDS);
        for (int nin = 1; nin <= 2; ++nin) {
          lc->rounds[nin] = first ? want : std::min(lc->rounds[nin], want);
          lc->wgcu[nin] = 16;
        }
      } else {
        for (int nin = 1; nin <= 2; ++nin) {
          // lines per tile: the LDS budget of one workgroup; threads: about
          // RX_ITEMS transform items each at the finest level, 64..256
          const int npair = nin * S;
          int64_t nl = ((int64_t)RX_LINE_LDS / 8 - RX_TAIL - (int64_t)r.n1 * (K1 + 1)) / line_doubles(npair, r.n1);
          nl = std::max<int64_t>(1, std::min<int64_t>(nl, r.npre[d - 1]));
          int th = 64;
          while (th < RX_THREADS && (int64_t)npair * nl * r.n1 > (int64_t)th * RX_ITEMS) th *= 2;
          for (int64_t p0 = 0; p0 < r.npre[d - 1]; p0 += nl)
            lc->tasks[nin].push_back(LineTask{i, (int32_t)std::min<int64_t>(nl, r.npre[d - 1] - p0), p0});
          lc->lds[nin] = std::max(lc->lds[nin], line_tile_doubles(npair, (int)nl, r.n1, K1) * sizeof(double));
          lc->threads[nin] = std::max(lc->threads[nin], th);
        }
      }
    }
    rh->cum_fin.push_back(rh->cum_fin.back() + (d >= 2 ? (int64_t)S * r.ntile[0] : 1));
    ri.push_back(r);
  }
  // stages whose tiles hold whole prefixes of a small hierarchical block
  // stage that block in LDS (expansion: its input; contraction, m >= 1: its
  // output)
  for (int m = 0; m + 1 <= d - 1; ++m) {
    int64_t mx = 0;
    bool whole = true;
    for (const RInst& r : ri) {
      whole = whole && r.ntile[m] == 1;
      mx = std::max(mx, r.gdof[d - m]);
    }
    rh->xs_lds[m] =
        whole && rh->llane[m] == 0 && mx * (int64_t)sizeof(double) <= RX_XS_LDS ? (int)(mx * sizeof(double)) : 0;
  }
  // level bucket per degree: the smallest of 7, 9, RX_LMAX levels that
  // holds every instance of that degree
  for (const RInst& r : ri) rh->lm[r.K1] = std::max(rh->lm[r.K1], r.N + 1);
  for (int& v : rh->lm) v = v <= 7 ? 7 : v <= 9 ? 9 : RX_LMAX;
  EH.resize(EH.size() + RX_LMAX * 4, 0.0);  // (whole-row reads of the last point of the last instance)
  rh->rws = ws;
  sgdg_status st;
  if ((st = up(plan, ri, &rh->dev.inst)) != SGDG_OK || (st = up(plan, rblk, &rh->dev.rblk)) != SGDG_OK ||
      (st = up(plan, rid, &rh->dev.rid)) != SGDG_OK || (st = up(plan, rbe, &rh->dev.rbe)) != SGDG_OK ||
      (st = up(plan, EL, &rh->dev.EL)) != SGDG_OK || (st = up(plan, EH, &rh->dev.EH)) != SGDG_OK ||
      (st = up(plan, w1, &rh->dev.w1)) != SGDG_OK || (st = up(plan, mats, &rh->dev.mats)) != SGDG_OK ||
      (st = up(plan, rh->cum_fin, &rh->dev.cum_fin)) != SGDG_OK)
    return st;
  for (int m = 0; m + 1 <= d - 1; ++m)
    if ((st = up(plan, rh->cum_x[m], &rh->dev.cum_x[m])) != SGDG_OK) return st;
  for (LineClass& lc : rh->lclass)
    for (int nin = 1; nin <= 2; ++nin) {
      if (lc.wave) {
        // room for the most tiles (one round each); the current shape's tiles are written into it
        lc.cap_tasks[nin] = wave_tiles(lc, 1).size();
        lc.tasks[nin] = wave_tiles(lc, 1);
        if ((st = up(plan, lc.tasks[nin], &lc.dev[nin])) != SGDG_OK) return st;
        lc.tasks[nin] = wave_tiles(lc, lc.rounds[nin]);
        const hipError_t e = hipMemcpy(lc.dev[nin], lc.tasks[nin].data(), lc.tasks[nin].size() * sizeof(LineTask),
                                       hipMemcpyHostToDevice);
        if (e != hipSuccess) return hip_fail(e, "hipMemcpy(line tiles)");
      } else if ((st = up(plan, lc.tasks[nin], &lc.dev[nin])) != SGDG_OK) {
        return st;
      }
    }
  if (hipDeviceGetAttribute(&rh->ncu, hipDeviceAttributeMultiprocessorCount, plan->device) != hipSuccess) {
    rh->ncu = 0;
    (void)hipGetLastError();
  }
  return set_line_lds(rh);
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
// (one round of loads per 64 instances)
// Every problem of the pass has converged (the count after the flags, kept
// by the convergence check): a launch of a finished stage iteration returns
// at once.
__device__ __forceinline__ bool all_converged(const RxArgs& a) {
  return a.conv && __builtin_amdgcn_readfirstlane(a.conv[a.nprob]) >= a.nprob;
}

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

// a[m] for a small kernel-argument array without a dynamic index (which would
// move the argument struct to scratch memory)
__device__ __forceinline__ const int64_t* pick(const int64_t* const (&a)[SGDG_MAX_D], int m) {
  const int64_t* r = a[0];
#pragma unroll
  for (int i = 1; i < SGDG_MAX_D; ++i)
    if (m == i) r = a[i];
  return r;
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

// The pointwise map of a pass at one point: u[s] = R U (mode RX_CORR also
// g[s] = R G); returns the values to project (before the quadrature weight).
__device__ __forceinline__ void rx_map(const double (*rx)[4][4], int S, int mode, double dt2, const double* u,
                                       const double* g, double* out) {
  if (mode == RX_CORR) {
    double J[2][2];
    rx_jac(rx, S, u, J);
    if (S == 1) {
      out[0] = g[0] / (1.0 - dt2 * J[0][0]);
      out[1] = 0.0;
    } else {
      const double A = 1.0 - dt2 * J[0][0], Bq = -dt2 * J[0][1];
      const double C = -dt2 * J[1][0], D = 1.0 - dt2 * J[1][1];
      const double det = A * D - Bq * C;
      out[0] = (D * g[0] - Bq * g[1]) / det;
      out[1] = (A * g[1] - C * g[0]) / det;
    }
  } else if (mode == RX_LOCAL) {
    // u - dt2 f(u) = w at this point, Newton from u = w (at most RX_LOCAL_MAX_ITER corrections)
    const double w0 = u[0], w1v = S > 1 ? u[1] : 0.0;
    const double wmag = fmax(1.0, fmax(fabs(w0), fabs(w1v)));
    double x[2] = {w0, w1v};
    for (int it = 0; it <= RX_LOCAL_MAX_ITER; ++it) {
      double f[2];
      rx_f(rx, S, x, f);
      const double g0 = x[0] - dt2 * f[0] - w0, g1 = S > 1 ? x[1] - dt2 * f[1] - w1v : 0.0;
      if (fmax(fabs(g0), fabs(g1)) <= RX_LOCAL_TOL * wmag || it == RX_LOCAL_MAX_ITER) break;
      double J[2][2];
      rx_jac(rx, S, x, J);
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
    rx_f(rx, S, u, out);
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

// Geometry of one fibre of stage m (fibres along axis m): the block of the
// (r-1)-dim grid (axes m+1..d-1, r = d - m) that holds element eo, and the
// start of the r-dim grid block (l, that block's levels) for every level l of
// axis m within the fibre's budget L.
template <int LM>
struct Fibre {
  int32_t rest, Sb;
  int L;
  int32_t bl[LM];  // offsets inside one r-dim grid (< 2^31 for every supported plan)
};

template <int LM>
__device__ __forceinline__ Fibre<LM> fibre_geometry(const RTables& R, const RInst& I, int r, int64_t eo) {
  Fibre<LM> F;
  const int N = I.N;
  const RBlk& B = R.rblk[I.blk_off[r - 1] + R.rbe[I.be_off[r - 1] + eo]];
  F.rest = (int32_t)(eo - B.start);
  F.Sb = B.size;
  F.L = N - B.lsum;
  int lin = 0, pw = 1;
  for (int t = r - 2; t >= 0; --t) {
    lin += B.lev[t] * pw;
    pw *= (N + 1);
  }
  const int32_t* __restrict__ id = R.rid + I.id_off[r];
  const RBlk* __restrict__ ib = R.rblk + I.blk_off[r];
  // levels past the budget keep a valid address (level 0's) and are masked by the caller
#pragma unroll
  for (int l = 0; l < LM; ++l) F.bl[l] = (int32_t)ib[id[(l <= F.L ? l : 0) * pw + lin]].start + F.rest;
  return F;
}

// ---------------------------------------------------------------- kernels

// Tile of stage m: (species, prefix, tile of 256 >> lam fibres), each fibre's
// points cut into 2^lam chunks.  The low ll chunk bits are lane bits (a wave
// holds 64 >> ll fibres times 2^ll chunks), the others wave bits (waves of
// the workgroup).  Without lane bits every wave holds 64 consecutive fibres
// and one chunk, so the point index -- and with it every basis-table and
// weight address -- is the same across the wave (LANES = false).
struct TileIdx {
  int s;
  int64_t pre;
  int64_t eo;  // this thread's fibre
  int qc;      // its chunk of points: (wave chunk << ll) | lane chunk
  int wc, lc;  // wave and lane chunk
  int fb;      // its wave's block of fibres
  int fpw;     // fibres per wave
};

template <bool LANES>
__device__ __forceinline__ TileIdx tile_index(const RInst& I, int m, int64_t le, int lam, int ll) {
  TileIdx t;
  const int ntile = I.ntile[m];
  const int64_t per_s = I.npre[m] * ntile;
  t.s = (int)(le / per_s);
  le -= (int64_t)t.s * per_s;
  t.pre = le / ntile;
  const int tt = (int)(le - t.pre * ntile);
  const int lw = LANES ? lam - ll : lam;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), ln = threadIdx.x & 63;
  t.wc = w >> (2 - lw);
  t.fb = w & ((4 >> lw) - 1);
  if (LANES) {
    t.fpw = 64 >> ll;
    t.lc = ln >> (6 - ll);
    t.qc = (t.wc << ll) | t.lc;
    t.eo = (int64_t)tt * (RX_THREADS >> lam) + t.fb * t.fpw + (ln & (t.fpw - 1));
  } else {
    t.fpw = 64;
    t.lc = 0;
    t.qc = t.wc;
    t.eo = (int64_t)tt * (RX_THREADS >> lam) + t.fb * 64 + ln;
  }
  return t;
}

// Largest level that any fibre of the calling wave holds (the level loops of
// a walk stop there: the same bound for the whole wave, so the basis-table
// loads stay wave-uniform).
__device__ __forceinline__ int wave_max_level(int L) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) L = max(L, __shfl_xor(L, off, 64));
  return __builtin_amdgcn_readfirstlane(L);
}

// Copy n doubles from global memory to LDS, four loads of every thread in
// flight together.
__device__ __forceinline__ void stage_block(double* __restrict__ dst, const double* __restrict__ src, int n) {
  for (int i0 = threadIdx.x; i0 < n; i0 += 4 * RX_THREADS) {
    double v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int i = i0 + u * RX_THREADS;
      v[u] = src[i < n ? i : 0];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (i0 + u * RX_THREADS < n) dst[i0 + u * RX_THREADS] = v[u];
  }
}

// expansion stage m: hierarchical along axis m -> point values, one tile bx
// (of the stage's tiles over all instances) of right-hand side rhs and input z.
// XS: the tile holds every fibre of its (species, prefix) and the prefix's
// hierarchical block is first copied to LDS (xs; the call with stage = true
// does only that, the caller synchronises), so that the walk reads only LDS
// and issues nothing but stores to global memory.
template <int K1, int LM, bool LANES, bool XS>
__device__ void rx_expand_body(const RTables& R, const double* __restrict__ EHg, int inst, int m, int64_t total,
                               const RxArgs& a, int64_t rws, int lam, int ll, double* xs, int64_t bx, int rhs,
                               int z, bool stage) {
  const RInst& I = R.inst[inst];
  const int d = I.d, r = d - m, N = I.N, S = I.S, np1 = I.np1;
  const TileIdx t = tile_index<LANES>(I, m, bx - pick(R.cum_x, m)[inst], lam, ll);
  const int64_t gd_in = I.gdof[r], gd_out = I.gdof[r - 1];
  double* xr = a.rws + (int64_t)rhs * rws;
  const double* __restrict__ in =
      m == 0 ? plan_in(a, z, (int64_t)rhs * total) + I.seg + (int64_t)t.s * I.ndof
             : xr + I.X_off[m] + (((int64_t)z * S + t.s) * I.npre[m] + t.pre) * gd_in;
  if constexpr (XS) {
    if (stage) {
      stage_block(xs, in, (int)gd_in);
      return;
    }
  }
  const bool valid = t.eo < gd_out;
  const Fibre<LM> F = fibre_geometry<LM>(R, I, r, valid ? t.eo : 0);
  if (!valid) return;
  const int Lw = wave_max_level(F.L);
  auto ld = [&](int64_t i) -> double {
    if constexpr (XS)
      return xs[i];
    else
      return in[i];
  };
  double* __restrict__ out =
      xr + I.X_off[m + 1] + (((int64_t)z * S + t.s) * I.npre[m + 1] + t.pre * np1) * gd_out + t.eo;
  const double* __restrict__ EH = EHg + I.EH_off;
  const int NL1 = N + 1;
  const int cw = (1 << N) >> lam, c0 = t.qc * cw;
  // coefficients of the current cell of every level (zero past the fibre's
  // budget); the level loops run to the wave's largest budget
  double cf[LM][K1];
#pragma unroll
  for (int l = 0; l < LM; ++l)
    if (l <= Lw) {
      const int j = l == 0 ? 0 : c0 >> (N - l + 1);
      const bool on = l <= F.L;
#pragma unroll
      for (int p = 0; p < K1; ++p) {
        const double v = ld(F.bl[l] + (int64_t)((on ? j : 0) * K1 + p) * F.Sb);
        cf[l][p] = on ? v : 0.0;
      }
    }
  for (int c = c0; c < c0 + cw; ++c) {
    if (c != c0) {
#pragma unroll
      for (int l = 1; l < LM; ++l)
        if (l <= Lw && (c & ((1 << (N - l + 1)) - 1)) == 0) {
          const int j = c >> (N - l + 1);
          const bool on = l <= F.L;
#pragma unroll
          for (int p = 0; p < K1; ++p) {
            const double v = ld(F.bl[l] + (int64_t)((on ? j : 0) * K1 + p) * F.Sb);
            cf[l][p] = on ? v : 0.0;
          }
        }
    }
#pragma unroll
    for (int gq = 0; gq < K1; ++gq) {
      const int q = c * K1 + gq;
      const double* __restrict__ eh = EH + (int64_t)q * NL1 * K1;  // the point's row: levels 0..N, K1 each
      double u = 0.0;
#pragma unroll
      for (int l = 0; l < LM; ++l)
        if (l <= Lw)
#pragma unroll
          for (int p = 0; p < K1; ++p) u += eh[l * K1 + p] * cf[l][p];
      out[(int64_t)q * gd_out] = u;
    }
  }
}

// one kernel per degree and level bucket LM >= N + 1 (register use follows
// K1 and LM); workgroups of instances of another degree return at once
// (the basis table is its own argument: its loads are wave-uniform and go
// through the scalar cache)
// The tiles of a staged (XS) launch go two to a workgroup, both blocks
// staged before either walk: half the workgroups to dispatch (a converged
// pass returns from every one of them), and no load after a store inside a
// workgroup.  xsd: LDS doubles per tile.
constexpr int RX_XS_TILES = 2;      // expansion
constexpr int RX_XS_TILES_CON = 2;  // contraction

// tile bx of stage m runs for right-hand side rhs: in range, of degree K1,
// problem not converged (inst: its instance)
template <int K1>
__device__ __forceinline__ bool tile_live(const RTables& R, const RxArgs& a, int ninst, int m, int64_t bx, int rhs,
                                          int& inst) {
  if (bx >= pick(R.cum_x, m)[ninst]) return false;
  inst = find_inst(pick(R.cum_x, m), ninst, bx);
  return R.inst[inst].K1 == K1 && !(a.conv && a.conv[rhs * ninst + inst]);
}

template <int K1, int LM, bool LANES, bool XS>
__global__ __launch_bounds__(RX_THREADS) void k_rx_expand(RTables R, const double* __restrict__ EHg, int ninst, int m,
                                                          int64_t total, RxArgs a, int64_t rws, int lam, int ll,
                                                          int xsd) {
  extern __shared__ double xs_dyn[];
  if (all_converged(a)) return;
  const int rhs = blockIdx.y, z = blockIdx.z;
  if constexpr (XS) {
    int inst[RX_XS_TILES];
    bool live[RX_XS_TILES];
#pragma unroll
    for (int j = 0; j < RX_XS_TILES; ++j) {
      const int64_t bx = (int64_t)blockIdx.x * RX_XS_TILES + j;
      live[j] = tile_live<K1>(R, a, ninst, m, bx, rhs, inst[j]);
      if (live[j])
        rx_expand_body<K1, LM, LANES, XS>(R, EHg, inst[j], m, total, a, rws, lam, ll, xs_dyn + j * xsd, bx, rhs, z,
                                          true);
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < RX_XS_TILES; ++j)
      if (live[j])
        rx_expand_body<K1, LM, LANES, XS>(R, EHg, inst[j], m, total, a, rws, lam, ll, xs_dyn + j * xsd,
                                          (int64_t)blockIdx.x * RX_XS_TILES + j, rhs, z, false);
  } else {
    int inst = 0;
    if (!tile_live<K1>(R, a, ninst, m, blockIdx.x, rhs, inst)) return;
    rx_expand_body<K1, LM, LANES, XS>(R, EHg, inst, m, total, a, rws, lam, ll, xs_dyn, blockIdx.x, rhs, z, false);
  }
}

// contraction stage m: weighted point values along axis m -> hierarchical
// (m >= 1 writes Y_m; m == 0 finishes plan vectors), grid (tiles, rhs).
// XS (m >= 1): the tile holds every fibre of its (species, prefix); the
// outputs are collected in an LDS image of the prefix's hierarchical block
// (ys) that the caller writes out after the workgroup's last walk, so that
// the walks issue only loads to global memory.
template <int K1, int LM, bool LANES, bool XS>
__device__ void rx_contract_body(const RTables& R, const double* __restrict__ EHg, const double* __restrict__ w1g,
                                 int inst, int m, int mode, int64_t total, const RxArgs& a, int64_t rws, int lam,
                                 int ll, int64_t nfin, double* ys, int64_t bx, int rhs) {
  // partial sums of the levels whose cells span several chunks: [wave][level <= 2][p][lane]
  __shared__ double red[4][3][K1][64];
  __shared__ double wsum[RX_THREADS / 64];
  if constexpr (XS) __syncthreads();  // (the workgroup's previous tile has finished with red)
  const RInst& I = R.inst[inst];
  const int ln = threadIdx.x & 63;
  const int d = I.d, r = d - m, N = I.N, np1 = I.np1;
  const int64_t le = bx - pick(R.cum_x, m)[inst];
  const TileIdx t = tile_index<LANES>(I, m, le, lam, ll);
  const int lw = LANES ? lam - ll : lam;
  const int w = t.wc * (4 >> lw) + t.fb;
  const int64_t gd_in = I.gdof[r - 1], gd_out = I.gdof[r];
  // every thread passes the barriers; threads past the fibre set emit nothing
  const bool valid = t.eo < gd_in;
  const Fibre<LM> F = fibre_geometry<LM>(R, I, r, valid ? t.eo : 0);
  const int L = valid ? F.L : -1;
  const int Lw = wave_max_level(L);
  double* xr = a.rws + (int64_t)rhs * rws;
  // (threads past the fibre set walk fibre 0's points; their sums, kept apart
  // from every valid fibre's, are never emitted)
  const double* __restrict__ in =
      xr + I.Y_off[m + 1] + ((int64_t)t.s * I.npre[m + 1] + t.pre * np1) * gd_in + (valid ? t.eo : 0);
  const double* __restrict__ EH = EHg + I.EH_off;
  const double* __restrict__ w1 = w1g + I.w_off;
  double* outm = m > 0 ? xr + I.Y_off[m] + ((int64_t)t.s * I.npre[m] + t.pre) * gd_out : nullptr;
  const int64_t base = (int64_t)rhs * total + I.seg + (int64_t)t.s * I.ndof;
  double g2 = 0.0;
  auto emit = [&](int l, int j, int p, double v) {
    const int64_t o = F.bl[l] + (int64_t)(j * K1 + p) * F.Sb;
    if constexpr (XS)
      ys[o] = v;
    else if (m > 0)
      outm[o] = v;
    else
      g2 += finish(a, mode, base + o, v);
  };
  const int NL1 = N + 1;
  const int cw = (1 << N) >> lam, c0 = t.qc * cw;
  double acc[LM][K1];
#pragma unroll
  for (int l = 0; l < LM; ++l)
#pragma unroll
    for (int p = 0; p < K1; ++p) acc[l][p] = 0.0;
  // the point values of CB cells are loaded together, one batch ahead of
  // their use (the last batch loads itself again: every iteration issues the
  // same loads, so the wait for a batch never includes the next one)
  constexpr int CB = LANES ? 1 : (K1 == 2 ? 4 : 2);
  double gv[CB][K1];
  auto fetch = [&](int cb, double (&g)[CB][K1]) {
#pragma unroll
    for (int b = 0; b < CB; ++b)
#pragma unroll
      for (int gq = 0; gq < K1; ++gq) {
        const int q = min(cb + b, c0 + cw - 1) * K1 + gq;
        g[b][gq] = in[(int64_t)q * gd_in];
      }
  };
  fetch(c0, gv);
  for (int cb = c0; cb < c0 + cw; cb += CB) {
    double gn[CB][K1];
    fetch(cb + CB < c0 + cw ? cb + CB : cb, gn);
#pragma unroll
    for (int b = 0; b < CB; ++b) {
      const int c = cb + b;
      if (c >= c0 + cw) continue;
#pragma unroll
      for (int gq = 0; gq < K1; ++gq) {
        const int q = c * K1 + gq;
        const double* __restrict__ eh = EH + (int64_t)q * NL1 * K1;
        const double g = w1[q] * gv[b][gq];
        if constexpr (XS) {
          // the whole row at once (one round of scalar loads; rows past the
          // instance's levels read the next row or the table's zero padding)
          double e[LM][K1];
#pragma unroll
          for (int l = 0; l < LM; ++l)
#pragma unroll
            for (int p = 0; p < K1; ++p) e[l][p] = eh[l * K1 + p];
#pragma unroll
          for (int l = 0; l < LM; ++l)
            if (l <= Lw)
#pragma unroll
              for (int p = 0; p < K1; ++p) acc[l][p] += e[l][p] * g;
        } else {
#pragma unroll
          for (int l = 0; l < LM; ++l)
            if (l <= Lw)
#pragma unroll
              for (int p = 0; p < K1; ++p) acc[l][p] += eh[l * K1 + p] * g;  // (unused past the fibre's budget)
        }
      }
      // levels whose cells lie inside one chunk: a cell is complete when the walk leaves it
#pragma unroll
      for (int l = 1; l < LM; ++l)
        if (l > lam && l <= L && ((c + 1) & ((1 << (N - l + 1)) - 1)) == 0) {
#pragma unroll
          for (int p = 0; p < K1; ++p) {
            emit(l, c >> (N - l + 1), p, acc[l][p]);
            acc[l][p] = 0.0;
          }
        }
    }
#pragma unroll
    for (int b = 0; b < CB; ++b)
#pragma unroll
      for (int gq = 0; gq < K1; ++gq) gv[b][gq] = gn[b][gq];
  }
  // coarser levels span 2^g chunks, g = lam - l + 1 (level 0: g = lam):
  // fixed-order butterfly over the lane bits of the chunk, then the wave of
  // the first chunk adds the waves' sums in order
  const int llv = LANES ? ll : 0;
  if (LANES) {
#pragma unroll
    for (int l = 0; l < LM; ++l)
      if (l <= lam) {
        const int gl = min(l == 0 ? lam : lam - l + 1, llv);
#pragma unroll
        for (int p = 0; p < K1; ++p) {
          double v = acc[l][p];
          for (int b = 0; b < gl; ++b) v += __shfl_xor(v, t.fpw << b, 64);
          acc[l][p] = v;
        }
      }
  }
  if (lw > 0) {
#pragma unroll
    for (int l = 0; l < 3; ++l)
      if (l <= lw)
#pragma unroll
        for (int p = 0; p < K1; ++p) red[w][l][p][ln] = acc[l][p];
    __syncthreads();
  }
  constexpr int LR = LANES ? LM : 3;  // levels that can span chunks (lam <= 2 without lane bits)
#pragma unroll
  for (int l = 0; l < LR; ++l)
    if (l <= lam) {
      const int g = l == 0 ? lam : lam - l + 1;  // log2 of the chunks per cell
      const int gl = min(g, llv), gw = g - gl;
      if (l <= L && (t.lc & ((1 << gl) - 1)) == 0 && (t.wc & ((1 << gw) - 1)) == 0) {
        const int j = l == 0 ? 0 : t.qc >> g;
#pragma unroll
        for (int p = 0; p < K1; ++p) {
          double v = acc[l][p];
          if (gw > 0 && l < 3) {
            v = 0.0;
            for (int cc = 0; cc < (1 << gw); ++cc) v += red[(t.wc + cc) * (4 >> lw) + t.fb][l][p][ln];
          }
          emit(l, j, p, v);
        }
      }
    }
  if (m == 0 && mode == RX_RESID) {
    g2 = block_sum(g2, wsum);
    if (threadIdx.x == 0) a.part[(int64_t)rhs * nfin + bx] = g2;
  }
}

template <int K1, int LM, bool LANES, bool XS>
__global__ __launch_bounds__(RX_THREADS) void k_rx_contract(RTables R, const double* __restrict__ EHg,
                                                            const double* __restrict__ w1g, int ninst, int m, int mode,
                                                            int64_t total, RxArgs a, int64_t rws, int lam, int ll,
                                                            int64_t nfin, int xsd) {
  extern __shared__ double ys_dyn[];
  if (all_converged(a)) return;
  const int rhs = blockIdx.y;
  if constexpr (XS) {
    int inst[RX_XS_TILES_CON];
    bool live[RX_XS_TILES_CON];
#pragma unroll
    for (int j = 0; j < RX_XS_TILES_CON; ++j) {
      const int64_t bx = (int64_t)blockIdx.x * RX_XS_TILES_CON + j;
      live[j] = tile_live<K1>(R, a, ninst, m, bx, rhs, inst[j]);
      if (live[j])
        rx_contract_body<K1, LM, LANES, XS>(R, EHg, w1g, inst[j], m, mode, total, a, rws, lam, ll, nfin,
                                            ys_dyn + j * xsd, bx, rhs);
    }
    __syncthreads();
    // every tile's hierarchical block to Y_m
#pragma unroll
    for (int j = 0; j < RX_XS_TILES_CON; ++j)
      if (live[j]) {
        const RInst& I = R.inst[inst[j]];
        const int64_t le = (int64_t)blockIdx.x * RX_XS_TILES_CON + j - pick(R.cum_x, m)[inst[j]];
        const int64_t per_s = I.npre[m] * I.ntile[m];  // (one tile per prefix)
        const int s = (int)(le / per_s);
        const int64_t pre = (le - (int64_t)s * per_s) / I.ntile[m];
        const int64_t gd_out = I.gdof[I.d - m];
        double* outm = a.rws + (int64_t)rhs * rws + I.Y_off[m] + ((int64_t)s * I.npre[m] + pre) * gd_out;
        const double* y = ys_dyn + j * xsd;
        for (int i = threadIdx.x; i < gd_out; i += RX_THREADS) outm[i] = y[i];
      }
  } else {
    int inst = 0;
    if (!tile_live<K1>(R, a, ninst, m, blockIdx.x, rhs, inst)) return;
    rx_contract_body<K1, LM, LANES, XS>(R, EHg, w1g, inst, m, mode, total, a, rws, lam, ll, nfin, ys_dyn, blockIdx.x,
                                        rhs);
  }
}

// Last axis: a tile of nl whole lines (consecutive prefixes).  LDS: the
// two-scale matrices, the reaction coefficients, the finest-cell basis at the
// Gauss points and the weights, then per line (pair = input * S + species,
// npair = 1, 2 or 4):
//   H [pair][n1]     the hierarchical inputs; later the projections and one
//                    of the two scaling buffers of the forward transform
//   SA[pair][n1]     cell coefficients of the inverse transform (the last step
//                    writes the finest level here); later the wavelets of
//                    the forward transform at their final places
//   SB[pair][n1/2]   the other scaling buffer of both transforms
// The transforms take two levels per barrier step (an item is a cell two
// levels above the finer one: its two children are formed in registers and
// their four children written out, or the reverse).  For d = 1 the line is
// the instance itself, read from and finished into plan vectors.
template <int K1>
__device__ void rx_line_tile(const RInst& I, int mode, int64_t total, const RxArgs& a, int64_t rws, int nin,
                             int64_t nfin, int64_t fin_index, int rhs, int64_t pre0, int nl, double* lds) {
  const int tid = threadIdx.x, nt = blockDim.x;
  const int d = I.d, N = I.N, S = I.S, n1 = I.n1, np1 = I.np1;
  const int npair = nin * S;
  const int lp = npair == 1 ? 0 : (npair == 2 ? 1 : 2);  // log2 npair
  const int ls = S == 1 ? 0 : 1;                        // log2 S
  const int LSL = 5 * npair * (n1 / 2);                 // doubles per line: 2.5 npair n1
  double* M = lds;                                      // 64
  double (*rx)[4][4] = (double (*)[4][4])(lds + 64);    // 32
  double* wsum = lds + 96;                              // 8
  double* EL = lds + RX_TAIL;                           // [q][p] finest-level cell basis, np1 K1
  double* w1 = EL + np1 * K1;                           // np1
  double* L0 = w1 + np1;                                // line buffers
  auto Hr = [&](int ln, int pr) { return L0 + (int64_t)ln * LSL + pr * n1; };
  auto SAr = [&](int ln, int pr) { return L0 + (int64_t)ln * LSL + (npair + pr) * n1; };
  auto SBr = [&](int ln, int pr) { return L0 + (int64_t)ln * LSL + 2 * npair * n1 + pr * (n1 / 2); };
  double* xr = a.rws + (int64_t)rhs * rws;
  // one level of the inverse transform: the two children of level-n cell c
  // (K1 values each) from s_n[c] and the level-(n+1) wavelets w[c]
  auto up = [&](const double* sc, const double* wc, double (&ch)[2][K1]) {
#pragma unroll
    for (int side = 0; side < 2; ++side)
#pragma unroll
      for (int q = 0; q < K1; ++q) {
        double acc = 0.0;
#pragma unroll
        for (int i = 0; i < K1; ++i) acc += M[side * 16 + q * K1 + i] * sc[i];
#pragma unroll
        for (int p = 0; p < K1; ++p) acc += M[32 + side * 16 + p * K1 + q] * wc[p];
        ch[side][q] = acc;
      }
  };
  // inverse transform, levels 1..N, two per step; the finest cells land in SA
  {
    const int ns = (N + 1) / 2;
    int n = 1;  // next level to form
    for (int st = 0; st < ns; ++st) {
      const bool toA = ((ns - 1 - st) & 1) == 0;
      const bool two = n + 1 <= N;
      const int nb = n - 1;  // items: cells of level n - 1
      for (int it = tid; it < (npair * nl) << nb; it += nt) {
        const int j = it & ((1 << nb) - 1), pl = it >> nb;
        const int pr = pl & (npair - 1), ln = pl >> lp;
        const double* h = Hr(ln, pr);
        const double* cur = n == 1 ? h : (toA ? SBr(ln, pr) : SAr(ln, pr));
        double* nxt = toA ? SAr(ln, pr) : SBr(ln, pr);
        double c1[2][K1];
        up(cur + j * K1, h + (K1 << (n - 1)) + j * K1, c1);
        if (!two) {
#pragma unroll
          for (int side = 0; side < 2; ++side)
#pragma unroll
            for (int q = 0; q < K1; ++q) nxt[(2 * j + side) * K1 + q] = c1[side][q];
        } else {
#pragma unroll
          for (int side = 0; side < 2; ++side) {
            double c2[2][K1];
            up(c1[side], h + (K1 << n) + (2 * j + side) * K1, c2);
#pragma unroll
            for (int s2 = 0; s2 < 2; ++s2)
#pragma unroll
              for (int q = 0; q < K1; ++q) nxt[(4 * j + 2 * side + s2) * K1 + q] = c2[s2][q];
          }
        }
      }
      __syncthreads();
      n += two ? 2 : 1;
    }
  }
  // pointwise map cell by cell: values at the K1 points of finest cell c of
  // every pair, map, weights, projection onto the cell's K1 functions, into H
  // of (input 0, species s)
  const double dt2 = a.dt2;
  for (int it = tid; it < nl << N; it += nt) {
    const int ln = it >> N, c = it - (ln << N);
    double pv[2][2][K1];  // [input][species][point]
#pragma unroll
    for (int z = 0; z < 2; ++z)
#pragma unroll
      for (int s = 0; s < 2; ++s) {
        double cc[K1];
        if (z < nin && s < S) {
          const double* src = (N == 0 ? Hr(ln, z * S + s) : SAr(ln, z * S + s)) + c * K1;
#pragma unroll
          for (int p = 0; p < K1; ++p) cc[p] = src[p];
        } else {
#pragma unroll
          for (int p = 0; p < K1; ++p) cc[p] = 0.0;
        }
#pragma unroll
        for (int gq = 0; gq < K1; ++gq) {
          const double* e = EL + (c * K1 + gq) * K1;
          double u = 0.0;
#pragma unroll
          for (int p = 0; p < K1; ++p) u += cc[p] * e[p];
          pv[z][s][gq] = u;
        }
      }
    double ow[2][K1];
#pragma unroll
    for (int gq = 0; gq < K1; ++gq) {
      const double u[2] = {pv[0][0][gq], pv[0][1][gq]};
      const double g[2] = {pv[1][0][gq], pv[1][1][gq]};
      double o[2];
      rx_map(rx, S, mode, dt2, u, g, o);
      const double wq = w1[c * K1 + gq];
      ow[0][gq] = wq * o[0];
      ow[1][gq] = wq * o[1];
    }
#pragma unroll
    for (int s = 0; s < 2; ++s)
      if (s < S) {
        double* h = Hr(ln, s) + c * K1;
#pragma unroll
        for (int p = 0; p < K1; ++p) {
          double acc = 0.0;
#pragma unroll
          for (int gq = 0; gq < K1; ++gq) acc += ow[s][gq] * EL[(c * K1 + gq) * K1 + p];
          h[p] = acc;
        }
      }
  }
  __syncthreads();
  // one level of the forward transform: parent cell coefficients (sc) and
  // wavelets (wc) from the two children sl, sr
  auto down = [&](const double* sl, const double* sr, double* sc, double* wc) {
#pragma unroll
    for (int i = 0; i < K1; ++i) {
      double a0 = 0.0, a1 = 0.0;
#pragma unroll
      for (int q = 0; q < K1; ++q) {
        a0 += M[q * K1 + i] * sl[q] + M[16 + q * K1 + i] * sr[q];
        a1 += M[32 + i * K1 + q] * sl[q] + M[48 + i * K1 + q] * sr[q];
      }
      sc[i] = a0;
      wc[i] = a1;
    }
  };
  // forward transform, levels N..1, two per step (from the projections in H;
  // cell coefficients alternate SB / H, wavelets to SA at their final places)
  int st = 0;
  for (int n = N; n >= 1; ++st) {
    const bool two = n >= 2;
    const bool fromH = (st & 1) == 0;
    const int nb = two ? n - 2 : n - 1;  // items: cells of the coarser output level
    for (int it = tid; it < (S * nl) << nb; it += nt) {
      const int j = it & ((1 << nb) - 1), pl = it >> nb;
      const int s = pl & (S - 1), ln = pl >> ls;
      const double* cur = fromH ? Hr(ln, s) : SBr(ln, s);
      double* nxt = fromH ? SBr(ln, s) : Hr(ln, s);
      double* fw = SAr(ln, s);
      if (!two) {
        double sc[K1], wc[K1];
        down(cur + (2 * j) * K1, cur + (2 * j + 1) * K1, sc, wc);
#pragma unroll
        for (int i = 0; i < K1; ++i) {
          nxt[j * K1 + i] = sc[i];
          fw[(K1 << (n - 1)) + j * K1 + i] = wc[i];
        }
      } else {
        double s1[2][K1];
#pragma unroll
        for (int side = 0; side < 2; ++side) {
          double wc[K1];
          down(cur + (4 * j + 2 * side) * K1, cur + (4 * j + 2 * side + 1) * K1, s1[side], wc);
#pragma unroll
          for (int i = 0; i < K1; ++i) fw[(K1 << (n - 1)) + (2 * j + side) * K1 + i] = wc[i];
        }
        double sc[K1], wc[K1];
        down(s1[0], s1[1], sc, wc);
#pragma unroll
        for (int i = 0; i < K1; ++i) {
          nxt[j * K1 + i] = sc[i];
          fw[(K1 << (n - 2)) + j * K1 + i] = wc[i];
        }
      }
    }
    __syncthreads();
    n -= two ? 2 : 1;
  }
  // s_0 is where the last step (for N = 0: the projection) left it
  const bool s0H = st == 0 || ((st - 1) & 1) == 1;
  auto coef = [&](int ln, int s, int e) -> double {
    return e < K1 ? (s0H ? Hr(ln, s) : SBr(ln, s))[e] : SAr(ln, s)[e];
  };
  if (d >= 2) {
    for (int s = 0; s < S; ++s) {
      double* out = xr + I.Y_off[d - 1] + ((int64_t)s * I.npre[d - 1] + pre0) * n1;
      for (int i = tid; i < nl * n1; i += nt) {
        const int ln = (i / K1) >> N, e = i - ln * n1;
        out[i] = coef(ln, s, e);
      }
    }
  } else {
    double g2 = 0.0;
    for (int s = 0; s < S; ++s) {
      const int64_t base = (int64_t)rhs * total + I.seg + (int64_t)s * I.ndof;
      for (int i = tid; i < n1; i += nt) g2 += finish(a, mode, base + i, coef(0, s, i));
    }
    if (mode == RX_RESID) {
      g2 = block_sum(g2, wsum);
      if (tid == 0) a.part[(int64_t)rhs * nfin + fin_index] = g2;
    }
  }
}

// One workgroup per (tile, right-hand side) of one class of instances (same
// degree, level and species count, so one LDS layout); the class sets the
// workgroup size (64..256 threads, a few transform items per thread), so the
// tiles of short lines run as single waves whose barriers cost almost nothing.
template <int K1>
__global__ __launch_bounds__(RX_THREADS) void k_rx_line(RTables R, const LineTask* __restrict__ tasks, int ninst,
                                                        int mode, int64_t total, RxArgs a, int64_t rws, int nin,
                                                        int64_t nfin) {
  extern __shared__ double lds[];
  const int tid = threadIdx.x, nt = blockDim.x;
  const LineTask t = tasks[blockIdx.x];
  const int rhs = blockIdx.y;
  if (all_converged(a) || (a.conv && a.conv[rhs * ninst + t.inst])) return;
  const RInst& I = R.inst[t.inst];
  const int d = I.d, N = I.N, S = I.S, np1 = I.np1, n1 = I.n1;
  const int npair = nin * S;
  const int LSL = 5 * npair * (n1 / 2);
  {
    const double* __restrict__ ELg = R.EL + I.EL_off + (int64_t)N * np1 * K1;
    const double* __restrict__ wg = R.w1 + I.w_off;
    double* EL = lds + RX_TAIL;
    for (int e = tid; e < 64; e += nt) lds[e] = R.mats[I.mats_off + e];
    for (int e = tid; e < 32; e += nt) lds[64 + e] = (&I.rx[0][0][0])[e];
    for (int e = tid; e < np1 * K1; e += nt) EL[e] = ELg[e];
    for (int e = tid; e < np1; e += nt) EL[np1 * K1 + e] = wg[e];
  }
  double* L0 = lds + RX_TAIL + np1 * (K1 + 1);
  const double* xr = a.rws + (int64_t)rhs * rws;
  for (int pr = 0; pr < npair; ++pr) {
    const int z = pr / S, sp = pr - z * S;
    const double* __restrict__ in = d == 1 ? plan_in(a, z, (int64_t)rhs * total) + I.seg + (int64_t)sp * I.ndof
                                           : xr + I.X_off[d - 1] + (((int64_t)z * S + sp) * I.npre[d - 1] + t.pre0) * n1;
    for (int i = tid; i < t.nl * n1; i += nt) {
      const int ln = (i / K1) >> N, e = i - ln * n1;
      L0[(int64_t)ln * LSL + pr * n1 + e] = in[i];
    }
  }
  __syncthreads();
  rx_line_tile<K1>(I, mode, total, a, rws, nin, nfin, R.cum_fin[t.inst], rhs, t.pre0, t.nl, lds);
}

// Last axis, wave form (d >= 2, N <= RX_WLINE_MAXN): a group of lanes takes a
// whole line; each lane owns a subtree of the line's cells (its level-h cell,
// 2^h lanes per line, and the up to WL_CPL<K1> finest cells below it).  A
// wave copies its lines (a contiguous run) into its own LDS buffer with
// coalesced loads.  The inverse fast multiwavelet transform (two-scale
// relations) runs down each lane's path to its level-h cell (the same
// coarse cells in every lane of a line) and then through its subtree in
// registers; the lane evaluates its Gauss points, applies the map and the
// weighted projection, and the forward transform climbs its subtree in
// registers, then the levels above h with the sibling cell fetched from the
// neighbouring lane group by a shuffle (the first lane of a parent's group
// writes its wavelets).  The projections overwrite the line's inputs in the
// wave's buffer (every input is read before the first output is written) and
// go back to HBM as one run.  No barriers; tiles are walked in a grid-stride
// loop (a pass whose problems have converged costs one flag test per tile).
// The formulas are the line kernel's (the same two-scale, point and
// projection sums); some sums are taken in another order, so the two forms
// agree to rounding, not bit for bit.
typedef __attribute__((address_space(3))) void* lds_ptr;

template <int K1>
constexpr int wl_cpl() {
  return K1 == 2 ? 8 : 4;  // finest cells per lane (at most)
}

// f and (for the correction and local modes) its Jacobian at one point,
// summing only the nonzero coefficients of the reaction polynomial: mask has
// bit s*16 + 4a + b set where c[s][a][b] != 0 (a wave-uniform value, so the
// loop and the coefficient loads are scalar).  The terms are taken in the
// order of rx_f / rx_jac and the skipped ones are zeros, so the values agree
// with those to the last bit.
template <int S, bool JAC>
__device__ __forceinline__ void wl_fj(const double* __restrict__ rxc, uint64_t mask, const double* u, double* f,
                                         double (*J)[2]) {
  const double u0 = u[0], u1 = S > 1 ? u[1] : 0.0;
  const double p0[4] = {1.0, u0, u0 * u0, u0 * u0 * u0};
  const double p1[4] = {1.0, u1, u1 * u1, u1 * u1 * u1};
  double fa[2] = {0.0, 0.0}, j0[2] = {0.0, 0.0}, j1[2] = {0.0, 0.0};
  for (uint64_t m = mask; m; m &= m - 1) {
    const int t = __builtin_ctzll(m);
    const int sp = t >> 4, aa = (t >> 2) & 3, bb = t & 3;
    const double c = rxc[t];
    const double pa = aa == 0 ? p0[0] : (aa == 1 ? p0[1] : (aa == 2 ? p0[2] : p0[3]));
    const double pb = bb == 0 ? p1[0] : (bb == 1 ? p1[1] : (bb == 2 ? p1[2] : p1[3]));
    const double v = c * pa * pb;
    if (sp == 0) fa[0] += v; else fa[1] += v;
    if (JAC) {
      if (aa > 0) {
        const double pm = aa == 1 ? p0[0] : (aa == 2 ? p0[1] : p0[2]);
        const double w = c * aa * pm * pb;
        if (sp == 0) j0[0] += w; else j0[1] += w;
      }
      if (bb > 0) {
        const double pm = bb == 1 ? p1[0] : (bb == 2 ? p1[1] : p1[2]);
        const double w = c * bb * pa * pm;
        if (sp == 0) j1[0] += w; else j1[1] += w;
      }
    }
  }
  f[0] = fa[0];
  f[1] = fa[1];
  if (JAC) {
    J[0][0] = j0[0];
    J[0][1] = j1[0];
    J[1][0] = j0[1];
    J[1][1] = j1[1];
  }
}

// The pointwise map of a pass (as rx_map) with wl_fj.
template <int S>
__device__ __forceinline__ void wl_map(const double* __restrict__ rxc, uint64_t mask, int mode, double dt2,
                                          const double* u, const double* g, double* out) {
  if (mode == RX_CORR) {
    double f[2], J[2][2];
    wl_fj<S, true>(rxc, mask, u, f, J);
    if (S == 1) {
      out[0] = g[0] / (1.0 - dt2 * J[0][0]);
      out[1] = 0.0;
    } else {
      const double A = 1.0 - dt2 * J[0][0], Bq = -dt2 * J[0][1];
      const double C = -dt2 * J[1][0], D = 1.0 - dt2 * J[1][1];
      const double det = A * D - Bq * C;
      out[0] = (D * g[0] - Bq * g[1]) / det;
      out[1] = (A * g[1] - C * g[0]) / det;
    }
  } else if (mode == RX_LOCAL) {
    const double w0 = u[0], w1v = S > 1 ? u[1] : 0.0;
    const double wmag = fmax(1.0, fmax(fabs(w0), fabs(w1v)));
    double x[2] = {w0, w1v};
    for (int it = 0; it <= RX_LOCAL_MAX_ITER; ++it) {
      double f[2], J[2][2];
      wl_fj<S, true>(rxc, mask, x, f, J);
      const double g0 = x[0] - dt2 * f[0] - w0, g1 = S > 1 ? x[1] - dt2 * f[1] - w1v : 0.0;
      if (fmax(fabs(g0), fabs(g1)) <= RX_LOCAL_TOL * wmag || it == RX_LOCAL_MAX_ITER) break;
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
    wl_fj<S, false>(rxc, mask, u, out, nullptr);
  }
}


template <int K1, int S, int NIN>
__device__ __forceinline__ void rx_wline_body(const RTables& R, const LineTask* __restrict__ tasks, int ntask,
                                              int ninst, int mode, const RxArgs& a, int64_t rws, int64_t nwork) {
  constexpr int NP = S * NIN;
  constexpr int CP = wl_cpl<K1>();
  constexpr int WL = 64 * K1 * CP;  // doubles of a wave's lines per pair
  __shared__ double Ms[64];     // ML, MR, cL, cR (16 each, row length K1)
  __shared__ double rxs[32];    // reaction coefficients
  __shared__ double stage[RX_THREADS / 64][NP * WL];  // each wave's lines, inputs then projections
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63, nwv = RX_THREADS / 64;
  // per-instance state, reloaded when the workgroup's instance changes
  int loaded = -1;
  int N = 0, n1 = 0, h = 0, LPL = 1, cpl = 1, LPW = 1, Lc = 0;
  int64_t xoff = 0, yoff = 0, npre = 0;
  uint64_t mask = 0;
  double mL[K1][K1], mR[K1][K1], cL[K1][K1], cR[K1][K1];  // two-scale matrices
  double ELn[K1][K1], wgq[K1];  // finest-level basis at the K1 points of a cell (the same in every cell), weights
  if (all_converged(a)) return;
  for (int64_t w = blockIdx.x; w < nwork; w += gridDim.x) {
    const int rhs = (int)(w / ntask);
    const LineTask t = tasks[w - (int64_t)rhs * ntask];
    if (a.conv && a.conv[rhs * ninst + t.inst]) continue;
    if (t.inst != loaded) {
      const RInst& I = R.inst[t.inst];
      __syncthreads();
      if (threadIdx.x < 64) Ms[threadIdx.x] = R.mats[I.mats_off + threadIdx.x];
      if (threadIdx.x < 32) rxs[threadIdx.x] = (&I.rx[0][0][0])[threadIdx.x];
      __syncthreads();
      loaded = t.inst;
      const int d = I.d;
      N = I.N;
      n1 = I.n1;
      xoff = I.X_off[d - 1];
      yoff = I.Y_off[d - 1];
      npre = I.npre[d - 1];
      mask = __ballot(lane < 16 * S && rxs[min(lane, 31)] != 0.0);
      cpl = min(CP, 1 << N);
      h = N - (31 - __clz(cpl));  // level at which a lane owns one cell
      LPL = 1 << h;
      LPW = 64 / LPL;
      Lc = lane & (LPL - 1);
#pragma unroll
      for (int i = 0; i < K1; ++i)
#pragma unroll
        for (int j = 0; j < K1; ++j) {
          mL[i][j] = Ms[i * K1 + j];
          mR[i][j] = Ms[16 + i * K1 + j];
          cL[i][j] = Ms[32 + i * K1 + j];
          cR[i][j] = Ms[48 + i * K1 + j];
        }
      const double* __restrict__ ELg = R.EL + I.EL_off + (int64_t)N * I.np1 * K1;
#pragma unroll
      for (int gq = 0; gq < K1; ++gq) {
        wgq[gq] = R.w1[I.w_off + gq];
#pragma unroll
        for (int p = 0; p < K1; ++p) ELn[gq][p] = ELg[gq * K1 + p];
      }
    }
    // children (left, right) of a cell from its coefficients and wavelets
    auto up2 = [&](const double* sc, const double* wc, double* cl, double* cr) {
#pragma unroll
      for (int q = 0; q < K1; ++q) {
        double al = 0.0, ar = 0.0;
#pragma unroll
        for (int i = 0; i < K1; ++i) {
          al += mL[q][i] * sc[i];
          ar += mR[q][i] * sc[i];
        }
#pragma unroll
        for (int p = 0; p < K1; ++p) {
          al += cL[p][q] * wc[p];
          ar += cR[p][q] * wc[p];
        }
        cl[q] = al;
        cr[q] = ar;
      }
    };
    // parent coefficients and wavelets from the two children
    auto down = [&](const double* sl, const double* sr, double* pc, double* wc) {
#pragma unroll
      for (int i = 0; i < K1; ++i) {
        double a0 = 0.0, a1 = 0.0;
#pragma unroll
        for (int q = 0; q < K1; ++q) {
          a0 += mL[q][i] * sl[q] + mR[q][i] * sr[q];
          a1 += cL[i][q] * sl[q] + cR[i][q] * sr[q];
        }
        pc[i] = a0;
        wc[i] = a1;
      }
    };
    double* xr = a.rws + (int64_t)rhs * rws;
    const double dt2 = a.dt2;
    double* buf = stage[wv];
    for (int l0 = wv * LPW; l0 < t.nl; l0 += nwv * LPW) {
      const int li = lane / LPL;
      const int nline = min(LPW, t.nl - l0);
      const bool act = li < nline;
      const int64_t pre0 = t.pre0 + l0;
      // the wave's lines go straight from HBM to its LDS buffer (direct
      // global -> LDS loads, all issued before the one wait; 16 bytes per lane
      // and instruction when the run is 16-byte aligned, else 4)
      const int ne = nline * n1;
#pragma unroll
      for (int pr = 0; pr < NP; ++pr) {
        const int z = pr / S, sp = pr - z * S;
        const double* __restrict__ src = xr + xoff + (((int64_t)z * S + sp) * npre + pre0) * n1;
        double* dst = buf + pr * WL;
        if (((uintptr_t)src & 15) == 0 && (ne & 1) == 0) {
#pragma unroll
          for (int u = 0; u < WL / 128; ++u)
            if (2 * (64 * u + lane) < ne)
              __builtin_amdgcn_global_load_lds((const void*)(src + 2 * (64 * u + lane)), (lds_ptr)(dst + 128 * u), 16,
                                               0, 0);
        } else {
          const uint32_t* s4 = (const uint32_t*)src;
          for (int u = 0; u < WL / 32; ++u)
            if (64 * u + lane < 2 * ne)
              __builtin_amdgcn_global_load_lds((const void*)(s4 + 64 * u + lane), (lds_ptr)(dst + 32 * u), 4, 0, 0);
        }
      }
      __builtin_amdgcn_s_waitcnt(0);  // the direct loads have landed
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      const int lq = act ? li : 0;
      // inverse transform: down the path to the lane's level-h cell, then its subtree
      double fin[NP][CP][K1];
#pragma unroll
      for (int pr = 0; pr < NP; ++pr) {
        const double* xl = buf + pr * WL + lq * n1;
        double sc[K1];
#pragma unroll
        for (int p = 0; p < K1; ++p) sc[p] = xl[p];
        for (int n = 1; n <= h; ++n) {
          const int jp = Lc >> (h - n + 1), side = (Lc >> (h - n)) & 1;
          double wc[K1], cl[K1], cr[K1];
#pragma unroll
          for (int p = 0; p < K1; ++p) wc[p] = xl[(K1 << (n - 1)) + jp * K1 + p];
          up2(sc, wc, cl, cr);
#pragma unroll
          for (int q = 0; q < K1; ++q) sc[q] = side ? cr[q] : cl[q];
        }
#pragma unroll
        for (int q = 0; q < K1; ++q) fin[pr][0][q] = sc[q];
        // subtree levels h+1..N: cells of level n below the lane's cell are
        // Lc 2^(n-h) + c, c < 2^(n-h); expanded in place from the last parent down
#pragma unroll
        for (int g = 1; g < CP; g *= 2)
          if (g < cpl) {
            const int n = h + 1 + (31 - __clz(g));  // level formed in this round (g parents)
#pragma unroll
            for (int c = CP / 2 - 1; c >= 0; --c)
              if (c < g) {
                double wc[K1], cl[K1], cr[K1];
#pragma unroll
                for (int p = 0; p < K1; ++p) wc[p] = xl[(K1 << (n - 1)) + (Lc * g + c) * K1 + p];
                up2(fin[pr][c], wc, cl, cr);
#pragma unroll
                for (int q = 0; q < K1; ++q) {
                  fin[pr][2 * c][q] = cl[q];
                  fin[pr][2 * c + 1][q] = cr[q];
                }
              }
          }
      }
      // values at the Gauss points, the map, weights, projection onto the cell's functions
      double pj[S][CP][K1];
#pragma unroll
      for (int tc = 0; tc < CP; ++tc)
        if (tc < cpl) {
          double ow[2][K1];
#pragma unroll
          for (int gq = 0; gq < K1; ++gq) {
            double u[NP];
#pragma unroll
            for (int pr = 0; pr < NP; ++pr) {
              double v = 0.0;
#pragma unroll
              for (int p = 0; p < K1; ++p) v += fin[pr][tc][p] * ELn[gq][p];
              u[pr] = v;
            }
            // pair z S + s: input z, species s
            double uu[2] = {u[0], 0.0}, gg[2] = {0.0, 0.0};
            if (S > 1) uu[1] = u[S > 1 ? 1 : 0];
            if (NIN > 1) gg[0] = u[NIN > 1 ? S : 0];
            if (NIN > 1 && S > 1) gg[1] = u[NP - 1];
            double o[2];
            wl_map<S>(rxs, mask, mode, dt2, uu, gg, o);
            ow[0][gq] = wgq[gq] * o[0];
            ow[1][gq] = wgq[gq] * o[1];
          }
#pragma unroll
          for (int sp = 0; sp < S; ++sp)
#pragma unroll
            for (int p = 0; p < K1; ++p) {
              double acc = 0.0;
#pragma unroll
              for (int gq = 0; gq < K1; ++gq) acc += ow[sp][gq] * ELn[gq][p];
              pj[sp][tc][p] = acc;
            }
        }
      // every input of the wave's lines has been read: the projections go to
      // the buffers of input 0 (pair sp)
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      // forward transform: the subtree in registers, then the levels above h
#pragma unroll
      for (int sp = 0; sp < S; ++sp) {
        double* yl = buf + sp * WL + lq * n1;
#pragma unroll
        for (int g = CP / 2; g >= 1; g /= 2)
          if (g < cpl) {
            const int n = h + 1 + (31 - __clz(g));  // level of the children combined in this round
#pragma unroll
            for (int c = 0; c < CP / 2; ++c)
              if (c < g) {
                double pc[K1], wc[K1];
                down(pj[sp][2 * c], pj[sp][2 * c + 1], pc, wc);
                if (act)
#pragma unroll
                  for (int p = 0; p < K1; ++p) yl[(K1 << (n - 1)) + (Lc * g + c) * K1 + p] = wc[p];
#pragma unroll
                for (int p = 0; p < K1; ++p) pj[sp][c][p] = pc[p];
              }
          }
        double sc[K1];
#pragma unroll
        for (int p = 0; p < K1; ++p) sc[p] = pj[sp][0][p];
        for (int n = h; n >= 1; --n) {
          const int off = 1 << (h - n), j = Lc >> (h - n);
          double sib[K1], pc[K1], wc[K1];
#pragma unroll
          for (int p = 0; p < K1; ++p) sib[p] = __shfl_xor(sc[p], off, 64);
          if (j & 1)
            down(sib, sc, pc, wc);
          else
            down(sc, sib, pc, wc);
          if (act && (Lc & (2 * off - 1)) == 0)
#pragma unroll
            for (int p = 0; p < K1; ++p) yl[(K1 << (n - 1)) + (j >> 1) * K1 + p] = wc[p];
#pragma unroll
          for (int p = 0; p < K1; ++p) sc[p] = pc[p];
        }
        if (act && Lc == 0)
#pragma unroll
          for (int p = 0; p < K1; ++p) yl[p] = sc[p];
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
      for (int sp = 0; sp < S; ++sp) {
        double* __restrict__ dst = xr + yoff + ((int64_t)sp * npre + pre0) * n1;
#pragma unroll
        for (int u0 = 0; u0 < WL / 64; u0 += 4) {
          double v[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) v[u] = buf[sp * WL + lane + 64 * (u0 + u)];
#pragma unroll
          for (int u = 0; u < 4; ++u)
            if (lane + 64 * (u0 + u) < ne) dst[lane + 64 * (u0 + u)] = v[u];
        }
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
  }
}

// The wave-form kernel with the compiler's register allocation, and with at
// most 168 VGPRs (three waves per SIMD, spilling what does not fit): which
// is faster depends on the instantiation and is measured by the autotuner.
template <int K1, int S, int NIN>
__global__ __launch_bounds__(RX_THREADS) void k_rx_wline(RTables R, const LineTask* __restrict__ tasks, int ntask,
                                                         int ninst, int mode, RxArgs a, int64_t rws, int64_t nwork) {
  rx_wline_body<K1, S, NIN>(R, tasks, ntask, ninst, mode, a, rws, nwork);
}
template <int K1, int S, int NIN>
__global__ __launch_bounds__(RX_THREADS) __attribute__((amdgpu_waves_per_eu(3))) void k_rx_wline_w3(
    RTables R, const LineTask* __restrict__ tasks, int ntask, int ninst, int mode, RxArgs a, int64_t rws,
    int64_t nwork) {
  rx_wline_body<K1, S, NIN>(R, tasks, ntask, ninst, mode, a, rws, nwork);
}

// The last-axis launch of one class of instances in a pass.
static void launch_line(const sgdg_plan* plan, const LineClass& lc, int nrhs, RxMode mode, const RxArgs& a,
                        hipStream_t s) {
  const RHost* rh = (const RHost*)plan->rdata;
  const int ninst = plan->ninst;
  const int nin = mode == RX_CORR ? 2 : 1;
  const int64_t nfin = rh->cum_fin.back();
  if (lc.wave) {
    const int ntask = (int)lc.tasks[nin].size();
    const int64_t nwork = (int64_t)ntask * nrhs;
    const unsigned grid = (unsigned)std::min<int64_t>(nwork, (int64_t)std::max(rh->ncu, 1) * lc.wgcu[nin]);
    auto wl = [&](auto k1, auto sp, auto ni) {
      constexpr int K1 = decltype(k1)::value, S = decltype(sp)::value, NIN = decltype(ni)::value;
      if (lc.waves[nin] == 3)
        hipLaunchKernelGGL((k_rx_wline_w3<K1, S, NIN>), dim3(grid), dim3(RX_THREADS), 0, s, rh->dev, lc.dev[nin],
                           ntask, ninst, (int)mode, a, rh->rws, nwork);
      else
        hipLaunchKernelGGL((k_rx_wline<K1, S, NIN>), dim3(grid), dim3(RX_THREADS), 0, s, rh->dev, lc.dev[nin], ntask,
                           ninst, (int)mode, a, rh->rws, nwork);
    };
    auto by_s = [&](auto k1) {
      if (lc.S == 1) {
        if (nin == 1) wl(k1, std::integral_constant<int, 1>(), std::integral_constant<int, 1>());
        else wl(k1, std::integral_constant<int, 1>(), std::integral_constant<int, 2>());
      } else {
        if (nin == 1) wl(k1, std::integral_constant<int, 2>(), std::integral_constant<int, 1>());
        else wl(k1, std::integral_constant<int, 2>(), std::integral_constant<int, 2>());
      }
    };
    if (lc.K1 == 2) by_s(std::integral_constant<int, 2>());
    else if (lc.K1 == 3) by_s(std::integral_constant<int, 3>());
    else by_s(std::integral_constant<int, 4>());
    return;
  }
  const dim3 grid((unsigned)lc.tasks[nin].size(), (unsigned)nrhs), blk((unsigned)lc.threads[nin]);
  switch (lc.K1) {
    case 2:
      hipLaunchKernelGGL(k_rx_line<2>, grid, blk, lc.lds[nin], s, rh->dev, lc.dev[nin], ninst, (int)mode, plan->total,
                         a, rh->rws, nin, nfin);
      break;
    case 3:
      hipLaunchKernelGGL(k_rx_line<3>, grid, blk, lc.lds[nin], s, rh->dev, lc.dev[nin], ninst, (int)mode, plan->total,
                         a, rh->rws, nin, nfin);
      break;
    default:
      hipLaunchKernelGGL(k_rx_line<4>, grid, blk, lc.lds[nin], s, rh->dev, lc.dev[nin], ninst, (int)mode, plan->total,
                         a, rh->rws, nin, nfin);
      break;
  }
}

void reaction_pass(const sgdg_plan* plan, int nrhs, RxMode mode, const RxArgs& a, hipStream_t s,
                   const std::function<void(int)>* mark) {
  const RHost* rh = (const RHost*)plan->rdata;
  const int d = plan->d, ninst = plan->ninst;
  const int nin = mode == RX_CORR ? 2 : 1;
  const int64_t nfin = rh->cum_fin.back();
  // every degree present in the plan gets its own launch of each stage
  auto each = [&](auto launch) {
    if (rh->k1mask & 4) launch(std::integral_constant<int, 2>());
    if (rh->k1mask & 8) launch(std::integral_constant<int, 3>());
    if (rh->k1mask & 16) launch(std::integral_constant<int, 4>());
  };
  using std::integral_constant;
  // a stage launch with its level bucket and its lane-chunk or LDS-staging
  // form picked at run time (lane chunks and staging never meet: staging
  // needs lam <= 2)
  auto forms = [&](int K1, int m, bool xs, auto go) {
    auto lm = [&](auto lanes, auto stg) {
      switch (rh->lm[K1]) {
        case 7: go(integral_constant<int, 7>(), lanes, stg); break;
        case 9: go(integral_constant<int, 9>(), lanes, stg); break;
        default: go(integral_constant<int, RX_LMAX>(), lanes, stg); break;
      }
    };
    if (rh->llane[m] > 0) lm(integral_constant<bool, true>(), integral_constant<bool, false>());
    else if (xs) lm(integral_constant<bool, false>(), integral_constant<bool, true>());
    else lm(integral_constant<bool, false>(), integral_constant<bool, false>());
  };
  for (int m = 0; m + 1 <= d - 1; ++m)
    each([&](auto k1) {
      if (mark) (*mark)(0);
      const int xs = rh->xs_lds[m];
      forms(decltype(k1)::value, m, xs > 0, [&](auto lmv, auto lanes, auto stg) {
        auto k = k_rx_expand<decltype(k1)::value, decltype(lmv)::value, decltype(lanes)::value, decltype(stg)::value>;
        const int64_t nt = rh->cum_x[m].back();
        const dim3 grid((unsigned)(stg ? (nt + RX_XS_TILES - 1) / RX_XS_TILES : nt), (unsigned)nrhs, (unsigned)nin);
        hipLaunchKernelGGL(k, grid, dim3(RX_THREADS), stg ? RX_XS_TILES * xs : 0, s, rh->dev,
                           (const double*)rh->dev.EH, ninst, m, plan->total, a, rh->rws, rh->lam[m], rh->llane[m],
                           xs / (int)sizeof(double));
      });
    });
  for (const LineClass& lc : rh->lclass) {
    if (mark) (*mark)(1);
    launch_line(plan, lc, nrhs, mode, a, s);
  }
  for (int m = d - 2; m >= 0; --m)
    each([&](auto k1) {
      if (mark) (*mark)(2);
      const int xs = m > 0 ? rh->xs_lds[m] : 0;
      forms(decltype(k1)::value, m, xs > 0, [&](auto lmv, auto lanes, auto stg) {
        auto k =
            k_rx_contract<decltype(k1)::value, decltype(lmv)::value, decltype(lanes)::value, decltype(stg)::value>;
        const int64_t nt = rh->cum_x[m].back();
        const dim3 grid((unsigned)(stg ? (nt + RX_XS_TILES_CON - 1) / RX_XS_TILES_CON : nt), (unsigned)nrhs);
        hipLaunchKernelGGL(k, grid, dim3(RX_THREADS), stg ? RX_XS_TILES_CON * xs : 0, s, rh->dev,
                           (const double*)rh->dev.EH, (const double*)rh->dev.w1, ninst, m, (int)mode, plan->total, a,
                           rh->rws, rh->lam[m], rh->llane[m], nfin, xs / (int)sizeof(double));
      });
    });
  if (mark) (*mark)(-1);
}

int reaction_line_classes(const sgdg_plan* plan) {
  const RHost* rh = (const RHost*)plan->rdata;
  return rh->supported ? (int)rh->lclass.size() : 0;
}
const LineClass& reaction_line_class(const sgdg_plan* plan, int c) { return ((const RHost*)plan->rdata)->lclass[c]; }

sgdg_status reaction_set_line_shape(sgdg_plan* plan, int c, int nin, int rounds, int wgcu, int waves) {
  RHost* rh = (RHost*)plan->rdata;
  if (!rh->supported || c < 0 || c >= (int)rh->lclass.size() || nin < 1 || nin > 2)
    return fail(SGDG_ERR_ARG, "line shape: no such class");
  LineClass& lc = rh->lclass[c];
  if (!lc.wave) return fail(SGDG_ERR_UNSUPPORTED, "line shape: the class runs the LDS-tile form");
  if (rounds < 1 || rounds > RX_WLINE_MAXROUNDS || wgcu < 1 || wgcu > 64)
    return fail(SGDG_ERR_ARG, "line shape: rounds must be in 1..64 and workgroups per CU in 1..64");
  if (waves != 0 && waves != 3) return fail(SGDG_ERR_ARG, "line shape: waves per SIMD must be 0 (compiler's) or 3");
  std::vector<LineTask> t = wave_tiles(lc, rounds);
  if (t.size() > lc.cap_tasks[nin]) return fail(SGDG_ERR_ARG, "line shape: too many tiles");
  const hipError_t e = hipMemcpy(lc.dev[nin], t.data(), t.size() * sizeof(LineTask), hipMemcpyHostToDevice);
  if (e != hipSuccess) return hip_fail(e, "hipMemcpy(line tiles)");
  lc.tasks[nin].swap(t);
  lc.rounds[nin] = rounds;
  lc.wgcu[nin] = wgcu;
  lc.waves[nin] = waves;
  return SGDG_OK;
}

void reaction_line_stage(const sgdg_plan* plan, int nrhs, RxMode mode, const RxArgs& a, hipStream_t s, int c) {
  launch_line(plan, ((const RHost*)plan->rdata)->lclass[c], nrhs, mode, a, s);
}

static sgdg_status set_line_lds(const RHost* rh) {
  int ll = 0;
  for (const LineClass& lc : rh->lclass) ll = std::max(ll, (int)std::max(lc.lds[1], lc.lds[2]));
  hipError_t e = hipFuncSetAttribute((const void*)k_rx_line<2>, hipFuncAttributeMaxDynamicSharedMemorySize, ll);
  if (e == hipSuccess)
    e = hipFuncSetAttribute((const void*)k_rx_line<3>, hipFuncAttributeMaxDynamicSharedMemorySize, ll);
  if (e == hipSuccess)
    e = hipFuncSetAttribute((const void*)k_rx_line<4>, hipFuncAttributeMaxDynamicSharedMemorySize, ll);
  if (e != hipSuccess) return hip_fail(e, "hipFuncSetAttribute(reaction line kernel LDS)");
  return SGDG_OK;
}

}  // namespace sgdg
