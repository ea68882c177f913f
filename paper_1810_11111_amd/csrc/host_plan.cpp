// Plan construction, host queries and initial-data projection.
//
// Index set (Sec. 2.1, eqs. 2.7-2.9): level blocks l with |l|_1 <= N, each a
// tensor of 1D hierarchical functions (eq. 2.8); canonical order as documented
// in sgdg.h.  Everything is built once on the host and uploaded (the paper
// assembles its 1D integrals once before the time evolution, Sec. 4 intro).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <functional>
#include <numeric>

#include "internal.h"

namespace sgdg {

static thread_local std::string g_last_error;

sgdg_status fail(sgdg_status st, const std::string& msg) {
  g_last_error = msg;
  return st;
}

sgdg_status hip_fail(hipError_t e, const char* what) {
  g_last_error = std::string(what) + ": " + hipGetErrorString(e);
  return SGDG_ERR_HIP;
}

size_t krylov_ws_bytes(const sgdg_plan* plan, int M, int nrhs);
size_t iif2_ws_bytes(const sgdg_plan* plan, int M, int nrhs);
sgdg_status reaction_build(sgdg_plan* plan);
void reaction_destroy(sgdg_plan* plan);

namespace {

std::vector<std::vector<int>> level_blocks(int d, int N) {
  std::vector<std::vector<int>> out;
  std::vector<int> l(d, 0);
  std::function<void(int, int)> rec = [&](int m, int rem) {
    if (m == d) {
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

// Lanes per output element for every block of an instance.  The work of an
// output is the number of row entries the sweep walks for it, summed over
// directions: in direction m, the entries of the 1D row of its target cell
// whose source cell lies within the level budget N - |l|_1 + l_m (maximum
// over the block's cells).  A coarse level's rows reach every finer cell
// under its support, so its work is up to ~2^(N - |l|_1) times that of the
// finest level; such blocks get lanes in proportion (powers of two, from
// APPLY_G up to APPLY_GMAX) so that no output needs more than about twice
// the iterations of a finest-level output.
std::vector<int> block_lanes(const sgdg_plan* p, const HostInstance& hi) {
  const int d = hi.desc.d, N = hi.desc.n;
  std::vector<int64_t> work(hi.blocks.size(), 0);
  int64_t wfine = 1;
  for (size_t b = 0; b < hi.blocks.size(); ++b) {
    const std::vector<int>& lev = hi.blocks[b];
    const int lsum = std::accumulate(lev.begin(), lev.end(), 0);
    int64_t w = 0;
    for (int m = 0; m < d; ++m) {
      const Op1D& op = p->ops[hi.dir_tab[m]];
      const int32_t lim = 1 << (N - lsum + lev[m]);
      const int l = lev[m];
      const int c_lo = l == 0 ? 0 : 1 << (l - 1), c_hi = l == 0 ? 1 : 1 << l;
      int64_t mx = 0;
      for (int c = c_lo; c < c_hi; ++c) {
        const int32_t* r0 = op.src.data() + op.cptr[c];
        const int32_t* r1 = op.src.data() + op.cptr[c + 1];
        mx = std::max<int64_t>(mx, std::lower_bound(r0, r1, lim) - r0);
      }
      w += mx;
    }
    work[b] = w;
    if (lsum == N) wfine = std::max(wfine, w);
  }
  std::vector<int> lanes(hi.blocks.size(), APPLY_G);
  for (size_t b = 0; b < hi.blocks.size(); ++b) {
    int g = APPLY_G;
    while (g < APPLY_GMAX && work[b] * APPLY_G > 2 * wfine * g) g *= 2;
    lanes[b] = g;
  }
  return lanes;
}

template <class T>
sgdg_status upload(sgdg_plan* p, const std::vector<T>& v, T** out) {
  size_t bytes = std::max<size_t>(1, v.size()) * sizeof(T);
  void* d = nullptr;
  hipError_t e = hipMalloc(&d, bytes);
  if (e != hipSuccess) return hip_fail(e, "hipMalloc(plan table)");
  p->allocations.push_back(d);
  if (!v.empty()) {
    e = hipMemcpy(d, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpy(plan table)");
  }
  *out = static_cast<T*>(d);
  return SGDG_OK;
}

}  // namespace

sgdg_status plan_upload(sgdg_plan* p, const void* src, size_t bytes, void** out) {
  void* d = nullptr;
  hipError_t e = hipMalloc(&d, std::max<size_t>(bytes, 1));
  if (e != hipSuccess) return hip_fail(e, "hipMalloc(plan table)");
  p->allocations.push_back(d);
  if (bytes) {
    e = hipMemcpy(d, src, bytes, hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpy(plan table)");
  }
  *out = d;
  return SGDG_OK;
}

}  // namespace sgdg

using namespace sgdg;

extern "C" const char* sgdg_last_error(void) { return g_last_error.c_str(); }

extern "C" sgdg_status sg_dg_destroy(sgdg_plan* plan) {
  if (!plan) return fail(SGDG_ERR_ARG, "sg_dg_destroy: null plan");
  hipDeviceSynchronize();
  reaction_destroy(plan);
  fibre_destroy(plan);
  for (void* p : plan->allocations) hipFree(p);
  delete plan;
  return SGDG_OK;
}

extern "C" sgdg_status sg_dg_build(const sgdg_desc* descs, int32_t ninst, int32_t prec, sgdg_plan** out) {
  if (!out) return fail(SGDG_ERR_ARG, "sg_dg_build: null output pointer");
  *out = nullptr;
  if (!descs || ninst <= 0) return fail(SGDG_ERR_ARG, "sg_dg_build: need at least one descriptor");
  if (prec < SGDG_FP64 || prec > SGDG_BF16_SWEEP) return fail(SGDG_ERR_ARG, "sg_dg_build: unknown precision");
  const int d = descs[0].d;
  for (int i = 0; i < ninst; ++i) {
    const sgdg_desc& ds = descs[i];
    if (ds.d < 1 || ds.d > SGDG_MAX_D) return fail(SGDG_ERR_ARG, "sg_dg_build: d must be in 1..6");
    if (ds.d != d) return fail(SGDG_ERR_ARG, "sg_dg_build: all instances of a plan must share d");
    if (ds.n < 0 || ds.n > 20) return fail(SGDG_ERR_ARG, "sg_dg_build: level N must be in 0..20");
    if (ds.k < 1 || ds.k > SGDG_MAX_K) return fail(SGDG_ERR_ARG, "sg_dg_build: degree k must be in 1..3");
    if (ds.nspecies < 1 || ds.nspecies > 2) return fail(SGDG_ERR_ARG, "sg_dg_build: nspecies must be 1 or 2");
    if (ds.bc != 0 && ds.bc != 1) return fail(SGDG_ERR_ARG, "sg_dg_build: bc must be 0 (periodic) or 1 (zero Dirichlet)");
    for (int s = 0; s < ds.nspecies; ++s)
      if (!(ds.D[s] > 0.0) || !std::isfinite(ds.D[s])) return fail(SGDG_ERR_ARG, "sg_dg_build: D_s must be positive");
    if (ds.kdiag)
      for (int m = 0; m < d; ++m) {
        const sgdg_kdiag& kd = ds.kdiag[m];
        if (!(kd.a0 - std::fabs(kd.a1) > 0.0)) return fail(SGDG_ERR_ARG, "sg_dg_build: k_ii must stay positive");
      }
    // work limit: ndof computed below must fit the 32-bit block sizes
  }
  int dev = 0;
  hipError_t he = hipGetDevice(&dev);
  if (he != hipSuccess) return hip_fail(he, "hipGetDevice");

  sgdg_plan* p = new sgdg_plan();
  p->ninst = ninst;
  p->d = d;
  p->prec = prec;
  p->device = dev;
  int64_t offset = 0;
  for (int i = 0; i < ninst; ++i) {
    HostInstance hi;
    hi.desc = descs[i];
    hi.desc.kdiag = nullptr;
    if (!(hi.desc.sigma > 0.0)) hi.desc.sigma = 20.0;
    for (int m = 0; m < d; ++m) hi.kdiag.push_back(descs[i].kdiag ? descs[i].kdiag[m] : sgdg_kdiag{1.0, 0.0, 0.0, 0.0});
    const int N = hi.desc.n, K1 = hi.desc.k + 1;
    hi.blocks = level_blocks(d, N);
    int64_t st = 0;
    for (auto& l : hi.blocks) {
      int64_t sz = 1;
      for (int m = 0; m < d; ++m) sz *= (int64_t)level_count(l[m]) * K1;
      if (sz > (int64_t)1 << 30) {
        delete p;
        return fail(SGDG_ERR_UNSUPPORTED, "sg_dg_build: level block too large");
      }
      hi.bstart.push_back(st);
      hi.bsize.push_back((int32_t)sz);
      st += sz;
    }
    hi.ndof = st;
    hi.offset = offset;
    int64_t np = 1;
    for (int m = 0; m < d; ++m) np *= (int64_t)K1 << N;
    hi.npoints = np;
    offset += hi.desc.nspecies * hi.ndof;
    // 1D operators per direction, shared between identical (N, k, sigma, bc, kdiag)
    for (int m = 0; m < d; ++m) {
      const sgdg_kdiag& kd = hi.kdiag[m];
      int found = -1;
      for (size_t o = 0; o < p->ops.size(); ++o) {
        const Op1D& op = p->ops[o];
        if (op.N == N && op.k == hi.desc.k && op.sigma == hi.desc.sigma && op.bc == hi.desc.bc && op.kd[0] == kd.a0 &&
            op.kd[1] == kd.a1 && op.kd[2] == kd.freq && op.kd[3] == kd.phase)
          found = (int)o;
      }
      if (found < 0) {
        p->ops.push_back(build_op1d(N, hi.desc.k, hi.desc.sigma, kd, hi.desc.bc));
        found = (int)p->ops.size() - 1;
      }
      hi.dir_tab.push_back(found);
    }
    p->inst.push_back(std::move(hi));
  }
  p->total = offset;

  // ||A_s||_inf: the row sum of a DOF is sum_i rowabs_i(r_i, N - |l| + l_i); its
  // maximum over a block separates over the axes.
  std::vector<std::vector<double>> rowabs(p->ops.size());
  for (size_t o = 0; o < p->ops.size(); ++o) {
    const Op1D& op = p->ops[o];
    const int K1 = op.k + 1, K2 = K1 * K1, N = op.N;
    const long nc = 1L << N;
    auto& ra = rowabs[o];
    ra.assign(nc * K1 * (N + 1), 0.0);
    for (long t = 0; t < nc; ++t)
      for (int e = op.cptr[t]; e < op.cptr[t + 1]; ++e) {
        long sc = op.src[e];
        int slev = 0;
        while (slev < 31 && (1L << slev) <= sc) ++slev;  // level of source cell (0 for cell 0)
        for (int pt = 0; pt < K1; ++pt) {
          double s = 0;
          for (int ps = 0; ps < K1; ++ps) s += std::fabs(op.val[(size_t)e * K2 + pt * K1 + ps]);
          for (int b = slev; b <= N; ++b) ra[(t * K1 + pt) * (N + 1) + b] += s;
        }
      }
  }
  for (auto& hi : p->inst) {
    const int N = hi.desc.n, K1 = hi.desc.k + 1;
    double best = 0;
    for (auto& l : hi.blocks) {
      int ls = std::accumulate(l.begin(), l.end(), 0);
      double tot = 0;
      for (int m = 0; m < d; ++m) {
        const auto& ra = rowabs[hi.dir_tab[m]];
        int budget = N - ls + l[m];
        long c0 = l[m] == 0 ? 0 : (1L << (l[m] - 1));
        double mx = 0;
        for (long j = 0; j < level_count(l[m]); ++j)
          for (int pt = 0; pt < K1; ++pt) mx = std::max(mx, ra[((c0 + j) * K1 + pt) * (N + 1) + budget]);
        tot += mx;
      }
      best = std::max(best, tot);
    }
    for (int s = 0; s < hi.desc.nspecies; ++s) hi.anorm[s] = hi.desc.D[s] * best;
  }

  // global blocks, chunks, per-instance device constants
  std::vector<int32_t> blkid;
  std::vector<int64_t> lstart;
  std::vector<BCsr> bcsr;
  std::vector<int32_t> cptr_all, src_all;
  std::vector<double> val_all;
  std::vector<int64_t> op_cptr_off(p->ops.size()), op_src_off(p->ops.size()), op_val_off(p->ops.size());
  for (size_t o = 0; o < p->ops.size(); ++o) {
    op_cptr_off[o] = (int64_t)cptr_all.size();
    op_src_off[o] = (int64_t)src_all.size();
    op_val_off[o] = (int64_t)val_all.size();
    cptr_all.insert(cptr_all.end(), p->ops[o].cptr.begin(), p->ops[o].cptr.end());
    src_all.insert(src_all.end(), p->ops[o].src.begin(), p->ops[o].src.end());
    val_all.insert(val_all.end(), p->ops[o].val.begin(), p->ops[o].val.end());
  }
  if (cptr_all.size() > (size_t)INT32_MAX || src_all.size() > (size_t)INT32_MAX) {
    delete p;
    return fail(SGDG_ERR_UNSUPPORTED, "sg_dg_build: operator tables too large");
  }
  for (int i = 0; i < ninst; ++i) {
    HostInstance& hi = p->inst[i];
    const int N = hi.desc.n;
    InstDev id{};
    id.N = N;
    id.k = hi.desc.k;
    id.S = hi.desc.nspecies;
    id.nb = (int32_t)hi.blocks.size();
    id.offset = hi.offset;
    id.ndof = hi.ndof;
    id.D[0] = hi.desc.D[0];
    id.D[1] = hi.desc.nspecies > 1 ? hi.desc.D[1] : 0.0;
    id.n1 = (hi.desc.k + 1) << N;
    std::memcpy(id.rx, hi.desc.rx, sizeof(id.rx));
    id.anorm[0] = hi.anorm[0];
    id.anorm[1] = hi.anorm[1];
    int pw = 1;
    for (int m = d - 1; m >= 0; --m) {
      id.pow[m] = pw;
      pw *= (N + 1);
    }
    id.blkid_off = (int32_t)blkid.size();
    std::vector<int32_t> tab(pw, -1);
    for (size_t b = 0; b < hi.blocks.size(); ++b) {
      int lin = 0;
      for (int m = 0; m < d; ++m) lin += hi.blocks[b][m] * id.pow[m];
      tab[lin] = (int32_t)lstart.size() + (int32_t)b;
    }
    // blkid entries index the global lstart table directly
    blkid.insert(blkid.end(), tab.begin(), tab.end());
    for (size_t b = 0; b < hi.blocks.size(); ++b) lstart.push_back(hi.bstart[b]);
    for (int m = 0; m < d; ++m) {
      int o = hi.dir_tab[m];
      id.bcsr_off[m] = (int32_t)bcsr.size();
      BCsr bc{};
      bc.cptr_off = op_cptr_off[o];
      bc.src_off = op_src_off[o];
      bc.val_off = op_val_off[o];
      bc.ncell = 1 << N;
      bc.k = hi.desc.k;
      bc.nnzb = (int32_t)p->ops[o].src.size();
      bcsr.push_back(bc);
    }
    id.gblk_off = (int32_t)p->gblk.size();
    for (int s = 0; s < hi.desc.nspecies; ++s) {
      int32_t seg_first = (int32_t)p->gblk.size();
      for (size_t b = 0; b < hi.blocks.size(); ++b) {
        GBlock g{};
        g.start = hi.offset + (int64_t)s * hi.ndof + hi.bstart[b];
        g.size = hi.bsize[b];
        g.inst = i;
        g.species = s;
        g.lsum = std::accumulate(hi.blocks[b].begin(), hi.blocks[b].end(), 0);
        for (int m = 0; m < d; ++m) {
          g.lev[m] = hi.blocks[b][m];
          g.ext[m] = level_count(hi.blocks[b][m]) * (hi.desc.k + 1);
        }
        p->gblk.push_back(g);
      }
      // chunks of this species segment: runs of consecutive elements whose
      // blocks share a lane count, at most CHUNK * APPLY_G / lanes elements
      int64_t segstart = hi.offset + (int64_t)s * hi.ndof;
      const std::vector<int> lanes = block_lanes(p, hi);
      int64_t c0 = 0;
      size_t bi = 0;
      while (c0 < hi.ndof) {
        while (hi.bstart[bi] + hi.bsize[bi] <= c0) ++bi;
        const int g = lanes[bi];
        const int64_t cap = CHUNK * APPLY_G / g;
        int64_t end = c0;
        size_t bj = bi;
        while (end < hi.ndof && end - c0 < cap) {
          while (hi.bstart[bj] + hi.bsize[bj] <= end) ++bj;
          if (lanes[bj] != g) break;
          end = std::min<int64_t>(hi.bstart[bj] + hi.bsize[bj], c0 + cap);
        }
        Chunk ch{};
        ch.start = segstart + c0;
        ch.count = (int32_t)(end - c0);
        int32_t b = seg_first;
        while (p->gblk[b].start + p->gblk[b].size <= ch.start) ++b;
        ch.b0 = b;
        int32_t b1 = b;
        while (p->gblk[b1].start + p->gblk[b1].size < ch.start + ch.count) ++b1;
        ch.b1 = b1;
        ch.inst = i;
        ch.species = s;
        ch.problem = i * 2 + s;
        ch.g = g;
        p->chunks.push_back(ch);
        c0 = end;
      }
    }
    p->instdev.push_back(id);
  }
  p->nchunks = (int32_t)p->chunks.size();
  p->nblocks = (int32_t)p->gblk.size();
  std::vector<int32_t> pc0(2 * ninst, 0), pnc(2 * ninst, 0);
  for (int32_t c = p->nchunks - 1; c >= 0; --c) {
    const Chunk& ch = p->chunks[c];
    pc0[ch.problem] = c;
    pnc[ch.problem]++;
  }
  for (Chunk& ch : p->chunks) {
    ch.pc0 = pc0[ch.problem];
    ch.pnc = pnc[ch.problem];
  }
  // sweep kinds: k and how much of the problem fits the LDS budget of the
  // staged sweeps (block table + row tables + x segment, then block values)
  const int xbytes = prec == SGDG_FP64 ? 8 : (prec == SGDG_FP32_SWEEP ? 4 : 2);
  const int vbytes = prec == SGDG_FP64 ? 8 : 4;
  p->chunk_lists.assign(SWEEP_TIERS * (SGDG_MAX_K + 1), {});
  p->list_lds.assign(SWEEP_TIERS * (SGDG_MAX_K + 1), 0);
  auto al16 = [](int64_t b) { return (b + 15) & ~(int64_t)15; };
  auto al256 = [](int64_t b) { return (b + 255) & ~(int64_t)255; };
  // rows of each direction's 1D operator that a chunk's outputs use: the
  // range of their target cells (the staged sweep copies only these)
  std::vector<StageRange> srange((size_t)p->nchunks * SGDG_MAX_D, StageRange{0, 0, 0, 0});
  for (int32_t c = 0; c < p->nchunks; ++c) {
    const Chunk& ch = p->chunks[c];
    const HostInstance& hi = p->inst[ch.inst];
    const int K1 = hi.desc.k + 1;
    int tlo[SGDG_MAX_D], thi[SGDG_MAX_D];
    for (int m = 0; m < d; ++m) {
      tlo[m] = INT32_MAX;
      thi[m] = -1;
    }
    for (int32_t b = ch.b0; b <= ch.b1; ++b) {
      const GBlock& gb = p->gblk[b];
      const int64_t e0 = std::max(ch.start, gb.start), e1 = std::min(ch.start + ch.count, gb.start + gb.size);
      for (int64_t g = e0; g < e1; ++g) {
        int64_t rem = g - gb.start;  // the sweep's decoding of a block-local index
        for (int m = d - 1; m >= 0; --m) {
          const int l = gb.lev[m];
          const int64_t ext = (int64_t)K1 << (l > 0 ? l - 1 : 0);
          const int64_t t = rem % ext;
          rem /= ext;
          const int tc = l == 0 ? 0 : (1 << (l - 1)) + (int)(t / K1);
          tlo[m] = std::min(tlo[m], tc);
          thi[m] = std::max(thi[m], tc);
        }
      }
    }
    // directions that share a 1D operator share one staged copy: the union
    // of their ranges (so a chunk never stages more than the whole tables)
    for (int m = 0; m < d; ++m) {
      int lo = tlo[m], hi_ = thi[m];
      for (int m2 = 0; m2 < d; ++m2)
        if (hi.dir_tab[m2] == hi.dir_tab[m]) {
          lo = std::min(lo, tlo[m2]);
          hi_ = std::max(hi_, thi[m2]);
        }
      const Op1D& op = p->ops[hi.dir_tab[m]];
      StageRange& r = srange[(size_t)c * SGDG_MAX_D + m];
      r.tlo = lo;
      r.nrow = hi_ - lo + 1;
      r.elo = op.cptr[lo];
      r.nent = op.cptr[hi_ + 1] - r.elo;
    }
  }
  for (int32_t c = 0; c < p->nchunks; ++c) {
    const HostInstance& hi = p->inst[p->chunks[c].inst];
    int64_t ntab = 1;
    for (int m = 0; m < d; ++m) ntab *= (hi.desc.n + 1);
    const int64_t kk = (int64_t)(hi.desc.k + 1) * (hi.desc.k + 1);
    // staged sweep: block table, then per direction the chunk's row pointers,
    // source cells (and block values), each region with 16 bytes of slack
    // rounded to 256 bytes for the direct global -> LDS copies.
    int64_t rows256 = 0, vals256 = 0;
    for (int m = 0; m < d; ++m) {
      bool seen = false;
      for (int m2 = 0; m2 < m; ++m2) seen = seen || hi.dir_tab[m2] == hi.dir_tab[m];
      if (seen) continue;
      const StageRange& r = srange[(size_t)c * SGDG_MAX_D + m];
      rows256 += al256(((int64_t)r.nrow + 1) * 4 + 16) + al256((int64_t)r.nent * 4 + 16);
      vals256 += al256((int64_t)r.nent * kk * vbytes + 16);
    }
    const int64_t lds1 = al256(ntab * 4) + rows256 + al256(hi.ndof * xbytes + 16);
    const int64_t lds2 = lds1 + vals256;
    const int tier = lds2 <= APPLY_LDS_BYTES_HOST ? 2 : (lds1 <= APPLY_LDS_BYTES_HOST ? 1 : 0);
    const int kind = hi.desc.k * SWEEP_TIERS + tier;
    p->chunk_lists[kind].push_back(c);
    if (tier > 0) p->list_lds[kind] = std::max(p->list_lds[kind], (int)(tier == 2 ? lds2 : lds1));
  }

  // Staged lists: workgroups go to the XCDs round-robin (workgroup t to XCD
  // t mod 8), and each XCD's L2 fetches what its workgroups stage.  Ordering
  // the list so that a problem's chunks land on their own subset of XCDs (a
  // share of the eight by problem count, or one XCD each when there are more
  // problems than XCDs) keeps every L2 to the segments and row tables of its
  // own problems.
  constexpr int NXCD = 8;
  for (size_t kind = 0; kind < p->chunk_lists.size(); ++kind) {
    std::vector<int32_t>& L = p->chunk_lists[kind];
    if (kind % SWEEP_TIERS == 0 || L.size() <= (size_t)NXCD) continue;
    std::vector<int32_t> probs;
    for (int32_t c : L)
      if (probs.empty() || probs.back() != p->chunks[c].problem) probs.push_back(p->chunks[c].problem);
    std::sort(probs.begin(), probs.end());
    probs.erase(std::unique(probs.begin(), probs.end()), probs.end());
    const int np = (int)probs.size();
    std::vector<std::vector<int32_t>> q(NXCD);
    std::vector<int> rr(np, 0);
    for (int32_t c : L) {
      const int pi = (int)(std::lower_bound(probs.begin(), probs.end(), p->chunks[c].problem) - probs.begin());
      int x;
      if (np <= NXCD) {
        const int x0 = pi * NXCD / np, x1 = (pi + 1) * NXCD / np;
        x = x0 + rr[pi]++ % std::max(1, x1 - x0);
      } else {
        x = pi % NXCD;
      }
      q[x].push_back(c);
    }
    std::vector<size_t> head(NXCD, 0);
    std::vector<int32_t> out;
    out.reserve(L.size());
    for (size_t t = 0; out.size() < L.size(); ++t) {
      int x = (int)(t % NXCD);
      if (head[x] == q[x].size()) {  // this XCD's queue is empty: take from the longest
        size_t best = 0;
        for (int y = 0; y < NXCD; ++y)
          if (q[y].size() - head[y] > best) {
            best = q[y].size() - head[y];
            x = y;
          }
      }
      out.push_back(q[x][head[x]++]);
    }
    L.swap(out);
  }

  sgdg_status st = SGDG_OK;
  std::vector<float> valf(val_all.begin(), val_all.end());
  if ((st = upload(p, p->gblk, &p->dev.gblk)) != SGDG_OK || (st = upload(p, srange, &p->dev.srange)) != SGDG_OK ||
      (st = upload(p, p->chunks, &p->dev.chunks)) != SGDG_OK ||
      (st = upload(p, p->instdev, &p->dev.inst)) != SGDG_OK || (st = upload(p, blkid, &p->dev.blkid)) != SGDG_OK ||
      (st = upload(p, lstart, &p->dev.lstart)) != SGDG_OK || (st = upload(p, bcsr, &p->dev.bcsr)) != SGDG_OK ||
      (st = upload(p, cptr_all, &p->dev.cptr)) != SGDG_OK || (st = upload(p, src_all, &p->dev.src)) != SGDG_OK ||
      (st = upload(p, val_all, &p->dev.val)) != SGDG_OK || (st = upload(p, valf, &p->dev.valf)) != SGDG_OK) {
    sg_dg_destroy(p);
    return st;
  }
  if ((st = upload(p, pc0, &p->dev.pchunk0)) != SGDG_OK || (st = upload(p, pnc, &p->dev.pnchunk)) != SGDG_OK) {
    sg_dg_destroy(p);
    return st;
  }
  p->pchunk0 = pc0;
  p->pnchunk = pnc;
  p->dev_chunk_lists.assign(p->chunk_lists.size(), nullptr);
  p->dev_tasks.assign(p->chunk_lists.size(), nullptr);
  for (size_t kind = 0; kind < p->chunk_lists.size(); ++kind) {
    if (p->chunk_lists[kind].empty()) continue;
    if ((st = upload(p, p->chunk_lists[kind], &p->dev_chunk_lists[kind])) != SGDG_OK) {
      sg_dg_destroy(p);
      return st;
    }
    if (kind % SWEEP_TIERS == 0) continue;
    std::vector<SweepTask> tasks(p->chunk_lists[kind].size());
    for (size_t e = 0; e < tasks.size(); ++e) {
      const int32_t c = p->chunk_lists[kind][e];
      const Chunk& ch = p->chunks[c];
      const HostInstance& hi = p->inst[ch.inst];
      const InstDev& id = p->instdev[ch.inst];
      const int64_t kk = (int64_t)(hi.desc.k + 1) * (hi.desc.k + 1);
      SweepTask& t = tasks[e];
      t = SweepTask{};
      t.start = ch.start;
      t.seg = hi.offset + (int64_t)ch.species * hi.ndof;
      t.ndof = hi.ndof;
      t.cid = c;
      t.count = ch.count;
      t.g = ch.g;
      t.inst = ch.inst;
      t.species = ch.species;
      t.b0 = ch.b0;
      t.b1 = ch.b1;
      t.ntab = 1;
      for (int m = 0; m < d; ++m) t.ntab *= (hi.desc.n + 1);
      t.blkid_off = id.blkid_off;
      for (int m = 0; m < d; ++m) {
        const BCsr& bc = bcsr[id.bcsr_off[m]];
        const StageRange& r = srange[(size_t)c * SGDG_MAX_D + m];
        t.cp[m] = bc.cptr_off + r.tlo;
        t.sp[m] = bc.src_off + r.elo;
        t.vp[m] = bc.val_off + (int64_t)r.elo * kk;
        t.nrow[m] = r.nrow;
        t.nent[m] = r.nent;
        t.tlo[m] = r.tlo;
        t.elo[m] = r.elo;
        for (int m2 = 0; m2 < m; ++m2)
          if (!((t.dup >> m) & 1u) && hi.dir_tab[m2] == hi.dir_tab[m]) t.dup |= 1u << m;
      }
    }
    if ((st = upload(p, tasks, &p->dev_tasks[kind])) != SGDG_OK) {
      sg_dg_destroy(p);
      return st;
    }
  }
  if ((st = reaction_build(p)) != SGDG_OK) {
    sg_dg_destroy(p);
    return st;
  }
  if (fibre_auto(p)) {
    if ((st = fibre_build(p, false)) != SGDG_OK) {
      sg_dg_destroy(p);
      return st;
    }
    p->fibre_on = true;
  }
  *out = p;
  return SGDG_OK;
}

extern "C" sgdg_status sg_dg_info(const sgdg_plan* plan, int32_t inst, int64_t* ndof, int64_t* offset,
                                  int64_t* npoints) {
  if (!plan) return fail(SGDG_ERR_ARG, "sg_dg_info: null plan");
  if (inst < 0 || inst >= plan->ninst) return fail(SGDG_ERR_ARG, "sg_dg_info: instance out of range");
  const HostInstance& hi = plan->inst[inst];
  if (ndof) *ndof = hi.ndof;
  if (offset) *offset = hi.offset;
  if (npoints) *npoints = hi.npoints;
  return SGDG_OK;
}

extern "C" sgdg_status sg_dg_total(const sgdg_plan* plan, int64_t* total) {
  if (!plan || !total) return fail(SGDG_ERR_ARG, "sg_dg_total: null argument");
  *total = plan->total;
  return SGDG_OK;
}

extern "C" sgdg_status sg_dg_workspace_size(const sgdg_plan* plan, int32_t M, int32_t nrhs, size_t* krylov_bytes,
                                            size_t* iif2_bytes) {
  if (!plan) return fail(SGDG_ERR_ARG, "sg_dg_workspace_size: null plan");
  if (M < 1 || M > SGDG_MAX_M) return fail(SGDG_ERR_ARG, "sg_dg_workspace_size: M must be in 1..48");
  if (nrhs < 1) return fail(SGDG_ERR_ARG, "sg_dg_workspace_size: nrhs must be positive");
  if (krylov_bytes) *krylov_bytes = krylov_ws_bytes(plan, M, nrhs);
  if (iif2_bytes) *iif2_bytes = iif2_ws_bytes(plan, M, nrhs);
  return SGDG_OK;
}

extern "C" sgdg_status sg_dg_layout(const sgdg_plan* plan, int32_t inst, int32_t* lev, int32_t* cell, int32_t* pp) {
  if (!plan || !lev || !cell || !pp) return fail(SGDG_ERR_ARG, "sg_dg_layout: null argument");
  if (inst < 0 || inst >= plan->ninst) return fail(SGDG_ERR_ARG, "sg_dg_layout: instance out of range");
  const HostInstance& hi = plan->inst[inst];
  const int d = plan->d, K1 = hi.desc.k + 1;
  int64_t a = 0;
  for (size_t b = 0; b < hi.blocks.size(); ++b) {
    const auto& l = hi.blocks[b];
    std::vector<int64_t> ext(d);
    for (int m = 0; m < d; ++m) ext[m] = (int64_t)level_count(l[m]) * K1;
    for (int64_t e = 0; e < hi.bsize[b]; ++e, ++a) {
      int64_t rem = e;
      for (int m = d - 1; m >= 0; --m) {
        int64_t t = rem % ext[m];
        rem /= ext[m];
        lev[a * d + m] = l[m];
        cell[a * d + m] = (int32_t)(t / K1);
        pp[a * d + m] = (int32_t)(t % K1);
      }
    }
  }
  return SGDG_OK;
}

extern "C" sgdg_status sg_dg_project(const sgdg_plan* plan, int32_t inst, double amp, const sgdg_factor1d* factors,
                                     double* out) {
  if (!plan || !factors || !out) return fail(SGDG_ERR_ARG, "sg_dg_project: null argument");
  if (inst < 0 || inst >= plan->ninst) return fail(SGDG_ERR_ARG, "sg_dg_project: instance out of range");
  const HostInstance& hi = plan->inst[inst];
  const int d = plan->d, N = hi.desc.n, k = hi.desc.k, K1 = k + 1;
  for (int m = 0; m < d; ++m)
    if (factors[m].kind != 0 && factors[m].kind != 1) return fail(SGDG_ERR_ARG, "sg_dg_project: unknown factor kind");
  const Basis1D& bs = basis1d(k);
  const long nc = 1L << N;
  const double h = std::ldexp(1.0, -N);
  std::vector<double> xg, wg;
  gauss01(16, xg, wg);
  std::vector<std::vector<double>> c1(d, std::vector<double>((size_t)K1 << N, 0.0));
  for (int m = 0; m < d; ++m) {
    const sgdg_factor1d& f = factors[m];
    for (long c = 0; c < nc; ++c)
      for (size_t g = 0; g < xg.size(); ++g) {
        double x = (c + xg[g]) * h;
        double gv = f.kind == 0 ? std::cos(2.0 * M_PI * f.a * x + f.b) : ((x >= f.a && x < f.b) ? 1.0 : 0.0);
        if (gv == 0.0) continue;
        double wv = wg[g] * h * gv;
        for (int l = 0; l <= N; ++l) {
          long j = l == 0 ? 0 : (c >> (N - l + 1));
          long cellidx = l == 0 ? 0 : ((1L << (l - 1)) + j);
          for (int p = 0; p < K1; ++p) c1[m][cellidx * K1 + p] += wv * hier_value(bs, l, (int)j, p, x, false);
        }
      }
  }
  int64_t a = 0;
  for (size_t b = 0; b < hi.blocks.size(); ++b) {
    const auto& l = hi.blocks[b];
    std::vector<int64_t> ext(d);
    for (int m = 0; m < d; ++m) ext[m] = (int64_t)level_count(l[m]) * K1;
    for (int64_t e = 0; e < hi.bsize[b]; ++e, ++a) {
      int64_t rem = e;
      double v = amp;
      for (int m = d - 1; m >= 0; --m) {
        int64_t t = rem % ext[m];
        rem /= ext[m];
        long cellidx = l[m] == 0 ? 0 : ((1L << (l[m] - 1)) + t / K1);
        v *= c1[m][cellidx * K1 + t % K1];
      }
      out[a] = v;
    }
  }
  return SGDG_OK;
}

extern "C" sgdg_status sg_dg_norm_inf(const sgdg_plan* plan, int32_t inst, int32_t species, double* out) {
  if (!plan || !out) return fail(SGDG_ERR_ARG, "sg_dg_norm_inf: null argument");
  if (inst < 0 || inst >= plan->ninst) return fail(SGDG_ERR_ARG, "sg_dg_norm_inf: instance out of range");
  if (species < 0 || species >= plan->inst[inst].desc.nspecies)
    return fail(SGDG_ERR_ARG, "sg_dg_norm_inf: species out of range");
  *out = plan->inst[inst].anorm[species];
  return SGDG_OK;
}
