// Operator sweep y = A x in fibre form (Sec. 2.1, eq. 2.10; the product
// structure of Sec. 4: A is a sum over directions i of the 1D operator B_i
// acting along axis i and the identity on the others).
//
// Along direction i the sparse grid splits into fibres: the DOFs that share
// the levels l_m and positions of every other axis m != i.  A fibre holds all
// levels l_i = 0..b of axis i, b = N - sum_{m != i} l_m, i.e. the complete
// hierarchical space of level b, and the direction-i term of A restricted to
// it is B_i restricted to levels 0..b.  On that space the hierarchical basis
// is an orthonormal change of basis of the level-b cell-Legendre basis, in
// which the restricted operator is block tridiagonal (build_ss_levels).  So
// per fibre: synthesis (hierarchical -> level-b single scale, the multiwavelet
// two-scale relation level by level), one block-tridiagonal product, analysis
// back to hierarchical coefficients, and the result scaled by -D_s is added
// to y.  O(length) work per fibre instead of walking every row of B_i, and x
// is read once per direction.
//
// One launch per direction (the first writes y, the others add to it) and
// polynomial degree.  A workgroup takes a tile staged in LDS (at most FB_CAP
// values) and transforms it in place: F whole fibres, or, for a fibre too
// long for one tile, F of its subtrees.  A long fibre of budget b is split at
// level s0: a first launch synthesises its levels 0..s0 into single-scale
// values on the 2^s0 level-s0 cells (scratch); each subtree below one such
// cell then runs as a tile of its own (its root value from scratch, levels
// s0+1..b from x; the two level-b cells just outside the tile, needed by the
// tridiagonal product, are synthesised along the neighbouring subtrees'
// edges), writing its levels s0+1..b to y and its root's image to scratch;
// a last launch analyses the level-s0 images back to levels 0..s0.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cstring>
#include <unordered_map>
#include <vector>

#include "internal.h"

namespace sgdg {

namespace {

constexpr int FB_NT = 256;     // threads per workgroup
constexpr int FB_CAP = 2048;   // values of one LDS tile (and as many old y values): 4 workgroups per CU
constexpr int FB_FMAX = 512;   // fibres per tile
constexpr int FB_LDS = 2 * FB_CAP * 8 + FB_FMAX * 8 + 32 * 8 + 8 * 8;
constexpr int XRUN = 32;       // consecutive tasks per XCD
constexpr int64_t FIBRE_AUTO_MIN = int64_t(1) << 19;  // DOFs

enum TileMode : int32_t { WHOLE = 0, SUBTREE = 1, COARSE_SYN = 2, COARSE_ANA = 3 };

struct FibreTask {
  int64_t base;   // level-base table entries base .. base + bfull: plan-vector offset of block (l_i = 0..bfull)
  int64_t sS;     // split fibre: scratch offset of its level-s0 single-scale values (2^s0 cells x K1)
  int64_t sT;     // ... and of their images under the tridiagonal product
  int64_t opoff;  // level bfull of the direction's single-scale operator in the level table
  double negD;    // -D_s
  int32_t mode;   // TileMode
  int32_t b;      // levels held by the tile, 0..b (whole fibre: its budget; subtree: bfull - s0; coarse: s0)
  int32_t bfull;  // fibre budget
  int32_t s0;     // subtree tiles: level of the subtree roots
  int32_t F;      // tile capacity (a power of two) ...
  int32_t nv;     // ... and its valid fibres / subtrees
  int32_t q0;     // first fibre (q = pre S + suf over the other axes' positions); the fibre of a split
  int32_t J0;     // subtree tiles: first subtree (level-s0 cell)
  int32_t S;      // product of the extents after the axis (stride of the axis)
  int32_t ucell;  // 1: operator blocks per cell, 0: one block triple per level (translation invariant)
};

struct TwoScale {
  double ML[16], MR[16], cL[16], cR[16];  // [q][i]: child q from parent i; [p][q]: wavelet p on child q
};

struct Launch {  // one kernel launch: the tasks of one phase of one (direction, degree) group
  std::vector<FibreTask> tasks;
  FibreTask* dtasks = nullptr;
  int uc = 0;  // operator blocks: 0 one triple per level for every task, 1 per cell for every task, 2 mixed
};

struct Group {  // direction dir, degree K1 - 1: coarse synthesis, tiles, coarse analysis
  int dir = 0, K1 = 2;
  Launch ph[3];
};

}  // namespace

struct FibreData {
  bool test_split = false;  // split every fibre of budget >= 2 (a test form)
  std::vector<void*> allocs;
  std::vector<Group> groups;
  int64_t* bases = nullptr;
  double* ops = nullptr;
  double* scratch = nullptr;
  TwoScale ts[SGDG_MAX_K + 2];  // host copy, by K1
  TwoScale* dts = nullptr;      // device copy
};

namespace {

typedef __attribute__((address_space(3))) void* lds_ptr;

__device__ __forceinline__ int cell_level(int c) { return c == 0 ? 0 : 32 - __clz(c); }

// Address of the value at level l, position t along the axis of the fibre
// (pre, suf): lb[l] + (pre ext_l + t) S + suf.
template <int K1>
__device__ __forceinline__ int64_t lvl_addr(const int64_t* lb, int l, int t, int pre, int suf, int S) {
  const int ext = K1 * (l == 0 ? 1 : (1 << (l - 1)));
  return lb[l] + ((int64_t)pre * ext + t) * S + suf;
}
// Element (cell c of a whole fibre in hierarchical order, component p).
template <int K1>
__device__ __forceinline__ int64_t elem_addr(const int64_t* lb, int c, int p, int pre, int suf, int S) {
  const int l = cell_level(c);
  const int c0 = l == 0 ? 0 : (1 << (l - 1));
  return lvl_addr<K1>(lb, l, (c - c0) * K1 + p, pre, suf, S);
}
// Element (cell c >= 1 of subtree J in its own hierarchical order, component
// p): level s0 + l' of the fibre, position J 2^(l'-1) + j'.
template <int K1>
__device__ __forceinline__ int64_t sub_addr(const int64_t* lb, int s0, int J, int c, int p, int pre, int suf, int S) {
  const int l = cell_level(c);
  const int h = 1 << (l - 1);
  return lvl_addr<K1>(lb, s0 + l, ((J * h) + (c - h)) * K1 + p, pre, suf, S);
}

// The level-b cell of subtree J at its left (side 0) or right (side 1) end:
// synthesis along that edge from the root value (scratch) and one wavelet per
// level.
template <int K1>
__device__ void edge_cell(const FibreTask& tk, const TwoScale& __restrict__ ts, const double* __restrict__ x,
                          const double* __restrict__ scratch, const int64_t* lb, int J, int side, int pre, int suf,
                          double* out) {
  double v[K1];
#pragma unroll
  for (int i = 0; i < K1; ++i) v[i] = scratch[tk.sS + (int64_t)J * K1 + i];
  for (int l = 1; l <= tk.b; ++l) {
    const int h = 1 << (l - 1);
    const int c = h + (side ? h - 1 : 0);  // leftmost / rightmost wavelet cell of level l in the subtree
    double w[K1], nv[K1];
#pragma unroll
    for (int p = 0; p < K1; ++p) w[p] = x[sub_addr<K1>(lb, tk.s0, J, c, p, pre, suf, tk.S)];
#pragma unroll
    for (int q = 0; q < K1; ++q) {
      double a = 0;
#pragma unroll
      for (int i = 0; i < K1; ++i)
        a += side ? ts.MR[q * K1 + i] * v[i] + ts.cR[i * K1 + q] * w[i] : ts.ML[q * K1 + i] * v[i] + ts.cL[i * K1 + q] * w[i];
      nv[q] = a;
    }
#pragma unroll
    for (int q = 0; q < K1; ++q) v[q] = nv[q];
  }
#pragma unroll
  for (int q = 0; q < K1; ++q) out[q] = v[q];
}

// One tile.  LDS layout [f][cell][p] for subtrees and for fibres along the
// last axis (S = 1: a fibre's values are contiguous in each block), else
// [cell][p][f] (consecutive fibres are consecutive in memory).
template <int K1, int UC>
__device__ void tile_body(const FibreTask& tk, const TwoScale& __restrict__ ts, const double* __restrict__ ops,
                          const double* __restrict__ x, double* __restrict__ y, double* __restrict__ scratch, int acc,
                          double* buf, double* ybuf, const int* fpre, const int* fsuf, const int64_t* lb,
                          double* halo) {
  constexpr int K2 = K1 * K1;
  constexpr int RS = (FB_CAP / (2 * K1) + FB_NT - 1) / FB_NT;  // parents per thread (one-level step)
  constexpr int RS2 = (FB_CAP / (4 * K1) + FB_NT - 1) / FB_NT; // grandparents per thread (two-level step)
  constexpr int RT = (FB_CAP / K1 + FB_NT - 1) / FB_NT;        // cells per thread (tridiagonal)
  const int tid = threadIdx.x;
  const int mode = tk.mode, b = tk.b, F = tk.F, S = tk.S;
  const int lF = 31 - __clz(F);
  const int C = 1 << b, L = K1 << b;
  const bool last = (S == 1) || mode == SUBTREE;
  const int fs = last ? L : 1, cs = last ? K1 : K1 * F, ps = last ? 1 : F;
  auto idx = [&](int f, int c, int p) { return f * fs + c * cs + p * ps; };
  const int nval = F * L;

  // Where value it of the tile comes from and where it goes: LDS slot it in
  // either layout (value order = layout order).  Source: x (hierarchical
  // coefficients), a subtree's root value or the coarse images (scratch);
  // destination: y, or scratch (coarse values, a subtree root's image).
  auto src_of = [&](int it, const double*& xs_, int64_t& yad) {
    xs_ = nullptr;
    yad = -1;
    if (it >= nval) return;
    int f, c, p, w;
    if (last) {
      f = (it >> b) / K1;
      w = it - f * L;
    } else {
      f = it & (F - 1);
      w = it >> lF;
    }
    c = w / K1;
    p = w - c * K1;
    if (f >= tk.nv) return;
    if (mode == SUBTREE) {
      if (c == 0) {
        xs_ = scratch + tk.sS + (int64_t)(tk.J0 + f) * K1 + p;
      } else {
        yad = sub_addr<K1>(lb, tk.s0, tk.J0 + f, c, p, fpre[f], fsuf[f], S);
        xs_ = x + yad;
      }
    } else {
      const int64_t a = elem_addr<K1>(lb, c, p, fpre[f], fsuf[f], S);
      xs_ = mode == COARSE_ANA ? scratch + tk.sT + it : x + a;
      if (mode != COARSE_SYN) yad = a;
    }
  };

  // load: direct global -> LDS copies, two lanes per value (its two 32-bit
  // halves), 32 values per wave instruction; the old y values of the tile
  // (when adding) land in ybuf at the same time
  {
    const int lane = tid & 63, half = lane & 1;
    for (int ch = tid >> 6; ch * 32 < nval; ch += FB_NT / 64) {
      const double* xs_;
      int64_t yad;
      src_of(ch * 32 + (lane >> 1), xs_, yad);
      if (xs_)
        __builtin_amdgcn_global_load_lds((const void*)((const uint32_t*)xs_ + half), (lds_ptr)(buf + ch * 32), 4, 0,
                                         0);
      if (acc && yad >= 0)
        __builtin_amdgcn_global_load_lds((const void*)((const uint32_t*)(y + yad) + half), (lds_ptr)(ybuf + ch * 32),
                                         4, 0, 0);
    }
  }
  if (mode == SUBTREE && tid < 2) {
    const int m = (1 << tk.s0) - 1;
    const int J = tid == 0 ? ((tk.J0 - 1) & m) : ((tk.J0 + tk.nv) & m);
    edge_cell<K1>(tk, ts, x, scratch, lb, J, 1 - tid, fpre[0], fsuf[0], halo + tid * K1);
  }
  __builtin_amdgcn_s_waitcnt(0);  // this thread's direct loads have landed
  __syncthreads();

  // two-scale relation: children (left, right) of a cell from its
  // coefficients and its wavelet's; parent and wavelet from the children
  auto children = [&](const double* sv, const double* w, double* lo, double* hi) {
#pragma unroll
    for (int q = 0; q < K1; ++q) {
      double a = 0, c = 0;
#pragma unroll
      for (int i = 0; i < K1; ++i) {
        a += ts.ML[q * K1 + i] * sv[i] + ts.cL[i * K1 + q] * w[i];
        c += ts.MR[q * K1 + i] * sv[i] + ts.cR[i * K1 + q] * w[i];
      }
      lo[q] = a;
      hi[q] = c;
    }
  };
  auto parent = [&](const double* vl, const double* vr, double* pa, double* wa) {
#pragma unroll
    for (int i = 0; i < K1; ++i) {
      double a = 0, c = 0;
#pragma unroll
      for (int q = 0; q < K1; ++q) {
        a += ts.ML[q * K1 + i] * vl[q] + ts.MR[q * K1 + i] * vr[q];
        c += ts.cL[i * K1 + q] * vl[q] + ts.cR[i * K1 + q] * vr[q];
      }
      pa[i] = a;
      wa[i] = c;
    }
  };
  // item it of a step with 2^ln cells per fibre on its coarse level
  auto item = [&](int it, int ln, int& f, int& j) {
    f = last ? (it >> ln) : (it & (F - 1));
    j = last ? (it & ((1 << ln) - 1)) : (it >> lF);
  };

  // synthesis, coarse to fine: one level (cells 2j, 2j+1 of level lo+1 from
  // cell j of level lo and wavelet n + j, n = 2^lo) when b is odd, then two
  // levels per pair of barriers (cells 4j..4j+3 of level lo+2 from cell j,
  // wavelet n + j of level lo+1 and wavelets 2n + 2j, 2n + 2j + 1 of level lo+2)
  if (mode != COARSE_ANA && b > 0) {
    int lo = 0;
    if (b & 1) {
      double st[RS][2 * K1];
#pragma unroll
      for (int r = 0; r < RS; ++r) {
        const int it = tid + r * FB_NT;
        if (it < F) {
          int f, j;
          item(it, 0, f, j);
          double sv[K1], w[K1];
#pragma unroll
          for (int i = 0; i < K1; ++i) {
            sv[i] = buf[idx(f, j, i)];
            w[i] = buf[idx(f, 1 + j, i)];
          }
          children(sv, w, st[r], st[r] + K1);
        }
      }
      __syncthreads();
#pragma unroll
      for (int r = 0; r < RS; ++r) {
        const int it = tid + r * FB_NT;
        if (it < F) {
          int f, j;
          item(it, 0, f, j);
#pragma unroll
          for (int q = 0; q < K1; ++q) {
            buf[idx(f, 2 * j, q)] = st[r][q];
            buf[idx(f, 2 * j + 1, q)] = st[r][K1 + q];
          }
        }
      }
      __syncthreads();
      lo = 1;
    }
    for (; lo + 2 <= b; lo += 2) {
      const int n = 1 << lo, items = F << lo;
      double st[RS2][4 * K1];
#pragma unroll
      for (int r = 0; r < RS2; ++r) {
        const int it = tid + r * FB_NT;
        if (it < items) {
          int f, j;
          item(it, lo, f, j);
          double sv[K1], w1[K1], wa[K1], wb[K1], m0[K1], m1[K1];
#pragma unroll
          for (int i = 0; i < K1; ++i) {
            sv[i] = buf[idx(f, j, i)];
            w1[i] = buf[idx(f, n + j, i)];
            wa[i] = buf[idx(f, 2 * n + 2 * j, i)];
            wb[i] = buf[idx(f, 2 * n + 2 * j + 1, i)];
          }
          children(sv, w1, m0, m1);
          children(m0, wa, st[r], st[r] + K1);
          children(m1, wb, st[r] + 2 * K1, st[r] + 3 * K1);
        }
        asm volatile("" ::: "memory");  // bounds the LDS reads kept in flight
      }
      __syncthreads();
#pragma unroll
      for (int r = 0; r < RS2; ++r) {
        const int it = tid + r * FB_NT;
        if (it < items) {
          int f, j;
          item(it, lo, f, j);
#pragma unroll
          for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int q = 0; q < K1; ++q) buf[idx(f, 4 * j + u, q)] = st[r][u * K1 + q];
        }
      }
      __syncthreads();
    }
  }

  // block-tridiagonal product on level bfull, scaled by -D_s: within each
  // whole fibre (cell indices mod 2^b), or across the tile's consecutive
  // subtrees with the edge cells outside it
  if (mode == WHOLE || mode == SUBTREE) {
    const int items = F << b;
    const int ulast = tk.nv * C - 1;  // subtree tiles: the last valid cell of the run
    double st[RT][K1];
    auto tri = [&](int r, const double* __restrict__ B0, int cstride) {
      const int it = tid + r * FB_NT;
      const int f = last ? (it >> b) : (it & (F - 1));
      const int c = last ? (it & (C - 1)) : (it >> lF);
      double sm[K1], s0[K1], sp[K1];
      int64_t creal;
      if (mode == SUBTREE) {
        const int u = f * C + c;
        creal = (int64_t)tk.J0 * C + u;
#pragma unroll
        for (int i = 0; i < K1; ++i) {
          sm[i] = u == 0 ? halo[i] : buf[(u - 1) * K1 + i];
          s0[i] = buf[u * K1 + i];
          sp[i] = u >= ulast ? halo[K1 + i] : buf[(u + 1) * K1 + i];
        }
      } else {
        const int cm = (c - 1) & (C - 1), cp = (c + 1) & (C - 1);
        creal = c;
#pragma unroll
        for (int i = 0; i < K1; ++i) {
          sm[i] = buf[idx(f, cm, i)];
          s0[i] = buf[idx(f, c, i)];
          sp[i] = buf[idx(f, cp, i)];
        }
      }
      const double* __restrict__ B = B0 + creal * cstride;
#pragma unroll
      for (int q = 0; q < K1; ++q) {
        double a = 0;
#pragma unroll
        for (int i = 0; i < K1; ++i)
          a += B[q * K1 + i] * sm[i] + B[K2 + q * K1 + i] * s0[i] + B[2 * K2 + q * K1 + i] * sp[i];
        st[r][q] = a * tk.negD;
      }
    };
    if (UC == 0 || (UC == 2 && !tk.ucell)) {
      // one block triple for every cell (a uniform address)
      const double* Bu = ops + tk.opoff;
#pragma unroll
      for (int r = 0; r < RT; ++r) {
        if (tid + r * FB_NT < items) tri(r, Bu, 0);
        asm volatile("" ::: "memory");
      }
    } else {
#pragma unroll
      for (int r = 0; r < RT; ++r) {
        if (tid + r * FB_NT < items) tri(r, ops + tk.opoff, 3 * K2);
        asm volatile("" ::: "memory");  // one cell's blocks in registers at a time
      }
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < RT; ++r) {
      const int it = tid + r * FB_NT;
      if (it < items) {
        const int f = last ? (it >> b) : (it & (F - 1));
        const int c = last ? (it & (C - 1)) : (it >> lF);
#pragma unroll
        for (int q = 0; q < K1; ++q) buf[idx(f, c, q)] = st[r][q];
      }
    }
    __syncthreads();
  }

  // analysis, fine to coarse: two levels per pair of barriers (cell j of
  // level lo, wavelet n + j of level lo+1 and wavelets 2n + 2j, 2n + 2j + 1 of
  // level lo+2 from cells 4j..4j+3 of level lo+2), then one level when b is odd
  if (mode != COARSE_SYN && b > 0) {
    int hi = b;
    for (; hi >= 2; hi -= 2) {
      const int lo = hi - 2, n = 1 << lo, items = F << lo;
      double st[RS2][4 * K1];
#pragma unroll
      for (int r = 0; r < RS2; ++r) {
        const int it = tid + r * FB_NT;
        if (it < items) {
          int f, j;
          item(it, lo, f, j);
          double v[4][K1], m0[K1], m1[K1];
#pragma unroll
          for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int q = 0; q < K1; ++q) v[u][q] = buf[idx(f, 4 * j + u, q)];
          parent(v[0], v[1], m0, st[r] + 2 * K1);
          parent(v[2], v[3], m1, st[r] + 3 * K1);
          parent(m0, m1, st[r], st[r] + K1);
        }
        asm volatile("" ::: "memory");
      }
      __syncthreads();
#pragma unroll
      for (int r = 0; r < RS2; ++r) {
        const int it = tid + r * FB_NT;
        if (it < items) {
          int f, j;
          item(it, lo, f, j);
#pragma unroll
          for (int i = 0; i < K1; ++i) {
            buf[idx(f, j, i)] = st[r][i];
            buf[idx(f, n + j, i)] = st[r][K1 + i];
            buf[idx(f, 2 * n + 2 * j, i)] = st[r][2 * K1 + i];
            buf[idx(f, 2 * n + 2 * j + 1, i)] = st[r][3 * K1 + i];
          }
        }
      }
      __syncthreads();
    }
    if (hi == 1) {
      double st[RS][2 * K1];
#pragma unroll
      for (int r = 0; r < RS; ++r) {
        const int it = tid + r * FB_NT;
        if (it < F) {
          int f, j;
          item(it, 0, f, j);
          double vl[K1], vr[K1];
#pragma unroll
          for (int q = 0; q < K1; ++q) {
            vl[q] = buf[idx(f, 2 * j, q)];
            vr[q] = buf[idx(f, 2 * j + 1, q)];
          }
          parent(vl, vr, st[r], st[r] + K1);
        }
      }
      __syncthreads();
#pragma unroll
      for (int r = 0; r < RS; ++r) {
        const int it = tid + r * FB_NT;
        if (it < F) {
          int f, j;
          item(it, 0, f, j);
#pragma unroll
          for (int i = 0; i < K1; ++i) {
            buf[idx(f, j, i)] = st[r][i];
            buf[idx(f, 1 + j, i)] = st[r][K1 + i];
          }
        }
      }
      __syncthreads();
    }
  }

  // store: y (plus its old value after the first direction), or the coarse
  // values / a subtree root's image to scratch
  for (int it = tid; it < nval; it += FB_NT) {
    const double* xs_;
    int64_t yad;
    src_of(it, xs_, yad);
    if (!xs_) continue;
    const double v = buf[it];
    if (yad >= 0)
      y[yad] = acc ? v + ybuf[it] : v;
    else if (mode == COARSE_SYN)
      scratch[tk.sS + it] = v;
    else  // a subtree's root
      scratch[tk.sT + (xs_ - (scratch + tk.sS))] = v;
  }
}

template <int K1, int UC>
__global__ __launch_bounds__(FB_NT) __attribute__((amdgpu_waves_per_eu(4))) void k_fibre(
    const FibreTask* __restrict__ tasks, const int64_t* __restrict__ bases, const double* __restrict__ ops,
    double* __restrict__ scratch, const double* __restrict__ x, double* __restrict__ y, int64_t xs, int64_t ys,
    int nrhs, int acc, const TwoScale* __restrict__ tsp) {
  extern __shared__ __align__(16) unsigned char smem[];
  const TwoScale& ts = *tsp;
  double* buf = (double*)smem;
  double* ybuf = buf + FB_CAP;
  int* fpre = (int*)(ybuf + FB_CAP);
  int* fsuf = fpre + FB_FMAX;
  int64_t* lb = (int64_t*)(fsuf + FB_FMAX);
  double* halo = (double*)(lb + 32);
  // workgroups go to the 8 XCDs round robin; the k-th workgroup of XCD x
  // takes task ((k / XRUN) 8 + x) XRUN + k % XRUN, so that runs of XRUN
  // consecutive tasks (tiles of neighbouring fibres, whose values share cache
  // lines) meet in one XCD's L2 (the list is padded to a multiple of 8 XRUN)
  const int k8 = blockIdx.x >> 3;
  const FibreTask tk = tasks[((k8 / XRUN) * 8 + (blockIdx.x & 7)) * XRUN + k8 % XRUN];
  const int tid = threadIdx.x;
  if (tid <= tk.bfull) lb[tid] = bases[tk.base + tid];
  for (int f = tid; f < tk.F; f += FB_NT) {
    const int q = tk.mode == SUBTREE ? tk.q0 : tk.q0 + f;
    fpre[f] = q / tk.S;
    fsuf[f] = q - fpre[f] * tk.S;
  }
  __syncthreads();
  for (int r = 0; r < nrhs; ++r) {
    tile_body<K1, UC>(tk, ts, ops, x + r * xs, y + r * ys, scratch, acc, buf, ybuf, fpre, fsuf, lb, halo);
    __syncthreads();
  }
}

inline int cells_at(int l) { return l == 0 ? 1 : (1 << (l - 1)); }

}  // namespace

// The automatic choice: FP64 plans whose every species segment is too large
// for the staged sweeps (all chunks take the global gather) and that are
// large enough for the fibre launches to pay off.
bool fibre_auto(const sgdg_plan* p) {
  if (p->prec != SGDG_FP64 || p->total < FIBRE_AUTO_MIN) return false;
  for (size_t kind = 0; kind < p->chunk_lists.size(); ++kind)
    if (kind % SWEEP_TIERS != 0 && !p->chunk_lists[kind].empty()) return false;
  return true;
}

void fibre_destroy(sgdg_plan* p) {
  if (!p->fdata) return;
  for (void* a : p->fdata->allocs) (void)hipFree(a);
  delete p->fdata;
  p->fdata = nullptr;
}

namespace {

sgdg_status fibre_upload(FibreData* fd, const void* src, size_t bytes, void** out) {
  void* d = nullptr;
  hipError_t e = hipMalloc(&d, std::max<size_t>(bytes, 1));
  if (e != hipSuccess) return hip_fail(e, "hipMalloc(fibre table)");
  fd->allocs.push_back(d);
  if (bytes) {
    e = hipMemcpy(d, src, bytes, hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpy(fibre table)");
  }
  *out = d;
  return SGDG_OK;
}

}  // namespace

// Host tables of the fibre form: the single-scale level operators of every
// 1D operator of the plan, the level-base table and the task lists.
sgdg_status fibre_build(sgdg_plan* p, bool test_split) {
  if (p->fdata && p->fdata->test_split == test_split) return SGDG_OK;
  fibre_destroy(p);
  auto* fd = new FibreData();
  fd->test_split = test_split;
  const int d = p->d;
  // single-scale operator levels per 1D operator
  std::vector<double> optab;
  std::vector<std::vector<int64_t>> opoff(p->ops.size());
  std::vector<int> opuni(p->ops.size(), 0);
  for (size_t o = 0; o < p->ops.size(); ++o) {
    bool uni = false;
    std::vector<int64_t> off;
    std::vector<double> T = build_ss_levels(p->ops[o], off, uni);
    for (auto& v : off) v += (int64_t)optab.size();
    opoff[o] = off;
    opuni[o] = uni ? 1 : 0;
    optab.insert(optab.end(), T.begin(), T.end());
  }
  for (int k = 1; k <= SGDG_MAX_K; ++k) {
    const Basis1D& bs = basis1d(k);
    TwoScale& t = fd->ts[k + 1];
    std::memset(&t, 0, sizeof(t));
    std::copy(bs.ML.begin(), bs.ML.end(), t.ML);
    std::copy(bs.MR.begin(), bs.MR.end(), t.MR);
    std::copy(bs.cL.begin(), bs.cL.end(), t.cL);
    std::copy(bs.cR.begin(), bs.cR.end(), t.cR);
  }
  std::vector<int64_t> bases;
  int64_t scratch_max = 0;
  for (int dir = 0; dir < d; ++dir)
    for (int K1 = 2; K1 <= SGDG_MAX_K + 1; ++K1) {
      Group g;
      g.dir = dir;
      g.K1 = K1;
      std::vector<FibreTask> syn, sub, whole, ana;
      int64_t scr = 0;
      int bmax = 0;  // subtree depth that fills a tile: K1 2^bmax <= FB_CAP
      while ((K1 << (bmax + 1)) <= FB_CAP) ++bmax;
      for (int ii = 0; ii < p->ninst; ++ii) {
        const HostInstance& hi = p->inst[ii];
        if (hi.desc.k + 1 != K1) continue;
        const int N = hi.desc.n;
        const int o = hi.dir_tab[dir];
        std::unordered_map<int64_t, int> blk;
        auto key = [&](const std::vector<int>& lv) {
          int64_t kk = 0;
          for (int m = 0; m < d; ++m) kk = kk * (N + 1) + lv[m];
          return kk;
        };
        for (size_t bi = 0; bi < hi.blocks.size(); ++bi) blk[key(hi.blocks[bi])] = (int)bi;
        for (size_t bi = 0; bi < hi.blocks.size(); ++bi) {
          std::vector<int> lv = hi.blocks[bi];
          if (lv[dir] != 0) continue;
          int lsum = 0;
          for (int m = 0; m < d; ++m) lsum += lv[m];
          const int b = N - lsum;
          int64_t P = 1, S = 1;
          for (int m = 0; m < d; ++m) {
            if (m == dir) continue;
            const int64_t e = (int64_t)K1 * cells_at(lv[m]);
            if (m < dir)
              P *= e;
            else
              S *= e;
          }
          const int64_t nf = P * S;
          // split level: fibres longer than a tile (or, in the test form, every
          // fibre of budget >= 2) are cut below level s0
          int s0 = -1;
          if (fd->test_split && b >= 2)
            s0 = b / 2;
          else if (b > bmax)
            s0 = b - bmax;
          if (s0 > bmax) {
            delete fd;
            return fail(SGDG_ERR_UNSUPPORTED, "fibre form: fibre too long for a two-level split");
          }
          for (int s = 0; s < hi.desc.nspecies; ++s) {
            const int64_t seg = hi.offset + (int64_t)s * hi.ndof;
            const int64_t base = (int64_t)bases.size();
            for (int li = 0; li <= b; ++li) {
              lv[dir] = li;
              const int bi2 = blk.at(key(lv));
              // every address (pre ext + t) S + suf of the fibre set stays inside its block
              if ((int64_t)hi.bsize[bi2] != P * K1 * cells_at(li) * S) {
                delete fd;
                return fail(SGDG_ERR_UNSUPPORTED, "fibre tables: block extents do not match the level tuple");
              }
              bases.push_back(seg + hi.bstart[bi2]);
            }
            lv[dir] = 0;
            FibreTask t{};
            t.base = base;
            t.opoff = opoff[o][b];
            t.ucell = opuni[o] ? 0 : 1;
            t.negD = -hi.desc.D[s];
            t.bfull = b;
            t.S = (int32_t)S;
            t.sS = t.sT = -1;
            if (s0 < 0) {
              const int64_t L = (int64_t)K1 << b;
              int F = 1;
              while (2 * F <= FB_FMAX && 2 * F * L <= FB_CAP && F < nf) F *= 2;
              t.mode = WHOLE;
              t.b = b;
              t.F = F;
              for (int64_t q0 = 0; q0 < nf; q0 += F) {
                t.q0 = (int32_t)q0;
                t.nv = (int32_t)std::min<int64_t>(F, nf - q0);
                whole.push_back(t);
              }
              continue;
            }
            const int bs = b - s0;                 // subtree depth
            const int64_t nsub = int64_t(1) << s0;  // subtrees per fibre
            int F = 1;
            while (2 * F <= FB_FMAX && (2 * F * K1 << bs) <= FB_CAP && 2 * F <= nsub) F *= 2;
            for (int64_t q = 0; q < nf; ++q) {
              FibreTask u = t;
              u.q0 = (int32_t)q;
              u.s0 = s0;
              u.sS = scr;
              u.sT = scr + (K1 << s0);
              scr += 2 * (K1 << s0);
              u.mode = COARSE_SYN;
              u.b = s0;
              u.F = u.nv = 1;
              syn.push_back(u);
              u.mode = COARSE_ANA;
              ana.push_back(u);
              u.mode = SUBTREE;
              u.b = bs;
              u.F = F;
              for (int64_t J0 = 0; J0 < nsub; J0 += F) {
                u.J0 = (int32_t)J0;
                u.nv = (int32_t)std::min<int64_t>(F, nsub - J0);
                sub.push_back(u);
              }
            }
          }
        }
      }
      if (whole.empty() && sub.empty()) continue;
      g.ph[0].tasks = syn;
      g.ph[1].tasks = sub;
      g.ph[1].tasks.insert(g.ph[1].tasks.end(), whole.begin(), whole.end());
      g.ph[2].tasks = ana;
      for (Launch& l : g.ph)
        if (!l.tasks.empty()) {
          bool any0 = false, any1 = false;
          for (const FibreTask& t : l.tasks) (t.ucell ? any1 : any0) = true;
          l.uc = any0 && any1 ? 2 : (any1 ? 1 : 0);
          FibreTask pad{};  // no valid fibre: loads and stores nothing
          pad.mode = WHOLE;
          pad.F = 1;
          pad.S = 1;
          pad.sS = pad.sT = -1;
          while (l.tasks.size() % (8 * XRUN)) l.tasks.push_back(pad);
        }
      scratch_max = std::max(scratch_max, scr);
      fd->groups.push_back(std::move(g));
    }
  p->fdata = fd;
  sgdg_status st;
  if ((st = fibre_upload(fd, bases.data(), bases.size() * sizeof(int64_t), (void**)&fd->bases)) != SGDG_OK) return st;
  if ((st = fibre_upload(fd, optab.data(), optab.size() * sizeof(double), (void**)&fd->ops)) != SGDG_OK) return st;
  if ((st = fibre_upload(fd, fd->ts, sizeof(fd->ts), (void**)&fd->dts)) != SGDG_OK) return st;
  for (Group& g : fd->groups)
    for (Launch& l : g.ph)
      if (!l.tasks.empty() &&
          (st = fibre_upload(fd, l.tasks.data(), l.tasks.size() * sizeof(FibreTask), (void**)&l.dtasks)) != SGDG_OK)
        return st;
  if (scratch_max > 0) {
    void* sp = nullptr;
    hipError_t e = hipMalloc(&sp, (size_t)scratch_max * sizeof(double));
    if (e != hipSuccess) return hip_fail(e, "hipMalloc(fibre scratch)");
    fd->allocs.push_back(sp);
    fd->scratch = (double*)sp;
  }
  return SGDG_OK;
}

template <int K1, int UC>
static void launch_uc(const FibreData& fd, const Launch& l, int nrhs, const double* x, double* y, int64_t xs,
                      int64_t ys, int acc, hipStream_t s) {
  static std::atomic<bool> attr{false};
  if (!attr.load()) {
    (void)hipFuncSetAttribute((const void*)k_fibre<K1, UC>, hipFuncAttributeMaxDynamicSharedMemorySize, FB_LDS);
    attr.store(true);
  }
  hipLaunchKernelGGL((k_fibre<K1, UC>), dim3((unsigned)l.tasks.size()), dim3(FB_NT), FB_LDS, s, l.dtasks, fd.bases,
                     fd.ops, fd.scratch, x, y, xs, ys, nrhs, acc, fd.dts + K1);
}

// The kernel is built for launches whose operators all keep one block triple
// per level (translation invariant: constant k, periodic), all keep one per
// cell, or a mix: the first two leave the other branch out of the register
// budget.
template <int K1>
static void launch_phase(const FibreData& fd, const Launch& l, int nrhs, const double* x, double* y, int64_t xs,
                         int64_t ys, int acc, hipStream_t s) {
  if (l.tasks.empty()) return;
  switch (l.uc) {
    case 0: launch_uc<K1, 0>(fd, l, nrhs, x, y, xs, ys, acc, s); break;
    case 1: launch_uc<K1, 1>(fd, l, nrhs, x, y, xs, ys, acc, s); break;
    default: launch_uc<K1, 2>(fd, l, nrhs, x, y, xs, ys, acc, s); break;
  }
}

template <int K1>
static void launch_group(const FibreData& fd, const Group& g, int nrhs, const double* x, double* y, int64_t xs,
                         int64_t ys, hipStream_t s) {
  const int acc = g.dir > 0 ? 1 : 0;
  if (g.ph[0].tasks.empty()) {
    launch_phase<K1>(fd, g.ph[1], nrhs, x, y, xs, ys, acc, s);
    return;
  }
  // split fibres: the coarse values in scratch serve one right-hand side at a time
  for (int r = 0; r < nrhs; ++r)
    for (const Launch& l : g.ph) launch_phase<K1>(fd, l, 1, x + r * xs, y + r * ys, xs, ys, acc, s);
}

void launch_fibre(const sgdg_plan* p, int nrhs, const double* x, double* y, int64_t xs, int64_t ys, hipStream_t s) {
  const FibreData& fd = *p->fdata;
  for (const Group& g : fd.groups) {
    switch (g.K1) {
      case 2: launch_group<2>(fd, g, nrhs, x, y, xs, ys, s); break;
      case 3: launch_group<3>(fd, g, nrhs, x, y, xs, ys, s); break;
      default: launch_group<4>(fd, g, nrhs, x, y, xs, ys, s); break;
    }
  }
}

}  // namespace sgdg

using namespace sgdg;

extern "C" sgdg_status sg_dg_sweep_form(sgdg_plan* plan, int32_t form) {
  if (!plan) return fail(SGDG_ERR_ARG, "sg_dg_sweep_form: null plan");
  if (form < 0 || form > 3) return fail(SGDG_ERR_ARG, "sg_dg_sweep_form: form must be 0..3");
  if (form == 0) form = fibre_auto(plan) ? 2 : 1;
  if (form >= 2) {
    if (plan->prec != SGDG_FP64)
      return fail(SGDG_ERR_UNSUPPORTED, "sg_dg_sweep_form: the fibre form runs FP64 plans only");
    hipError_t e = hipSetDevice(plan->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    e = hipDeviceSynchronize();  // tables of an earlier selection may be in use
    if (e != hipSuccess) return hip_fail(e, "hipDeviceSynchronize");
    sgdg_status st = fibre_build(plan, form == 3);
    if (st != SGDG_OK) {
      fibre_destroy(plan);
      plan->fibre_on = false;
      return st;
    }
  }
  plan->fibre_on = (form >= 2);
  return SGDG_OK;
}
