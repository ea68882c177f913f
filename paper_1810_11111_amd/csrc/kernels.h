// Device-side building blocks shared by the sweep, Krylov and reaction kernels.
#pragma once

#include <hip/hip_runtime.h>

#include "internal.h"

namespace sgdg {

// bfloat16 stored as its 16 high float bits; round to nearest even on store.
__device__ __forceinline__ float bf16_to_f(uint16_t b) { return __uint_as_float(((uint32_t)b) << 16); }
__device__ __forceinline__ uint16_t f_to_bf16(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));  // inf/nan
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

// Precision policies of a sweep: input element, output element, matrix value, accumulator.
struct PrecF64 {
  using X = double;
  using Y = double;
  using V = double;
  using A = double;
  __device__ static A load(const X* p) { return *p; }
  __device__ static const V* vals(const DevTables& T) { return T.val; }
};
struct PrecF32 {
  using X = float;
  using Y = float;
  using V = float;
  using A = float;
  __device__ static A load(const X* p) { return *p; }
  __device__ static const V* vals(const DevTables& T) { return T.valf; }
};
struct PrecBF16 {
  using X = uint16_t;
  using Y = float;
  using V = float;
  using A = float;
  __device__ static A load(const X* p) { return bf16_to_f(*p); }
  __device__ static const V* vals(const DevTables& T) { return T.valf; }
};

// Locate the level block of global element g inside chunk ch (binary search
// over the chunk's block range).
__device__ __forceinline__ int find_block(const DevTables& T, const Chunk& ch, int64_t g) {
  int lo = ch.b0, hi = ch.b1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (T.gblk[mid].start <= g)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

// Source of the gathered x values: global memory with the plan's block
// tables, or the problem's segment staged in LDS with its block-start table.
template <class P>
struct SrcGlobal {
  const typename P::X* __restrict__ x;  // start of the plan vector
  const int32_t* __restrict__ blkid;    // instance's (N+1)^d table into lstart
  const int64_t* __restrict__ lstart;
  int64_t seg;                          // start of the species segment
  __device__ __forceinline__ int64_t block_base(int lin) const { return seg + lstart[blkid[lin]]; }
  __device__ __forceinline__ typename P::A load(int64_t i) const { return P::load(x + i); }
};
template <class P>
struct SrcLds {
  const typename P::X* x;  // LDS copy of the species segment
  const int32_t* bst;      // LDS: block start inside the segment per level tuple
  __device__ __forceinline__ int64_t block_base(int lin) const { return bst[lin]; }
  __device__ __forceinline__ typename P::A load(int64_t i) const { return P::load(x + i); }
};

// Row structure of the 1D operators: from global memory, or staged in LDS
// (cptr / src of every direction copied to one LDS array).
struct RowsGlobal {
  const int32_t* cptr;
  const int32_t* src;
  __device__ __forceinline__ int rp(const BCsr& bc, int i, int t) const { return cptr[bc.cptr_off + t]; }
  __device__ __forceinline__ int sc(const BCsr& bc, int i, int e) const { return src[bc.src_off + e]; }
};
struct RowsLds {
  const int32_t* cptr[SGDG_MAX_D];  // LDS, per direction: row pointers of target cells tlo.. (entry numbers of the CSR)
  const int32_t* src[SGDG_MAX_D];   // LDS: source cells of entries elo..
  int32_t tlo[SGDG_MAX_D], elo[SGDG_MAX_D];
  // entry numbers relative to elo (so that src[e] and the block values of entry e are at e)
  __device__ __forceinline__ int rp(const BCsr& bc, int i, int t) const { return cptr[i][t - tlo[i]] - elo[i]; }
  __device__ __forceinline__ int sc(const BCsr& bc, int i, int e) const { return src[i][e]; }
};

// Block values of the 1D operators: global table, or each direction's table
// staged in LDS.
template <class P>
struct ValsGlobal {
  const typename P::V* __restrict__ v;
  __device__ __forceinline__ const typename P::V* row(const BCsr& bc, int i) const { return v + bc.val_off; }
};
template <class P>
struct ValsLds {
  const typename P::V* v[SGDG_MAX_D];
  __device__ __forceinline__ const typename P::V* row(const BCsr& bc, int i) const { return v[i]; }
};

// Partial y_g = (A x)_g for one output element g of a plan vector, from the
// row entries e = e0 + lane, e0 + lane + G, ... of every direction (G lanes
// share one output; the caller sums the G partials).  Already scaled by
// -D_s.  Rows of B_i are walked in ascending source cell order, so the block
// base of a source level is looked up once per level, not per entry.
template <int D, int K, class P, class Src, class Rows, class Vals>
__device__ __forceinline__ typename P::A apply_one(const DevTables& T, const GBlock& B, const InstDev& I, int64_t g,
                                                   int lane, int G, const Src& xs, const Rows& rows, const Vals& vs) {
  using A = typename P::A;
  using V = typename P::V;
  constexpr int K1 = K + 1;
  int ext[D], sh[D], t[D], lev[D];
  int L = (int)(g - B.start);
  {
    int rem = L;
    for (int m = D - 1; m >= 0; --m) {
      lev[m] = B.lev[m];
      sh[m] = lev[m] > 0 ? lev[m] - 1 : 0;
      ext[m] = K1 << sh[m];
      int q = (rem / K1) >> sh[m];
      t[m] = rem - q * ext[m];
      rem = q;
    }
  }
  // strides, prefix (axes before i) and suffix (axes after i) offsets
  int str[D];
  str[D - 1] = 1;
  for (int m = D - 2; m >= 0; --m) str[m] = str[m + 1] * ext[m + 1];
  int pre[D + 1], suf[D + 1];
  pre[0] = 0;
  for (int m = 0; m < D; ++m) pre[m + 1] = pre[m] * ext[m] + t[m];
  suf[D] = 0;
  for (int m = D - 1; m >= 0; --m) suf[m] = suf[m + 1] + t[m] * str[m];
  int linall = 0;
  for (int m = 0; m < D; ++m) linall += lev[m] * I.pow[m];

  A acc = 0;
#pragma unroll
  for (int i = 0; i < D; ++i) {
    const int li = lev[i];
    const int budget = I.N - B.lsum + li;
    const int lim = 1 << budget;
    const int pt = t[i] % K1;
    const int jt = t[i] / K1;
    const int tcell = li == 0 ? 0 : (1 << (li - 1)) + jt;
    const int S = str[i];
    const int Ahi = pre[i];
    const int Blo = suf[i + 1];
    const int lin = linall - li * I.pow[i];
    const BCsr bc = T.bcsr[I.bcsr_off[i]];
    const int e0 = rows.rp(bc, i, tcell);
    const int e1 = rows.rp(bc, i, tcell + 1);
    const V* __restrict__ vrow = vs.row(bc, i) + pt * K1;
    int cur_lc = -1;
    int64_t bbase = 0;
    int extc = K1;
    for (int e = e0 + lane; e < e1; e += G) {
      const int sc = rows.sc(bc, i, e);
      if (sc >= lim) break;
      const int lc = sc == 0 ? 0 : 32 - __clz(sc);
      if (lc != cur_lc) {
        cur_lc = lc;
        bbase = xs.block_base(lin + lc * I.pow[i]);
        extc = lc == 0 ? K1 : (K1 << (lc - 1));
      }
      const int jc = sc == 0 ? 0 : sc - (1 << (lc - 1));
      const int64_t base = bbase + (int64_t)(Ahi * extc + jc * K1) * S + Blo;
      const V* __restrict__ v = vrow + (int64_t)e * K1 * K1;
#pragma unroll
      for (int pc = 0; pc < K1; ++pc) acc += (A)v[pc] * xs.load(base + (int64_t)pc * S);
    }
  }
  return acc * (A)(-I.D[B.species]);
}

// LDS budget of the staged sweeps (block table, row tables, x segment and,
// when they fit, the block values).
constexpr int APPLY_LDS_BYTES = APPLY_LDS_BYTES_HOST;

template <class P>
void launch_apply(const sgdg_plan* plan, int nrhs, const void* x, void* y, int64_t xs, int64_t ys, hipStream_t s);

// Arnoldi form of the sweep: after y = A x of a chunk, the same workgroup
// writes the chunk's partial inner products <v_i, y>, i = 0..j, of the basis
// vectors V (element type TV, [i][rhs][total]) to part[(rhs * nchunks + chunk)
// * ld + i].
struct DotArgs {
  const void* V;
  double* part;
  int32_t j, ld, nchunks, nrhs;
  int64_t total;
};
template <class P, class TV>
void launch_apply_dots(const sgdg_plan* plan, int nrhs, const void* x, void* y, const DotArgs& da, hipStream_t s);

}  // namespace sgdg
