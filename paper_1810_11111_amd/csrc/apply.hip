// Matrix-free application of the sparse-grid interior-penalty operator.
//
// A = - sum_i D_s (I x .. x B_i x .. x I) restricted to the sparse index set
// (Sec. 2.1, eq. 2.10 with orthonormal basis; the "unidirectional principle"
// of Sec. 4).  For an output DOF with level tuple l and axis-i position t_i,
// direction i contributes sum over source cells of B_i[(l_i,t_i),(l'_i,t'_i)]
// times x at the same position on every other axis, for source levels
// l'_i <= N - |l| + l_i (the fibre's level budget, i.e. the leading block of
// the level-N 1D operator).  Each lane produces one output entry (no atomics,
// no read-modify-write of y); rows of B_i are stored as cell blocks so a
// group of K+1 consecutive source entries shares one index decode.
//
// Three tiers, chosen per chunk when the plan is built: when the species
// segment, its level-block table and the chunk's rows of the 1D operators fit
// in LDS, every workgroup first stages them there and gathers from LDS (small
// problems are latency bound: a gather then costs LDS latency, not L2
// latency), and when the block values fit as well they are staged too;
// otherwise the gathers read global memory, with the source-block starts the
// chunk needs in an LDS table and the row entries loaded a few at a time.
// Each output gets 4..64 lanes (APPLY_G and up, by the length of its rows), so
// the heavy rows of coarse levels do not hold back a chunk.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <type_traits>

#include "internal.h"
#include "kernels.h"

namespace sgdg {

// Chunk-level inner products of the Arnoldi form (DotArgs): wl holds the
// chunk's sweep output (zero past its end); wave w takes basis vectors
// i = w, w + nwaves, ..., DB of them at a time with all their loads in
// flight together; the order of every sum is fixed.
template <class TV>
__device__ __forceinline__ void chunk_dots_out(const DotArgs& da, int c, int rhs, const Chunk& ch, const double* wl) {
  constexpr int DB = 4, QN = CHUNK / 64;
  const int wv = threadIdx.x >> 6, ln = threadIdx.x & 63, nw = blockDim.x >> 6;
  double w[QN];
#pragma unroll
  for (int u = 0; u < QN; ++u) w[u] = wl[ln + 64 * u];
  for (int i0 = wv; i0 <= da.j; i0 += DB * nw) {
    double x[DB][QN];
#pragma unroll
    for (int b = 0; b < DB; ++b) {
      const int i = min(i0 + b * nw, da.j);
      const TV* v = (const TV*)da.V + ((int64_t)i * da.nrhs + rhs) * da.total + ch.start;
#pragma unroll
      for (int u = 0; u < QN; ++u) x[b][u] = (double)v[min(ln + 64 * u, ch.count - 1)];
    }
#pragma unroll
    for (int b = 0; b < DB; ++b) {
      double s = 0.0;
#pragma unroll
      for (int u = 0; u < QN; ++u)
        if (ln + 64 * u < ch.count) s += x[b][u] * w[u];
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
      if (ln == 0 && i0 + b * nw <= da.j) da.part[((int64_t)rhs * da.nchunks + c) * da.ld + i0 + b * nw] = s;
    }
  }
}

// The staged kernel's form of the same products: 16 waves, so wave w takes
// i = w, w + 16, w + 32 (i <= j <= SGDG_MAX_M - 1); the basis entries are
// loaded into registers at kernel start (pre_basis) so that their latency
// overlaps the staging and the sweep.  Same summation order as above.
constexpr int PRE_W = CHUNK * APPLY_G / 64;
constexpr int PRE_I = (SGDG_MAX_M + PRE_W - 1) / PRE_W;
constexpr int PRE_Q = CHUNK / 64;
static_assert(PRE_W == 16, "the staged kernel has 16 waves");

template <class TV, int PI>
__device__ __forceinline__ void pre_basis(const DotArgs& da, int rhs, const Chunk& ch, double (&vp)[PI][PRE_Q]) {
  const int wv = threadIdx.x >> 6, ln = threadIdx.x & 63;
#pragma unroll
  for (int a = 0; a < PI; ++a) {
    const int i = wv + a * PRE_W;
#pragma unroll
    for (int b = 0; b < PRE_Q; ++b)  // clamped indices: no load sits under a branch; the excess is masked later
      vp[a][b] = (double)((const TV*)da.V + ((int64_t)min(i, da.j) * da.nrhs + rhs) * da.total +
                          ch.start)[min(ln + 64 * b, ch.count - 1)];
  }
}

template <int PI>
__device__ __forceinline__ void chunk_dots_pre(const DotArgs& da, int c, int rhs, const Chunk& ch,
                                               const double (&vp)[PI][PRE_Q], const double* wl) {
  const int wv = threadIdx.x >> 6, ln = threadIdx.x & 63;
#pragma unroll
  for (int a = 0; a < PI; ++a) {
    const int i = wv + a * PRE_W;
    if (i > da.j) break;
    double s = 0.0;
#pragma unroll
    for (int b = 0; b < PRE_Q; ++b) s += (ln + 64 * b < ch.count ? vp[a][b] : 0.0) * wl[ln + 64 * b];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    if (ln == 0) da.part[((int64_t)rhs * da.nchunks + c) * da.ld + i] = s;
  }
}

// Global-gather form of apply_one for the outputs of a chunk's first block:
// the source block of level lc in direction i starts at bb[i * BB_L + lc]
// (a table the workgroup builds in LDS), and each lane takes its row entries
// RB at a time -- their source cells loaded together, then every block value
// and x entry of the RB entries, then the products -- so a round costs three
// dependent memory round trips where the entry-by-entry walk costs two per
// entry plus two table loads per source level.  Entries past the row or the
// level budget are masked (their clamped loads stay inside the source
// blocks), and the walk ends with the round that reaches the budget; the
// products are summed in the order apply_one sums them.
constexpr int BB_L = 32;

// (measured for d=3 N=16 k=1 before the wave-uniform walk below: 2 entries
// per lane per round 1.60 ms, 4: 1.64, 8: 1.88, the entry-by-entry walk 2.20;
// with it, 2 entries per round there as well: 1.49 ms, 4: 1.52, 8: 1.59)
template <int K>
constexpr int batch_entries() {
  return 2;
}

template <int D, int K, class P>
__device__ __forceinline__ typename P::A apply_one_batched(const DevTables& T, const GBlock& B, const InstDev& I,
                                                           int64_t g, int lane, int G,
                                                           const typename P::X* __restrict__ x, const int64_t* bb) {
  using A = typename P::A;
  using V = typename P::V;
  constexpr int K1 = K + 1;
  constexpr int RB = batch_entries<K>();
  int ext[D], sh[D], t[D], lev[D];
  {
    int rem = (int)(g - B.start);
    for (int m = D - 1; m >= 0; --m) {
      lev[m] = B.lev[m];
      sh[m] = lev[m] > 0 ? lev[m] - 1 : 0;
      ext[m] = K1 << sh[m];
      const int q = (rem / K1) >> sh[m];
      t[m] = rem - q * ext[m];
      rem = q;
    }
  }
  int str[D];
  str[D - 1] = 1;
  for (int m = D - 2; m >= 0; --m) str[m] = str[m + 1] * ext[m + 1];
  int pre[D + 1], suf[D + 1];
  pre[0] = 0;
  for (int m = 0; m < D; ++m) pre[m + 1] = pre[m] * ext[m] + t[m];
  suf[D] = 0;
  for (int m = D - 1; m >= 0; --m) suf[m] = suf[m + 1] + t[m] * str[m];
  const V* __restrict__ vals = P::vals(T);
  A acc = 0;
#pragma unroll
  for (int i = 0; i < D; ++i) {
    const int li = lev[i];
    const int lim = 1 << (I.N - B.lsum + li);
    const int pt = t[i] % K1, jt = t[i] / K1;
    const int tcell = li == 0 ? 0 : (1 << (li - 1)) + jt;
    const int S = str[i], Ahi = pre[i], Blo = suf[i + 1];
    const BCsr bc = T.bcsr[I.bcsr_off[i]];
    const int32_t* __restrict__ srow = T.src + bc.src_off;
    const int64_t* bbi = bb + i * BB_L;
    // when every lane of the wave reads the same row (one lane per output,
    // and the wave's outputs differ only in the axes after i), the row is
    // walked once with wave-uniform loads of its source cells and block
    // values; only x differs between the lanes, at consecutive addresses
    const int tc0 = __builtin_amdgcn_readfirstlane(tcell);
    const int pt0 = __builtin_amdgcn_readfirstlane(pt);
    const int ah0 = __builtin_amdgcn_readfirstlane(Ahi);
    if (G == 1 && __builtin_amdgcn_ballot_w64(tcell != tc0 || pt != pt0 || Ahi != ah0) == 0) {
      constexpr int RU = 2;
      const int u0 = T.cptr[bc.cptr_off + tc0], u1 = T.cptr[bc.cptr_off + tc0 + 1];
      const V* __restrict__ vrow0 = vals + bc.val_off + pt0 * K1;
      for (int eb = u0; eb < u1; eb += RU) {
        int sc[RU];
#pragma unroll
        for (int r = 0; r < RU; ++r) sc[r] = srow[min(eb + r, u1 - 1)];
        A xv[RU][K1];
        V vv[RU][K1];
        bool ok[RU];
#pragma unroll
        for (int r = 0; r < RU; ++r) {
          ok[r] = eb + r < u1 && sc[r] < lim;
          const int lc = ok[r] && sc[r] > 0 ? 32 - __clz(sc[r]) : 0;
          const int extc = lc == 0 ? K1 : (K1 << (lc - 1));
          const int jc = lc == 0 ? 0 : sc[r] - (1 << (lc - 1));
          const int64_t base = bbi[lc] + (int64_t)(ah0 * extc + jc * K1) * S + Blo;
          const V* __restrict__ v = vrow0 + (int64_t)min(eb + r, u1 - 1) * K1 * K1;
#pragma unroll
          for (int pc = 0; pc < K1; ++pc) {
            vv[r][pc] = v[pc];
            xv[r][pc] = P::load(x + base + (int64_t)pc * S);
          }
        }
#pragma unroll
        for (int r = 0; r < RU; ++r)
#pragma unroll
          for (int pc = 0; pc < K1; ++pc) acc += (ok[r] ? (A)vv[r][pc] : (A)0) * (ok[r] ? xv[r][pc] : (A)0);
        if (sc[RU - 1] >= lim) break;
      }
      continue;
    }
    const int e0 = T.cptr[bc.cptr_off + tcell], e1 = T.cptr[bc.cptr_off + tcell + 1];
    const V* __restrict__ vrow = vals + bc.val_off + pt * K1;
    for (int eb = e0 + lane; eb < e1; eb += RB * G) {
      int sc[RB];
#pragma unroll
      for (int r = 0; r < RB; ++r) sc[r] = srow[min(eb + r * G, e1 - 1)];
      A xv[RB][K1];
      V vv[RB][K1];
      bool ok[RB];
#pragma unroll
      for (int r = 0; r < RB; ++r) {
        ok[r] = eb + r * G < e1 && sc[r] < lim;
        const int lc = ok[r] && sc[r] > 0 ? 32 - __clz(sc[r]) : 0;
        const int extc = lc == 0 ? K1 : (K1 << (lc - 1));
        const int jc = lc == 0 ? 0 : sc[r] - (1 << (lc - 1));
        const int64_t base = bbi[lc] + (int64_t)(Ahi * extc + jc * K1) * S + Blo;
        const V* __restrict__ v = vrow + (int64_t)min(eb + r * G, e1 - 1) * K1 * K1;
#pragma unroll
        for (int pc = 0; pc < K1; ++pc) {
          vv[r][pc] = v[pc];
          xv[r][pc] = P::load(x + base + (int64_t)pc * S);
        }
      }
#pragma unroll
      for (int r = 0; r < RB; ++r)
#pragma unroll
        for (int pc = 0; pc < K1; ++pc) acc += (ok[r] ? (A)vv[r][pc] : (A)0) * (ok[r] ? xv[r][pc] : (A)0);
      // a row lists its source cells in ascending order (coarse levels
      // first), so once an entry is past the level budget the rest are too
      if (sc[RB - 1] >= lim) break;
    }
  }
  return acc * (A)(-I.D[B.species]);
}

template <int D, int K, class P, class TV>
__global__ __launch_bounds__(CHUNK) void apply_kernel(DevTables T, const int32_t* __restrict__ list,
                                                      const typename P::X* __restrict__ x, typename P::Y* __restrict__ y,
                                                      int64_t xstride, int64_t ystride, DotArgs da) {
  const int c = list[blockIdx.x];
  const Chunk ch = T.chunks[c];
  const int tid = threadIdx.x;
  const int64_t rhs = blockIdx.y;
  // start of every source block the chunk's first block reads, per direction
  // and source level (one thread each, all loads in flight together)
  __shared__ int64_t bb[SGDG_MAX_D * BB_L];
  const GBlock& B0 = T.gblk[ch.b0];
  const InstDev& I0 = T.inst[B0.inst];
  const bool tab = I0.N < BB_L;
  if (tab && tid < D * BB_L) {
    const int i = tid / BB_L, lc = tid - i * BB_L;
    if (lc <= I0.N - B0.lsum + B0.lev[i]) {
      int lin = (lc - B0.lev[i]) * I0.pow[i];
      for (int m = 0; m < D; ++m) lin += B0.lev[m] * I0.pow[m];
      bb[tid] = I0.offset + (int64_t)B0.species * I0.ndof + T.lstart[T.blkid[I0.blkid_off + lin]];
    }
  }
  __syncthreads();
  // chunks of heavy (coarse-level) rows give each output several lanes
  const int G = ch.g / APPLY_G;
  const int e = tid / G, lane = tid - e * G;
  const bool active = e < ch.count;
  typename P::A acc = 0;
  if (active) {
    const int64_t g = ch.start + e;
    if (tab && g < B0.start + B0.size) {
      acc = apply_one_batched<D, K, P>(T, B0, I0, g, lane, G, x + rhs * xstride, bb);
    } else {
      const GBlock& B = T.gblk[find_block(T, ch, g)];
      const InstDev& I = T.inst[B.inst];
      SrcGlobal<P> xs{x + rhs * xstride, T.blkid + I.blkid_off, T.lstart, I.offset + (int64_t)B.species * I.ndof};
      RowsGlobal rows{T.cptr, T.src};
      ValsGlobal<P> vs{P::vals(T)};
      acc = apply_one<D, K, P>(T, B, I, g, lane, G, xs, rows, vs);
    }
  }
  for (int o = 1; o < G; o <<= 1) acc += __shfl_xor(acc, o, 64);
  const typename P::Y out = (typename P::Y)acc;
  if (active && lane == 0) y[rhs * ystride + ch.start + e] = out;
  if constexpr (!std::is_void_v<TV>) {
    __shared__ double wl[CHUNK];
    wl[tid] = 0.0;
    __syncthreads();
    if (active && lane == 0) wl[e] = (double)out;
    __syncthreads();
    chunk_dots_out<TV>(da, c, (int)rhs, ch, wl);
  }
}

constexpr int64_t lds_al256(int64_t b) { return (b + 255) & ~(int64_t)255; }

typedef __attribute__((address_space(3))) void* lds_void_ptr;

// Direct global -> LDS copy (global_load_lds: one instruction moves 16 bytes
// per lane of a wave, lane l's bytes landing at the wave's LDS address + 16 l;
// 4-byte variant for the unaligned ends) of nbytes (a multiple of 4) from a
// 4-byte aligned src into the 16-byte aligned LDS region dst, which must hold
// nbytes + 16 bytes.  The copy keeps src's position within its 16-byte line,
// so the returned LDS pointer of the array is dst + (src mod 16).  Pieces of
// 64 lines go to the waves in turn; lanes past the end are inactive, so
// nothing outside the array is read.  Nothing waits here: the caller waits for
// vmcnt(0) and synchronises before the LDS is read.
__device__ __forceinline__ void* dma_copy(void* dst, const void* src, int64_t nbytes, int wave, int nwave, int lane) {
  const uintptr_t s = (uintptr_t)src, s_al = s & ~(uintptr_t)15, e = s + (uintptr_t)nbytes;
  unsigned char* base = (unsigned char*)dst;  // LDS image of global address t: base + (t - s_al)
  const uintptr_t a = (s + 15) & ~(uintptr_t)15, b = e & ~(uintptr_t)15;
  if (nbytes <= 0) return base + (s - s_al);
  if (a >= b) {
    // no whole 16-byte line inside: at most 7 dwords, one 4-byte instruction
    const int n = (int)(nbytes >> 2);
    if (wave == 0 && lane < n)
      __builtin_amdgcn_global_load_lds((const void*)(s + 4 * (uintptr_t)lane), (lds_void_ptr)(base + (s - s_al)), 4, 0,
                                       0);
    return base + (s - s_al);
  }
  const int nh = (int)((a - s) >> 2), nt = (int)((e - b) >> 2);
  if (wave == 0 && lane < nh)
    __builtin_amdgcn_global_load_lds((const void*)(s + 4 * (uintptr_t)lane), (lds_void_ptr)(base + (s - s_al)), 4, 0, 0);
  if (wave == nwave - 1 && lane < nt)
    __builtin_amdgcn_global_load_lds((const void*)(b + 4 * (uintptr_t)lane), (lds_void_ptr)(base + (b - s_al)), 4, 0, 0);
  const int64_t n16 = (int64_t)((b - a) >> 4);
  unsigned char* mid = base + (a - s_al);
  for (int64_t q = wave; q * 64 < n16; q += nwave) {
    const int64_t idx = q * 64 + lane;
    if (idx < n16)
      __builtin_amdgcn_global_load_lds((const void*)(a + 16 * (uintptr_t)idx), (lds_void_ptr)(mid + q * 1024), 16, 0, 0);
  }
  return base + (s - s_al);
}

// Staged variant: the workgroup copies the problem's level-block table, the
// row tables of its distinct 1D operators, its x segment and (STAGE_VALS) the
// block values into LDS, then APPLY_G lanes share each output element and
// split its row entries; their partial sums are combined in a fixed order.
// PI: rounds of 16 basis vectors the fused inner products need (j < 16 PI)
template <int D, int K, class P, bool STAGE_VALS, class TV, int PI>
__global__ __launch_bounds__(CHUNK* APPLY_G) void apply_kernel_lds(DevTables T, const SweepTask* __restrict__ tasks,
                                                                   const typename P::X* __restrict__ x,
                                                                   typename P::Y* __restrict__ y, int64_t xstride,
                                                                   int64_t ystride, DotArgs da) {
  using V = typename P::V;
  extern __shared__ __align__(16) unsigned char smem[];
  // one record holds everything needed before the first copy
  const SweepTask& tk = tasks[blockIdx.x];
  const int cid = tk.cid;
  Chunk ch{};
  ch.start = tk.start;
  ch.count = tk.count;
  ch.b0 = tk.b0;
  ch.b1 = tk.b1;
  ch.inst = tk.inst;
  ch.species = tk.species;
  ch.g = tk.g;
  const int tid = threadIdx.x;
  const int nthr = blockDim.x;
  const int64_t rhs = blockIdx.y;
  const int64_t seg = tk.seg, ndof = tk.ndof;
  const int ntab = tk.ntab;
  double vpre[PI][PRE_Q];
  if constexpr (!std::is_void_v<TV>) pre_basis<TV, PI>(da, (int)rhs, ch, vpre);
  // LDS layout (regions of 256-byte multiples with 16 bytes of slack, as the
  // direct copies keep each array's offset within its 16-byte line):
  // block-start table | per direction: the chunk's row pointers, source cells
  // | x segment | (STAGE_VALS) per direction: the chunk's block values.  The
  // tables and x are moved by direct global -> LDS copies, all in flight
  // together; only the block-start table goes through VGPRs.
  const int wave = tid >> 6, wl64 = tid & 63, nwave = nthr >> 6;
  int32_t* bst = (int32_t*)smem;
  const int bid = tid < ntab ? T.blkid[tk.blkid_off + tid] : -1;
  unsigned char* cur = smem + lds_al256((int64_t)ntab * 4);
  // per direction, only the rows this chunk's outputs use (row pointers,
  // source cells and, with STAGE_VALS, block values); directions sharing an
  // operator share its copy (every index below is a compile-time constant
  // after unrolling, so the pointer tables stay in registers)
  RowsLds rows;
  ValsLds<P> vl;
  const unsigned dup = tk.dup;
#pragma unroll
  for (int i = 0; i < D; ++i) {
    rows.tlo[i] = tk.tlo[i];
    rows.elo[i] = tk.elo[i];
#pragma unroll
    for (int i2 = 0; i2 < i; ++i2)
      if (((dup >> i) & 1u) && tk.cp[i2] == tk.cp[i]) {
        rows.cptr[i] = rows.cptr[i2];
        rows.src[i] = rows.src[i2];
      }
    if ((dup >> i) & 1u) continue;
    rows.cptr[i] = (int32_t*)dma_copy(cur, T.cptr + tk.cp[i], ((int64_t)tk.nrow[i] + 1) * 4, wave, nwave, wl64);
    cur += lds_al256(((int64_t)tk.nrow[i] + 1) * 4 + 16);
    rows.src[i] = (int32_t*)dma_copy(cur, T.src + tk.sp[i], (int64_t)tk.nent[i] * 4, wave, nwave, wl64);
    cur += lds_al256((int64_t)tk.nent[i] * 4 + 16);
  }
  typename P::X* xl = (typename P::X*)cur;
  const typename P::X* __restrict__ xg = x + rhs * xstride + seg;
  if constexpr (sizeof(typename P::X) >= 4)
    xl = (typename P::X*)dma_copy(cur, xg, ndof * (int64_t)sizeof(typename P::X), wave, nwave, wl64);
  else
    for (int64_t i = tid; i < ndof; i += nthr) xl[i] = xg[i];
  cur += lds_al256(ndof * (int64_t)sizeof(typename P::X) + 16);
  {
    const V* __restrict__ vals = P::vals(T);
    constexpr int64_t KK = (int64_t)(K + 1) * (K + 1);
#pragma unroll
    for (int i = 0; i < D; ++i) {
#pragma unroll
      for (int i2 = 0; i2 < i; ++i2)
        if (((dup >> i) & 1u) && tk.cp[i2] == tk.cp[i]) vl.v[i] = vl.v[i2];
      if ((dup >> i) & 1u) continue;
      if constexpr (STAGE_VALS) {
        vl.v[i] = (V*)dma_copy(cur, vals + tk.vp[i], (int64_t)tk.nent[i] * KK * (int64_t)sizeof(V), wave, nwave, wl64);
        cur += lds_al256((int64_t)tk.nent[i] * KK * (int64_t)sizeof(V) + 16);
      } else {
        vl.v[i] = vals + tk.vp[i];  // the block values stay in global memory
      }
    }
  }
  if (tid < ntab) bst[tid] = bid >= 0 ? (int32_t)T.lstart[bid] : -1;
  // tables larger than the workgroup ((N+1)^d > 1024, e.g. d = 4, N >= 5)
  for (int t2 = tid + nthr; t2 < ntab; t2 += nthr) {
    const int b2 = T.blkid[tk.blkid_off + t2];
    bst[t2] = b2 >= 0 ? (int32_t)T.lstart[b2] : -1;
  }
  __builtin_amdgcn_s_waitcnt(0);  // the direct copies have landed
  __syncthreads();
  // ch.g lanes per output: APPLY_G for most chunks, more for the chunks of
  // coarse levels, whose rows reach every finer cell under their support
  const int G = ch.g;
  const int e = tid / G;
  const int lane = tid - e * G;
  const bool active = e < ch.count;
  typename P::A acc = 0;
  if (active) {
    const InstDev& I = T.inst[ch.inst];
    const int64_t g = ch.start + e;
    const GBlock& B = T.gblk[find_block(T, ch, g)];
    SrcLds<P> xs{xl, bst};
    acc = apply_one<D, K, P>(T, B, I, g, lane, G, xs, rows, vl);
  }
  // fixed-order combination of the lane partials (butterfly within each
  // aligned group of G lanes)
  for (int o = 1; o < G; o <<= 1) acc += __shfl_xor(acc, o, 64);
  const typename P::Y out = (typename P::Y)acc;
  if (active && lane == 0) y[rhs * ystride + ch.start + e] = out;
  if constexpr (!std::is_void_v<TV>) {
    __syncthreads();  // the staged tables are dead; reuse the LDS for the chunk output
    double* wl = (double*)smem;
    if (tid < CHUNK) wl[tid] = 0.0;
    __syncthreads();
    if (active && lane == 0) wl[e] = (double)out;
    __syncthreads();
    chunk_dots_pre<PI>(da, cid, (int)rhs, ch, vpre, wl);
  }
}

template <int D, int K, class P, bool SV, class TV>
static void launch_staged(const sgdg_plan* plan, int kind, int nrhs, const void* x, void* y, int64_t xs, int64_t ys,
                          const DotArgs& da, hipStream_t s) {
  // the Arnoldi form reuses the LDS for one chunk of output (CHUNK doubles)
  const int lds = std::max(plan->list_lds[kind], std::is_void_v<TV> ? 0 : (int)(CHUNK * sizeof(double)));
  static std::atomic<int> attr_set{0};
  if (attr_set.load() < lds) {
    hipFuncSetAttribute((const void*)apply_kernel_lds<D, K, P, SV, TV, 1>, hipFuncAttributeMaxDynamicSharedMemorySize,
                        APPLY_LDS_BYTES);
    if constexpr (!std::is_void_v<TV>) {
      hipFuncSetAttribute((const void*)apply_kernel_lds<D, K, P, SV, TV, 2>,
                          hipFuncAttributeMaxDynamicSharedMemorySize, APPLY_LDS_BYTES);
      hipFuncSetAttribute((const void*)apply_kernel_lds<D, K, P, SV, TV, PRE_I>,
                          hipFuncAttributeMaxDynamicSharedMemorySize, APPLY_LDS_BYTES);
    }
    attr_set.store(APPLY_LDS_BYTES);
  }
  const dim3 grid((unsigned)plan->chunk_lists[kind].size(), (unsigned)nrhs), blk(CHUNK * APPLY_G);
  const SweepTask* tk = plan->dev_tasks[kind];
  const auto* xp = (const typename P::X*)x;
  auto* yp = (typename P::Y*)y;
  // the basis vectors loaded for the fused inner products: only as many
  // rounds of 16 as step j needs
  if (std::is_void_v<TV> || da.j < PRE_W)
    hipLaunchKernelGGL((apply_kernel_lds<D, K, P, SV, TV, 1>), grid, blk, lds, s, plan->dev, tk, xp, yp, xs, ys, da);
  else if (da.j < 2 * PRE_W)
    hipLaunchKernelGGL((apply_kernel_lds<D, K, P, SV, TV, 2>), grid, blk, lds, s, plan->dev, tk, xp, yp, xs, ys, da);
  else
    hipLaunchKernelGGL((apply_kernel_lds<D, K, P, SV, TV, PRE_I>), grid, blk, lds, s, plan->dev, tk, xp, yp, xs, ys,
                       da);
}

template <int D, int K, class P, class TV>
static void launch_kind(const sgdg_plan* plan, int nrhs, const void* x, void* y, int64_t xs, int64_t ys,
                        const DotArgs& da, hipStream_t s) {
  const int k0 = K * SWEEP_TIERS;
  if (!plan->chunk_lists[k0].empty())
    hipLaunchKernelGGL((apply_kernel<D, K, P, TV>), dim3((unsigned)plan->chunk_lists[k0].size(), (unsigned)nrhs),
                       dim3(CHUNK), 0, s, plan->dev, plan->dev_chunk_lists[k0], (const typename P::X*)x,
                       (typename P::Y*)y, xs, ys, da);
  if (!plan->chunk_lists[k0 + 1].empty()) launch_staged<D, K, P, false, TV>(plan, k0 + 1, nrhs, x, y, xs, ys, da, s);
  if (!plan->chunk_lists[k0 + 2].empty()) launch_staged<D, K, P, true, TV>(plan, k0 + 2, nrhs, x, y, xs, ys, da, s);
}

template <int D, class P, class TV>
static void launch_apply_d(const sgdg_plan* plan, int nrhs, const void* x, void* y, int64_t xs, int64_t ys,
                           const DotArgs& da, hipStream_t s) {
  launch_kind<D, 1, P, TV>(plan, nrhs, x, y, xs, ys, da, s);
  launch_kind<D, 2, P, TV>(plan, nrhs, x, y, xs, ys, da, s);
  launch_kind<D, 3, P, TV>(plan, nrhs, x, y, xs, ys, da, s);
}

template <class P, class TV>
static void launch_any(const sgdg_plan* plan, int nrhs, const void* x, void* y, int64_t xs, int64_t ys,
                       const DotArgs& da, hipStream_t s) {
  switch (plan->d) {
    case 1: launch_apply_d<1, P, TV>(plan, nrhs, x, y, xs, ys, da, s); break;
    case 2: launch_apply_d<2, P, TV>(plan, nrhs, x, y, xs, ys, da, s); break;
    case 3: launch_apply_d<3, P, TV>(plan, nrhs, x, y, xs, ys, da, s); break;
    case 4: launch_apply_d<4, P, TV>(plan, nrhs, x, y, xs, ys, da, s); break;
    case 5: launch_apply_d<5, P, TV>(plan, nrhs, x, y, xs, ys, da, s); break;
    case 6: launch_apply_d<6, P, TV>(plan, nrhs, x, y, xs, ys, da, s); break;
  }
}

template <class P>
void launch_apply(const sgdg_plan* plan, int nrhs, const void* x, void* y, int64_t xs, int64_t ys, hipStream_t s) {
  if constexpr (std::is_same_v<P, PrecF64>)
    if (plan->fibre_on) {
      launch_fibre(plan, nrhs, (const double*)x, (double*)y, xs, ys, s);
      return;
    }
  launch_any<P, void>(plan, nrhs, x, y, xs, ys, DotArgs{}, s);
}

template <class P, class TV>
void launch_apply_dots(const sgdg_plan* plan, int nrhs, const void* x, void* y, const DotArgs& da, hipStream_t s) {
  launch_any<P, TV>(plan, nrhs, x, y, plan->total, plan->total, da, s);
}

template void launch_apply<PrecF64>(const sgdg_plan*, int, const void*, void*, int64_t, int64_t, hipStream_t);
template void launch_apply<PrecF32>(const sgdg_plan*, int, const void*, void*, int64_t, int64_t, hipStream_t);
template void launch_apply<PrecBF16>(const sgdg_plan*, int, const void*, void*, int64_t, int64_t, hipStream_t);
template void launch_apply_dots<PrecF64, double>(const sgdg_plan*, int, const void*, void*, const DotArgs&, hipStream_t);
template void launch_apply_dots<PrecF32, float>(const sgdg_plan*, int, const void*, void*, const DotArgs&, hipStream_t);
template void launch_apply_dots<PrecBF16, float>(const sgdg_plan*, int, const void*, void*, const DotArgs&, hipStream_t);

}  // namespace sgdg

using namespace sgdg;

extern "C" sgdg_status sg_dg_apply(const sgdg_plan* plan, int32_t nrhs, const void* x, void* y, void* stream) {
  if (!plan) return fail(SGDG_ERR_ARG, "sg_dg_apply: null plan");
  if (nrhs < 1 || nrhs > 65535) return fail(SGDG_ERR_ARG, "sg_dg_apply: nrhs must be in 1..65535");
  if (!x || !y) return fail(SGDG_ERR_ARG, "sg_dg_apply: null vector");
  if (x == y) return fail(SGDG_ERR_ARG, "sg_dg_apply: x and y must not alias");
  hipStream_t s = (hipStream_t)stream;
  switch (plan->prec) {
    case SGDG_FP64: launch_apply<PrecF64>(plan, nrhs, x, y, plan->total, plan->total, s); break;
    case SGDG_FP32_SWEEP: launch_apply<PrecF32>(plan, nrhs, x, y, plan->total, plan->total, s); break;
    default: launch_apply<PrecBF16>(plan, nrhs, x, y, plan->total, plan->total, s); break;
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "sg_dg_apply launch");
  return SGDG_OK;
}
