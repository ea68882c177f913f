// Persistent Arnoldi process (Sec. 3, eq. 3.7) for small problems.
//
// The multi-kernel form in krylov.hip pays a kernel boundary per reduction
// and re-stages the operator tables into LDS for every sweep.  When every
// chunk of the plan belongs to one LDS-staged sweep list and the grid (chunks
// x right-hand sides) fits the device at one workgroup per compute unit, all M
// steps can instead run in one cooperative launch (opt-in, see
// arnoldi_persistent): each
// workgroup owns one chunk, stages its problem's level table, row tables and
// block values once, and per step
//   A  stages x = v_j of its species segment,
//   B  sweeps its chunk (w = A v_j) and writes the chunk partials <v_i, w>,
//   -- grid barrier --
//   C  h1 = <V, w> (fixed-order reduction), w1 = w - V h1, partials <v_i, w1>
//      and |w1|^2,
//   -- grid barrier --
//   D  h2, |w2|^2 = |w1|^2 - |h2|^2, breakdown test, v_{j+1} = w2 / |w2|,
//   -- grid barrier --
// exactly the arithmetic of the multi-kernel form (classical Gram-Schmidt
// applied twice, FP64 reductions in a fixed order), so every workgroup of a
// problem takes the same breakdown decision.  w and w1 of a chunk stay in LDS.
//
// Coherence without cache flushes.  The eight XCDs of the chip have separate
// L2 caches, so data one workgroup writes for another (chunk partials, the
// basis vector v_{j+1}) is written and read with device-scope atomic stores
// and loads, which are coherent across XCDs; everything a workgroup reads
// only from its own chunk (earlier basis vectors) is read through the caches
// and stays resident across steps.  The grid barrier therefore needs no L2
// write-back or invalidate: each wave waits for its own stores to complete,
// the workgroup meets at s_barrier, one thread arrives on a counter and
// waits for the generation word to move (bounded wait: past the limit it
// raises the error word, every workgroup leaves, and k_expm reports
// SGDG_ERR_HIP).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cstdlib>
#include <cstring>
#include <type_traits>

#include "internal.h"
#include "kernels.h"
#include "krylov.h"

namespace sgdg {

constexpr int PA_THREADS = CHUNK * APPLY_G;
constexpr int PA_OVERLAY = (2 * CHUNK + 64 + PA_THREADS) * 8;  // wl, w1l, h, red (bytes)
constexpr int PA_SPIN_LIMIT = 1 << 24;
// dynamic LDS limit of the persistent kernel (its barrier flag takes a little static LDS)
constexpr int PA_LDS_MAX = APPLY_LDS_BYTES - 64;

struct GridBar {
  uint32_t* w;  // [0] arrivals, [1] generation, [2] error
  uint32_t nb;
};

__device__ __forceinline__ bool grid_sync(const GridBar& gb) {
  __shared__ int ok_s;
  __builtin_amdgcn_s_waitcnt(0);  // this wave's (coherent) stores have completed
  __syncthreads();
  if (threadIdx.x == 0) {
    const uint32_t g = __hip_atomic_load(gb.w + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const uint32_t a = __hip_atomic_fetch_add(gb.w, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (a == gb.nb - 1) {
      __hip_atomic_store(gb.w, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __builtin_amdgcn_s_waitcnt(0);
      __hip_atomic_store(gb.w + 1, g + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    } else {
      int spins = 0;
      while (__hip_atomic_load(gb.w + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == g) {
        if (++spins > PA_SPIN_LIMIT || __hip_atomic_load(gb.w + 2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
          __hip_atomic_store(gb.w + 2, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          break;
        }
        __builtin_amdgcn_s_sleep(1);
      }
    }
    ok_s = __hip_atomic_load(gb.w + 2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0u;
  }
  __syncthreads();
  return ok_s != 0;  // one decision for the whole workgroup
}

// device-scope (cross-XCD coherent) access to data shared between workgroups
template <class T>
__device__ __forceinline__ T ld_shared(const T* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <class T>
__device__ __forceinline__ void st_shared(T* p, T v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// h[i] = sum over the problem's nc chunks of part[row0 + q][i], i < cols, in a
// fixed order (slices of the workgroup, then slices in index order)
__device__ __forceinline__ void pa_reduce(const double* __restrict__ part, int64_t row0, int nc, int ld, int cols,
                                          double* red, double* h) {
  const int tid = threadIdx.x;
  const int S = PA_THREADS / cols;
  if (tid < cols * S) {
    const int i = tid / S, sl = tid - i * S;
    double acc = 0.0;
    for (int q = sl; q < nc; q += S) acc += ld_shared(part + (row0 + q) * ld + i);
    red[tid] = acc;
  }
  __syncthreads();
  if (tid < cols) {
    double t = 0.0;
    for (int q = 0; q < S; ++q) t += red[tid * S + q];
    h[tid] = t;
  }
  __syncthreads();
}

// chunk partials out[i] = sum_e V_i[e] * u[e] (i < nv) and, with norm,
// out[nv] = sum_e u[e]^2; wave w takes vectors w, w + 16, ...
template <class TV>
__device__ __forceinline__ void pa_dots(const KrylovWs& ws, int nv, bool norm, int nrhs, int rhs, int64_t total,
                                        const Chunk& ch, const double* u, double* out) {
  const int wv = threadIdx.x >> 6, ln = threadIdx.x & 63, nw = blockDim.x >> 6;
  const int cols = nv + (norm ? 1 : 0);
  for (int i = wv; i < cols; i += nw) {
    double s = 0.0;
    if (i < nv) {
      const TV* v = (const TV*)ws.V + ((int64_t)i * nrhs + rhs) * total + ch.start;
      if (i == 0)  // written by an earlier kernel: read it coherently
        for (int q = ln; q < ch.count; q += 64) s += (double)ld_shared(v + q) * u[q];
      else  // written by this workgroup in this launch
        for (int q = ln; q < ch.count; q += 64) s += (double)v[q] * u[q];
    } else {
      for (int q = ln; q < ch.count; q += 64) s += u[q] * u[q];
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    if (ln == 0) st_shared(out + i, s);
  }
}

template <int D, int K, class P, bool SV, class TV>
__global__ __launch_bounds__(PA_THREADS) void k_arnoldi(DevTables T, const int32_t* __restrict__ list, int M,
                                                        KrylovWs ws, int nchunks, int ninst, int64_t total,
                                                        int xregion, GridBar gb) {
  using V = typename P::V;
  using X = typename P::X;
  extern __shared__ __align__(16) unsigned char smem[];
  const int cid = list[blockIdx.x];
  const int rhs = blockIdx.y, nrhs = gridDim.y;
  const int tid = threadIdx.x;
  const Chunk ch = T.chunks[cid];
  const InstDev& I = T.inst[ch.inst];
  const int p = (rhs * ninst + ch.inst) * 2 + ch.species;
  const int c0 = ch.pc0, nc = ch.pnc;
  const int64_t seg = I.offset + (int64_t)ch.species * I.ndof;
  const int Mp = (int)min((int64_t)M, I.ndof);
  const double brk = KRYLOV_BREAKDOWN_REL * I.anorm[ch.species];

  // ---- one-time staging: level-block table, row tables, block values
  int ntab = 1;
  for (int m = 0; m < D; ++m) ntab *= (I.N + 1);
  int32_t* bst = (int32_t*)smem;
  for (int i = tid; i < ntab; i += PA_THREADS) {
    const int b = T.blkid[I.blkid_off + i];
    bst[i] = b >= 0 ? (int32_t)T.lstart[b] : -1;
  }
  RowsLds rows;
  ValsLds<P> vl;
  unsigned dup = 0;
  int32_t* rp = bst + ntab;
#pragma unroll
  for (int i = 0; i < D; ++i) {
    const BCsr bc = T.bcsr[I.bcsr_off[i]];
#pragma unroll
    for (int i2 = 0; i2 < i; ++i2)
      if (!((dup >> i) & 1u) && T.bcsr[I.bcsr_off[i2]].cptr_off == bc.cptr_off) {
        rows.cptr[i] = rows.cptr[i2];
        rows.src[i] = rows.src[i2];
        rows.tlo[i] = 0;
        rows.elo[i] = 0;
        dup |= 1u << i;
      }
    if ((dup >> i) & 1u) continue;
    rows.tlo[i] = 0;  // whole tables
    rows.elo[i] = 0;
    rows.cptr[i] = rp;
    for (int t = tid; t <= bc.ncell; t += PA_THREADS) rp[t] = T.cptr[bc.cptr_off + t];
    rp += bc.ncell + 1;
    rows.src[i] = rp;
    for (int t = tid; t < bc.nnzb; t += PA_THREADS) rp[t] = T.src[bc.src_off + t];
    rp += bc.nnzb;
  }
  unsigned char* cur = smem + ((((unsigned char*)rp - smem) + 15) & ~15);
  X* xl = (X*)cur;
  // overlay of the x region, live between the end of a sweep and the next staging
  double* wl = (double*)cur;
  double* w1l = wl + CHUNK;
  double* hs = w1l + CHUNK;
  double* red = hs + 64;
  cur += xregion;
  if constexpr (SV) {
    const V* __restrict__ vals = P::vals(T);
#pragma unroll
    for (int i = 0; i < D; ++i) {
      const BCsr bc = T.bcsr[I.bcsr_off[i]];
#pragma unroll
      for (int i2 = 0; i2 < i; ++i2)
        if (T.bcsr[I.bcsr_off[i2]].cptr_off == bc.cptr_off) vl.v[i] = vl.v[i2];
      if ((dup >> i) & 1u) continue;
      V* dst = (V*)cur;
      const int64_t nv = (int64_t)bc.nnzb * (K + 1) * (K + 1);
      for (int64_t t = tid; t < nv; t += PA_THREADS) dst[t] = vals[bc.val_off + t];
      vl.v[i] = dst;
      cur += (nv * (int64_t)sizeof(V) + 15) & ~15;
    }
  }
  const int G = ch.g;  // lanes per output (more for the heavy rows of coarse levels)
  const int e = tid / G, lane = tid - e * G;
  const bool active = e < ch.count;
  const int64_t g = ch.start + e;
  const GBlock* Bp = active ? &T.gblk[find_block(T, ch, g)] : nullptr;
  bool finished = ws.done[p] != 0;  // v = 0 (set by k_norm)
  const int64_t ldp = M + 2;
  double* part1 = ws.part1 + ((int64_t)rhs * nchunks + cid) * ldp;
  double* part2 = ws.part2 + ((int64_t)rhs * nchunks + cid) * ldp;
  const int64_t prow0 = (int64_t)rhs * nchunks + c0;
  double* Hp = ws.H + (int64_t)p * (M + 1) * M;

  for (int j = 0; j < M; ++j) {
    // ---- A + B: stage v_j, sweep the chunk, partials <v_i, w>
    if (!finished) {
      // v_j of the whole species segment (other chunks written by other workgroups)
      const TV* vg = (const TV*)ws.V + ((int64_t)j * nrhs + rhs) * total + seg;
      __syncthreads();  // the overlay of the previous step is dead
      for (int64_t i = tid; i < I.ndof; i += PA_THREADS) {
        const TV v = ld_shared(vg + i);
        if constexpr (std::is_same_v<X, uint16_t>)
          xl[i] = f_to_bf16((float)v);
        else
          xl[i] = (X)v;
      }
      __syncthreads();
      typename P::A acc = 0;
      if (active) {
        SrcLds<P> xs{xl, bst};
        if constexpr (SV)
          acc = apply_one<D, K, P>(T, *Bp, I, g, lane, G, xs, rows, vl);
        else
          acc = apply_one<D, K, P>(T, *Bp, I, g, lane, G, xs, rows, ValsGlobal<P>{P::vals(T)});
      }
      for (int o = 1; o < G; o <<= 1) acc += __shfl_xor(acc, o, 64);
      __syncthreads();  // x is dead: the overlay takes its place
      if (tid < CHUNK) wl[tid] = 0.0;
      __syncthreads();
      if (active && lane == 0) wl[e] = (double)(typename P::Y)acc;
      __syncthreads();
      pa_dots<TV>(ws, j + 1, false, nrhs, rhs, total, ch, wl, part1);
    }
    if (!grid_sync(gb)) return;
    // ---- C: h1, w1 = w - V h1, partials <v_i, w1>, |w1|^2
    if (!finished) {
      pa_reduce(ws.part1, prow0, nc, (int)ldp, j + 1, red, hs);
      if (cid == c0 && tid <= j) Hp[tid * M + j] = hs[tid];
      if (tid < CHUNK) {
        double a = 0.0;
        if (tid < ch.count) {
          a = wl[tid];
          const int64_t gg = ch.start + tid;
          a -= hs[0] * (double)ld_shared((const TV*)ws.V + (int64_t)rhs * total + gg);
          for (int i = 1; i <= j; ++i) a -= hs[i] * (double)((const TV*)ws.V)[((int64_t)i * nrhs + rhs) * total + gg];
        }
        w1l[tid] = a;
      }
      __syncthreads();
      pa_dots<TV>(ws, j + 1, true, nrhs, rhs, total, ch, w1l, part2);
    }
    if (!grid_sync(gb)) return;
    // ---- D: h2, |w2|, breakdown test, v_{j+1}
    if (!finished) {
      pa_reduce(ws.part2, prow0, nc, (int)ldp, j + 2, red, hs);
      double n2 = hs[j + 1];
      for (int i = 0; i <= j; ++i) n2 -= hs[i] * hs[i];
      const double hn = sqrt(fmax(n2, 0.0));
      if (cid == c0 && tid <= j) Hp[tid * M + j] += hs[tid];
      if (cid == c0 && tid == 0) Hp[(j + 1) * M + j] = hn;
      const bool stop = !(hn > brk) || (j + 1 >= Mp);
      if (stop) {
        if (cid == c0 && tid == 0) {
          ws.m[p] = j + 1;
          ws.done[p] = 1;
        }
        finished = true;
      } else if (tid < ch.count) {
        const int64_t gg = ch.start + tid;
        double a = w1l[tid] - hs[0] * (double)ld_shared((const TV*)ws.V + (int64_t)rhs * total + gg);
        for (int i = 1; i <= j; ++i) a -= hs[i] * (double)((const TV*)ws.V)[((int64_t)i * nrhs + rhs) * total + gg];
        const double x = a / hn;
        st_shared((TV*)ws.V + ((int64_t)(j + 1) * nrhs + rhs) * total + gg, (TV)x);
      }
    }
    if (!grid_sync(gb)) return;
  }
}

static int device_cus() {
  static std::atomic<int> cus{0};
  int c = cus.load();
  if (c == 0) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
      c = 0;
    cus.store(c > 0 ? c : -1);
  }
  return c > 0 ? c : 0;
}

template <int D, int K, class P, bool SV, class TV>
static bool launch_pa(const sgdg_plan* plan, int kind, int nrhs, int M, const KrylovWs& ws, int lds, int xregion,
                      hipStream_t s) {
  static std::atomic<int> attr_set{0};
  if (attr_set.load() == 0) {
    if (hipFuncSetAttribute((const void*)k_arnoldi<D, K, P, SV, TV>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            PA_LDS_MAX) != hipSuccess) {
      (void)hipGetLastError();
      return false;
    }
    attr_set.store(1);
  }
  DevTables T = plan->dev;
  const int32_t* list = plan->dev_chunk_lists[kind];
  int Mv = M, nch = plan->nchunks, ninst = plan->ninst;
  int64_t total = plan->total;
  KrylovWs w = ws;
  GridBar gb{ws.bar, (uint32_t)(plan->chunk_lists[kind].size() * (size_t)nrhs)};
  void* args[] = {&T, &list, &Mv, &w, &nch, &ninst, &total, &xregion, &gb};
  const hipError_t e = hipLaunchCooperativeKernel((const void*)k_arnoldi<D, K, P, SV, TV>,
                                                  dim3((unsigned)plan->chunk_lists[kind].size(), (unsigned)nrhs),
                                                  dim3(PA_THREADS), args, (unsigned)lds, s);
  if (e != hipSuccess) {
    (void)hipGetLastError();  // clear: the caller falls back to the multi-kernel form
    return false;
  }
  return true;
}

template <int D, class P, class TV>
static bool pa_dispatch_k(const sgdg_plan* plan, int k, bool sv, int kind, int nrhs, int M, const KrylovWs& ws,
                          int lds, int xregion, hipStream_t s) {
  switch (k * 2 + (sv ? 1 : 0)) {
    case 2: return launch_pa<D, 1, P, false, TV>(plan, kind, nrhs, M, ws, lds, xregion, s);
    case 3: return launch_pa<D, 1, P, true, TV>(plan, kind, nrhs, M, ws, lds, xregion, s);
    case 4: return launch_pa<D, 2, P, false, TV>(plan, kind, nrhs, M, ws, lds, xregion, s);
    case 5: return launch_pa<D, 2, P, true, TV>(plan, kind, nrhs, M, ws, lds, xregion, s);
    case 6: return launch_pa<D, 3, P, false, TV>(plan, kind, nrhs, M, ws, lds, xregion, s);
    case 7: return launch_pa<D, 3, P, true, TV>(plan, kind, nrhs, M, ws, lds, xregion, s);
  }
  return false;
}

template <class P, class TV>
static bool pa_dispatch(const sgdg_plan* plan, int k, bool sv, int kind, int nrhs, int M, const KrylovWs& ws,
                        int lds, int xregion, hipStream_t s) {
  switch (plan->d) {
    case 1: return pa_dispatch_k<1, P, TV>(plan, k, sv, kind, nrhs, M, ws, lds, xregion, s);
    case 2: return pa_dispatch_k<2, P, TV>(plan, k, sv, kind, nrhs, M, ws, lds, xregion, s);
    case 3: return pa_dispatch_k<3, P, TV>(plan, k, sv, kind, nrhs, M, ws, lds, xregion, s);
    case 4: return pa_dispatch_k<4, P, TV>(plan, k, sv, kind, nrhs, M, ws, lds, xregion, s);
  }
  return false;
}

bool arnoldi_persistent(const sgdg_plan* plan, int nrhs, int M, const KrylovWs& ws, hipStream_t s) {
  // opt-in (SGDG_ARNOLDI=persistent): measured on MI355X for the 2 x 5184-DOF
  // Schnakenberg plan it takes 27 us per Arnoldi step against 25 us for the
  // launch-per-pass form -- three grid barriers (about 2.8 us each after the
  // last arrival) cost as much as three graph-launched kernel boundaries
  const char* env = std::getenv("SGDG_ARNOLDI");
  if (!env || std::strcmp(env, "persistent") != 0) return false;
  if (plan->d > 4) return false;
  // every chunk in one staged list
  int kind = -1;
  for (size_t kd = 0; kd < plan->chunk_lists.size(); ++kd)
    if ((int)plan->chunk_lists[kd].size() == plan->nchunks) kind = (int)kd;
  if (kind < 0 || kind % SWEEP_TIERS == 0) return false;
  const int k = kind / SWEEP_TIERS;
  const bool sv = kind % SWEEP_TIERS == 2;
  const int64_t grid = (int64_t)plan->nchunks * nrhs;
  const int cus = device_cus();
  if (cus == 0 || grid > cus) return false;
  // LDS: the staged sweep layout with the x region widened to hold the overlay
  const int xbytes = plan->prec == SGDG_FP64 ? 8 : (plan->prec == SGDG_FP32_SWEEP ? 4 : 2);
  int64_t max_x = 0;
  for (const HostInstance& hi : plan->inst) max_x = std::max<int64_t>(max_x, hi.ndof * xbytes);
  const int xregion = (int)((std::max<int64_t>(max_x, PA_OVERLAY) + 15) & ~(int64_t)15);
  const int lds = plan->list_fixed[kind] + xregion;
  if (lds > PA_LDS_MAX) return false;
  switch (plan->prec) {
    case SGDG_FP64: return pa_dispatch<PrecF64, double>(plan, k, sv, kind, nrhs, M, ws, lds, xregion, s);
    case SGDG_FP32_SWEEP: return pa_dispatch<PrecF32, float>(plan, k, sv, kind, nrhs, M, ws, lds, xregion, s);
    default: return pa_dispatch<PrecBF16, float>(plan, k, sv, kind, nrhs, M, ws, lds, xregion, s);
  }
}

}  // namespace sgdg
