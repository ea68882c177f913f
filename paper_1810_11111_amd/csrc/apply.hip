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
// Two variants: when a species segment (and its level-block table) fits in
// LDS, every workgroup first stages the whole segment there and gathers from
// LDS (small problems are latency bound: the gathers then cost LDS latency,
// not L2 latency); otherwise the gathers read global memory.
#include <hip/hip_runtime.h>

#include <atomic>

#include "internal.h"
#include "kernels.h"

namespace sgdg {

template <int D, int K, class P>
__global__ __launch_bounds__(CHUNK) void apply_kernel(DevTables T, const int32_t* __restrict__ list,
                                                      const typename P::X* __restrict__ x, typename P::Y* __restrict__ y,
                                                      int64_t xstride, int64_t ystride) {
  const Chunk ch = T.chunks[list[blockIdx.x]];
  const int tid = threadIdx.x;
  if (tid >= ch.count) return;
  const int64_t g = ch.start + tid;
  const int64_t rhs = blockIdx.y;
  const GBlock& B = T.gblk[find_block(T, ch, g)];
  const InstDev& I = T.inst[B.inst];
  SrcGlobal<P> xs{x + rhs * xstride, T.blkid + I.blkid_off, T.lstart, I.offset + (int64_t)B.species * I.ndof};
  RowsGlobal rows{T.cptr, T.src};
  y[rhs * ystride + g] = (typename P::Y)apply_one<D, K, P>(T, B, I, g, xs, rows);
}

// Staged variant: one 64-lane workgroup per quarter chunk, so a small problem
// spreads over four times as many compute units (the gathers are bound by
// per-CU load throughput, not by the staging copy).
constexpr int SUB = 4;

template <int D, int K, class P>
__global__ __launch_bounds__(CHUNK / SUB) void apply_kernel_lds(DevTables T, const int32_t* __restrict__ list,
                                                                const typename P::X* __restrict__ x,
                                                                typename P::Y* __restrict__ y, int64_t xstride,
                                                                int64_t ystride) {
  extern __shared__ __align__(16) unsigned char smem[];
  const Chunk ch = T.chunks[list[blockIdx.x / SUB]];
  const int sub = blockIdx.x % SUB;
  const int tid = threadIdx.x;
  const int64_t rhs = blockIdx.y;
  const InstDev& I = T.inst[ch.inst];
  const int64_t seg = I.offset + (int64_t)ch.species * I.ndof;
  int ntab = 1;
  for (int m = 0; m < D; ++m) ntab *= (I.N + 1);
  int32_t* bst = (int32_t*)smem;
  for (int i = tid; i < ntab; i += blockDim.x) {
    const int b = T.blkid[I.blkid_off + i];
    bst[i] = b >= 0 ? (int32_t)T.lstart[b] : -1;
  }
  // row pointers and source cells of each distinct 1D operator of the instance
  RowsLds rows;
  int32_t* rp = bst + ntab;
  for (int i = 0; i < D; ++i) {
    const BCsr bc = T.bcsr[I.bcsr_off[i]];
    int same = -1;
    for (int i2 = 0; i2 < i; ++i2)
      if (T.bcsr[I.bcsr_off[i2]].cptr_off == bc.cptr_off) same = i2;
    if (same >= 0) {
      rows.cptr[i] = rows.cptr[same];
      rows.src[i] = rows.src[same];
      continue;
    }
    rows.cptr[i] = rp;
    for (int t = tid; t <= bc.ncell; t += blockDim.x) rp[t] = T.cptr[bc.cptr_off + t];
    rp += bc.ncell + 1;
    rows.src[i] = rp;
    for (int t = tid; t < bc.nnzb; t += blockDim.x) rp[t] = T.src[bc.src_off + t];
    rp += bc.nnzb;
  }
  typename P::X* xl = (typename P::X*)(smem + ((((unsigned char*)rp - smem) + 15) & ~15));
  const typename P::X* __restrict__ xg = x + rhs * xstride + seg;
  for (int64_t i = tid; i < I.ndof; i += blockDim.x) xl[i] = xg[i];
  __syncthreads();
  const int e = sub * (CHUNK / SUB) + tid;
  if (e >= ch.count) return;
  const int64_t g = ch.start + e;
  const GBlock& B = T.gblk[find_block(T, ch, g)];
  SrcLds<P> xs{xl, bst};
  y[rhs * ystride + g] = (typename P::Y)apply_one<D, K, P>(T, B, I, g, xs, rows);
}

template <int D, int K, class P>
static void launch_kind(const sgdg_plan* plan, int nrhs, const void* x, void* y, int64_t xs, int64_t ys,
                        hipStream_t s) {
  const int kg = K * 2 + 0, ks = K * 2 + 1;
  if (!plan->chunk_lists[kg].empty())
    hipLaunchKernelGGL((apply_kernel<D, K, P>), dim3((unsigned)plan->chunk_lists[kg].size(), (unsigned)nrhs),
                       dim3(CHUNK), 0, s, plan->dev, plan->dev_chunk_lists[kg], (const typename P::X*)x,
                       (typename P::Y*)y, xs, ys);
  if (!plan->chunk_lists[ks].empty()) {
    const int lds = plan->list_lds[ks];
    static std::atomic<int> attr_set{0};
    if (attr_set.load() < lds) {
      hipFuncSetAttribute((const void*)apply_kernel_lds<D, K, P>, hipFuncAttributeMaxDynamicSharedMemorySize,
                          APPLY_LDS_BYTES);
      attr_set.store(APPLY_LDS_BYTES);
    }
    hipLaunchKernelGGL((apply_kernel_lds<D, K, P>),
                       dim3((unsigned)plan->chunk_lists[ks].size() * SUB, (unsigned)nrhs), dim3(CHUNK / SUB), lds, s,
                       plan->dev, plan->dev_chunk_lists[ks], (const typename P::X*)x, (typename P::Y*)y, xs, ys);
  }
}

template <int D, class P>
static void launch_apply_d(const sgdg_plan* plan, int nrhs, const void* x, void* y, int64_t xs, int64_t ys,
                           hipStream_t s) {
  launch_kind<D, 1, P>(plan, nrhs, x, y, xs, ys, s);
  launch_kind<D, 2, P>(plan, nrhs, x, y, xs, ys, s);
  launch_kind<D, 3, P>(plan, nrhs, x, y, xs, ys, s);
}

template <class P>
void launch_apply(const sgdg_plan* plan, int nrhs, const void* x, void* y, int64_t xs, int64_t ys, hipStream_t s) {
  switch (plan->d) {
    case 1: launch_apply_d<1, P>(plan, nrhs, x, y, xs, ys, s); break;
    case 2: launch_apply_d<2, P>(plan, nrhs, x, y, xs, ys, s); break;
    case 3: launch_apply_d<3, P>(plan, nrhs, x, y, xs, ys, s); break;
    case 4: launch_apply_d<4, P>(plan, nrhs, x, y, xs, ys, s); break;
    case 5: launch_apply_d<5, P>(plan, nrhs, x, y, xs, ys, s); break;
    case 6: launch_apply_d<6, P>(plan, nrhs, x, y, xs, ys, s); break;
  }
}

template void launch_apply<PrecF64>(const sgdg_plan*, int, const void*, void*, int64_t, int64_t, hipStream_t);
template void launch_apply<PrecF32>(const sgdg_plan*, int, const void*, void*, int64_t, int64_t, hipStream_t);
template void launch_apply<PrecBF16>(const sgdg_plan*, int, const void*, void*, int64_t, int64_t, hipStream_t);

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
