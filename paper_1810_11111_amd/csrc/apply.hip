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
#include <hip/hip_runtime.h>

#include "internal.h"
#include "kernels.h"

namespace sgdg {

template <int D, int K, class P>
__global__ __launch_bounds__(CHUNK) void apply_kernel(DevTables T, const int32_t* __restrict__ list, int64_t total,
                                                      const typename P::X* __restrict__ x, typename P::Y* __restrict__ y,
                                                      int64_t xstride, int64_t ystride) {
  const Chunk ch = T.chunks[list[blockIdx.x]];
  const int tid = threadIdx.x;
  if (tid >= ch.count) return;
  const int64_t g = ch.start + tid;
  const int64_t rhs = blockIdx.y;
  const typename P::X* xr = x + rhs * xstride;
  typename P::Y* yr = y + rhs * ystride;
  const typename P::A acc = apply_one<D, K, P>(T, ch, g, xr);
  yr[g] = (typename P::Y)acc;
}

template <int D, int K, class P>
static void launch_apply_dk(const sgdg_plan* plan, int nrhs, const void* x, void* y, int64_t xs, int64_t ys,
                            hipStream_t s) {
  const auto& list = plan->chunks_by_k[K];
  if (list.empty()) return;
  dim3 grid((unsigned)list.size(), (unsigned)nrhs);
  hipLaunchKernelGGL((apply_kernel<D, K, P>), grid, dim3(CHUNK), 0, s, plan->dev, plan->dev_chunk_lists[K], plan->total,
                     (const typename P::X*)x, (typename P::Y*)y, xs, ys);
}

template <int D, class P>
static void launch_apply_d(const sgdg_plan* plan, int nrhs, const void* x, void* y, int64_t xs, int64_t ys,
                           hipStream_t s) {
  launch_apply_dk<D, 1, P>(plan, nrhs, x, y, xs, ys, s);
  launch_apply_dk<D, 2, P>(plan, nrhs, x, y, xs, ys, s);
  launch_apply_dk<D, 3, P>(plan, nrhs, x, y, xs, ys, s);
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
