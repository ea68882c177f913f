// IIF2 and IIF3 time steps (Sec. 3, eqs. 3.5 and 3.6) with the implicit
// reaction stage, and the explicit SSP Runge-Kutta comparators of Sec. 4.
//
//   v = U^n + dt/2 F(U^n);  W = exp(A dt) v  (one Krylov problem per species);
//   solve  U - dt/2 F(U) = W  by the pointwise quasi-Newton iteration
//     U <- U - P[(I_s - dt/2 J_f(u_q))^{-1} (R G)_q],  G = U - dt/2 F(U) - W,
//   from U = W + dt/2 F(U^n), until ||G||_2 <= tol max(1, ||W||_2) per instance.
//
// The paper solves the stage with Newton's method (Sec. 4, Example 3; Sec. 5:
// the sparse basis couples every unknown); the pointwise iteration has the
// same root.  Control stays on the device: a check kernel sets a per-instance
// convergence flag that every later kernel of the step reads, so a step is a
// fixed launch sequence (newton_max + 1 residual passes) that can be captured
// in a graph; converged instances skip their work.
//
// IIF3 (eq. 3.6, coefficients of eq. 3.4: 5/12, 2/3, -1/12):
//   W = exp(A dt)(U^n + 2/3 dt F^n) + exp(2 A dt)(-1/12 dt F^{n-1}),
//   solve U - 5/12 dt F(U) = W the same way from U = W + 5/12 dt F^n.
#include <hip/hip_runtime.h>

#include <array>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <tuple>
#include <functional>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "internal.h"
#include "kernels.h"
#include "krylov.h"
#include "reaction.h"

namespace sgdg {

static size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

struct IifWs {
  KrylovWs kws;
  double* rws;
  double *v, *W, *G, *F, *W2;
  double *part, *partw, *wnorm;
  int32_t* conv;
};

size_t iif2_ws_bytes(const sgdg_plan* plan, int M, int nrhs) {
  const size_t tot = (size_t)plan->total * nrhs;
  size_t b = al256(krylov_ws_bytes(plan, M, nrhs));
  b += al256((size_t)reaction_ws_doubles(plan) * nrhs * 8);
  b += 5 * al256(tot * 8);
  b += al256((size_t)nrhs * reaction_final_fibres(plan) * 8);
  b += al256((size_t)nrhs * plan->nchunks * 8);
  b += al256((size_t)nrhs * plan->ninst * 8);
  b += al256(((size_t)nrhs * plan->ninst + 1) * 4);
  return b;
}

static IifWs carve(const sgdg_plan* plan, int M, int nrhs, void* base) {
  const size_t tot = (size_t)plan->total * nrhs;
  char* p = (char*)base;
  auto take = [&](size_t bytes) {
    char* r = p;
    p += al256(bytes);
    return (void*)r;
  };
  IifWs w{};
  void* kb = take(krylov_ws_bytes(plan, M, nrhs));
  w.kws = krylov_carve(plan, M, nrhs, kb);
  w.rws = (double*)take((size_t)reaction_ws_doubles(plan) * nrhs * 8);
  w.v = (double*)take(tot * 8);
  w.W = (double*)take(tot * 8);
  w.G = (double*)take(tot * 8);
  w.F = (double*)take(tot * 8);
  w.W2 = (double*)take(tot * 8);
  w.part = (double*)take((size_t)nrhs * reaction_final_fibres(plan) * 8);
  w.partw = (double*)take((size_t)nrhs * plan->nchunks * 8);
  w.wnorm = (double*)take((size_t)nrhs * plan->ninst * 8);
  w.conv = (int32_t*)take(((size_t)nrhs * plan->ninst + 1) * 4);  // flags, then their count
  return w;
}

// out = x + a y
__global__ __launch_bounds__(256) void k_axpy(double* __restrict__ out, const double* __restrict__ x, double a,
                                              const double* __restrict__ y, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = x[i] + a * y[i];
}

// out = a x + b y + c z
__global__ __launch_bounds__(256) void k_lin3(double* __restrict__ out, double a, const double* __restrict__ x, double b,
                                              const double* __restrict__ y, double c, const double* __restrict__ z,
                                              int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = a * x[i] + b * y[i] + c * z[i];
}

// out = y
__global__ __launch_bounds__(256) void k_copy(double* __restrict__ out, const double* __restrict__ y, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = y[i];
}

// U = W + dt2 F, per-chunk ||W||^2, reset of the convergence flags
__global__ __launch_bounds__(CHUNK) void k_stage_init(DevTables T, int ninst, int nchunks, int64_t total, double dt2,
                                                      double* __restrict__ U, const double* __restrict__ W,
                                                      const double* __restrict__ F, double* __restrict__ partw,
                                                      int32_t* __restrict__ conv) {
  const int c = blockIdx.x, rhs = blockIdx.y, tid = threadIdx.x;
  const Chunk ch = T.chunks[c];
  double w2 = 0.0;
  if (tid < ch.count) {
    const int64_t gi = (int64_t)rhs * total + ch.start + tid;
    const double w = W[gi];
    U[gi] = w + dt2 * F[gi];
    w2 = w * w;
  }
  for (int off = 32; off > 0; off >>= 1) w2 += __shfl_xor(w2, off, 64);
  __shared__ double red[CHUNK / 64];
  if ((tid & 63) == 0) red[tid >> 6] = w2;
  __syncthreads();
  if (tid == 0) {
    double t = 0.0;
    for (int w = 0; w < CHUNK / 64; ++w) t += red[w];
    partw[(int64_t)rhs * nchunks + c] = t;
    if (c == T.pchunk0[ch.inst * 2] ) conv[rhs * ninst + ch.inst] = 0;
    if (c == 0 && rhs == 0) conv[(int64_t)ninst * gridDim.y] = 0;  // the count of flags set
  }
}

// one workgroup per (rhs, instance): ||G||, convergence decision, statistics
// fixed-order sum of a[i0 .. i0+n) by one 64-lane wave (lane-strided, then butterfly)
__device__ __forceinline__ double wave_fixed_sum(const double* __restrict__ a, int64_t i0, int64_t n) {
  double t = 0.0;
  for (int64_t q = threadIdx.x; q < n; q += 64) t += a[i0 + q];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) t += __shfl_xor(t, off, 64);
  return t;
}

__global__ __launch_bounds__(64) void k_check(DevTables T, const int64_t* __restrict__ cum_fin, int ninst,
                                              int nchunks, int64_t nfin, int it, int newton_max, double tol,
                                              const double* __restrict__ part, const double* __restrict__ partw,
                                              double* __restrict__ wnorm, int32_t* __restrict__ conv,
                                              sgdg_stats* __restrict__ stats) {
  const int inst = blockIdx.x, rhs = blockIdx.y;
  const int ci = rhs * ninst + inst;
  if (conv[ci]) return;
  const int S = T.inst[inst].S;
  const int c0 = T.pchunk0[inst * 2];
  int nc = T.pnchunk[inst * 2];
  if (S > 1) nc += T.pnchunk[inst * 2 + 1];
  if (it == 0) {
    const double t = wave_fixed_sum(partw, (int64_t)rhs * nchunks + c0, nc);
    if (threadIdx.x == 0) wnorm[ci] = sqrt(t);
  }
  const double t = wave_fixed_sum(part, (int64_t)rhs * nfin + cum_fin[inst], cum_fin[inst + 1] - cum_fin[inst]);
  if (threadIdx.x != 0) return;
  const double res = sqrt(t);
  const bool fin = isfinite(res);
  const bool ok = fin && res <= tol * fmax(1.0, wnorm[ci]);
  const bool last = it >= newton_max;
  if (ok || !fin || last) {
    conv[ci] = 1;
    atomicAdd(&conv[gridDim.x * gridDim.y], 1);  // (grid: one workgroup per problem)
  }
  if (stats)
    for (int s = 0; s < S; ++s) {
      sgdg_stats& st = stats[ci * 2 + s];
      st.newton_iters = it;
      st.residual = res;
      if (!fin)
        st.status = SGDG_ERR_NONFINITE;
      else if (!ok && last && st.status == SGDG_OK)
        st.status = SGDG_ERR_NOCONV;
    }
}

// U - c (F(U) + S) = W from U = W + c F (F holds the full right-hand side of
// the old level on entry and F(U) + S of the accepted iterate on return; S
// may be null)
static void implicit_stage(const sgdg_plan* plan, int nrhs, double c, double* U, double* F, const double* S,
                           const IifWs& w, double newton_tol, int newton_max, sgdg_stats* stats, hipStream_t s) {
  const dim3 cgrid((unsigned)plan->nchunks, (unsigned)nrhs);
  const int64_t n = plan->total * (int64_t)nrhs;
  const dim3 vg((unsigned)((n + 255) / 256)), vb(256);
  // a source S at the new level: U - c (P f(R U) + S) = W  <=>  U - c P f(R U) = W + c S
  if (S) hipLaunchKernelGGL(k_axpy, vg, vb, 0, s, w.W, w.W, c, S, n);
  hipLaunchKernelGGL(k_stage_init, cgrid, dim3(CHUNK), 0, s, plan->dev, plan->ninst, plan->nchunks, plan->total, c, U,
                     w.W, F, w.partw, w.conv);
  RxArgs a{};
  a.rws = w.rws;
  a.dt2 = c;
  a.U = U;
  a.W = w.W;
  a.F = F;
  a.Gout = w.G;
  a.G = w.G;
  a.part = w.part;
  a.conv = w.conv;
  a.nprob = plan->ninst * nrhs;
  const int64_t nfin = reaction_final_fibres(plan);
  for (int it = 0; it <= newton_max; ++it) {
    reaction_pass(plan, nrhs, RX_RESID, a, s);
    hipLaunchKernelGGL(k_check, dim3((unsigned)plan->ninst, (unsigned)nrhs), dim3(64), 0, s, plan->dev,
                       ((const RHost*)plan->rdata)->dev.cum_fin, plan->ninst, plan->nchunks, nfin, it, newton_max,
                       newton_tol, w.part, w.partw, w.wnorm, w.conv, stats);
    if (it < newton_max) reaction_pass(plan, nrhs, RX_CORR, a, s);
  }
  if (S) hipLaunchKernelGGL(k_axpy, vg, vb, 0, s, F, F, 1.0, S, n);  // F(U) of the new level includes S
}

static sgdg_status check_launch(const char* what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, what);
  return SGDG_OK;
}

}  // namespace sgdg

using namespace sgdg;

extern "C" sgdg_status sgdg_reaction(const sgdg_plan* plan, int32_t nrhs, const double* U, double* F, const double* S,
                                     void* workspace, size_t workspace_bytes, void* stream) {
  if (!plan) return fail(SGDG_ERR_ARG, "sgdg_reaction: null plan");
  if (nrhs < 1 || nrhs > 65535) return fail(SGDG_ERR_ARG, "sgdg_reaction: nrhs must be in 1..65535");
  if (!U || !F || !workspace) return fail(SGDG_ERR_ARG, "sgdg_reaction: null device pointer");
  if ((const void*)U == (const void*)F || (const void*)S == (const void*)F)
    return fail(SGDG_ERR_ARG, "sgdg_reaction: F must not alias U or S");
  if (!reaction_supported(plan)) return fail(SGDG_ERR_UNSUPPORTED, "sgdg_reaction: (k+1) 2^N above 2048 per axis (1024 with two species)");
  if (workspace_bytes < iif2_ws_bytes(plan, 1, nrhs)) return fail(SGDG_ERR_ARG, "sgdg_reaction: workspace too small");
  IifWs w = carve(plan, 1, nrhs, workspace);
  RxArgs a{};
  a.U = const_cast<double*>(U);
  a.F = F;
  a.rws = w.rws;
  reaction_pass(plan, nrhs, RX_F, a, (hipStream_t)stream);
  if (S) {
    const int64_t n = plan->total * (int64_t)nrhs;
    hipLaunchKernelGGL(k_axpy, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, (hipStream_t)stream, F, F, 1.0, S, n);
  }
  return check_launch("sgdg_reaction launch");
}

extern "C" sgdg_status sgdg_reaction_timed(const sgdg_plan* plan, int32_t nrhs, const double* U, double* F,
                                           void* workspace, size_t workspace_bytes, float* stage_ms, int32_t* stage_kind,
                                           int32_t* nstage, void* stream) {
  if (!plan) return fail(SGDG_ERR_ARG, "sgdg_reaction_timed: null plan");
  if (nrhs < 1 || nrhs > 65535) return fail(SGDG_ERR_ARG, "sgdg_reaction_timed: nrhs must be in 1..65535");
  if (!U || !F || !workspace || !stage_ms || !stage_kind || !nstage)
    return fail(SGDG_ERR_ARG, "sgdg_reaction_timed: null pointer");
  if ((const void*)U == (const void*)F) return fail(SGDG_ERR_ARG, "sgdg_reaction_timed: F must not alias U");
  if (!reaction_supported(plan))
    return fail(SGDG_ERR_UNSUPPORTED, "sgdg_reaction_timed: (k+1) 2^N above 2048 per axis (1024 with two species)");
  if (workspace_bytes < iif2_ws_bytes(plan, 1, nrhs))
    return fail(SGDG_ERR_ARG, "sgdg_reaction_timed: workspace too small");
  const int cap = *nstage;
  if (cap < 1) return fail(SGDG_ERR_ARG, "sgdg_reaction_timed: *nstage must be positive");
  hipStream_t s = (hipStream_t)stream;
  IifWs w = carve(plan, 1, nrhs, workspace);
  RxArgs a{};
  a.U = const_cast<double*>(U);
  a.F = F;
  a.rws = w.rws;
  // one event before every launch and one after the last
  std::vector<hipEvent_t> ev;
  std::vector<int> kind;
  sgdg_status st = SGDG_OK;
  const std::function<void(int)> mark = [&](int k) {
    hipEvent_t e;
    if (st != SGDG_OK) return;
    if (hipEventCreate(&e) != hipSuccess || hipEventRecord(e, s) != hipSuccess) {
      st = SGDG_ERR_HIP;
      return;
    }
    ev.push_back(e);
    kind.push_back(k);
  };
  reaction_pass(plan, nrhs, RX_F, a, s, &mark);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess && st == SGDG_OK) e = hipStreamSynchronize(s);
  int n = 0;
  for (size_t i = 0; e == hipSuccess && st == SGDG_OK && i + 1 < ev.size() && n < cap; ++i, ++n) {
    float ms = 0.f;
    e = hipEventElapsedTime(&ms, ev[i], ev[i + 1]);
    stage_ms[n] = ms;
    stage_kind[n] = kind[i];
  }
  for (hipEvent_t x : ev) (void)hipEventDestroy(x);
  if (st != SGDG_OK) return hip_fail(hipErrorUnknown, "sgdg_reaction_timed events");
  if (e != hipSuccess) return hip_fail(e, "sgdg_reaction_timed");
  *nstage = n;
  return SGDG_OK;
}

extern "C" sgdg_status iif2_step(const sgdg_plan* plan, int32_t nrhs, double dt, int32_t M, double* U, double* Fcache,
                                 const double* S_next, double newton_tol, int32_t newton_max, void* workspace,
                                 size_t workspace_bytes, sgdg_stats* stats, void* stream) {
  if (!plan) return fail(SGDG_ERR_ARG, "iif2_step: null plan");
  if (nrhs < 1 || nrhs > 65535) return fail(SGDG_ERR_ARG, "iif2_step: nrhs must be in 1..65535");
  if (M < 1 || M > SGDG_MAX_M) return fail(SGDG_ERR_ARG, "iif2_step: M must be in 1..48");
  if (!(dt > 0.0) || !std::isfinite(dt)) return fail(SGDG_ERR_ARG, "iif2_step: dt must be positive");
  if (!(newton_tol >= 0.0)) return fail(SGDG_ERR_ARG, "iif2_step: newton_tol must be >= 0");
  if (newton_max < 0 || newton_max > 1000) return fail(SGDG_ERR_ARG, "iif2_step: newton_max must be in 0..1000");
  if (!U || !workspace) return fail(SGDG_ERR_ARG, "iif2_step: null device pointer");
  if (U == Fcache || (const double*)U == S_next || (S_next && (const double*)Fcache == S_next))
    return fail(SGDG_ERR_ARG, "iif2_step: U, Fcache and S_next must not alias");
  if (S_next && !Fcache) return fail(SGDG_ERR_ARG, "iif2_step: a source needs the F cache (F of the old level)");
  if (!reaction_supported(plan)) return fail(SGDG_ERR_UNSUPPORTED, "iif2_step: (k+1) 2^N above 2048 per axis (1024 with two species)");
  if (workspace_bytes < iif2_ws_bytes(plan, M, nrhs)) return fail(SGDG_ERR_ARG, "iif2_step: workspace too small");
  hipStream_t s = (hipStream_t)stream;
  IifWs w = carve(plan, M, nrhs, workspace);
  const double dt2 = 0.5 * dt;
  const int64_t n = plan->total * (int64_t)nrhs;
  double* F = Fcache ? Fcache : w.F;
  RxArgs a{};
  a.rws = w.rws;
  a.dt2 = dt2;
  if (!Fcache) {
    a.U = U;
    a.F = F;
    reaction_pass(plan, nrhs, RX_F, a, s);
  }
  const KrylovIn vin{w.v, U, F, dt2};  // v = U + dt/2 F, formed by the first Krylov kernel
  sgdg_status st = krylov_run(plan, nrhs, dt, M, w.v, w.W, w.kws, stats, s, &vin);
  if (st != SGDG_OK) return st;
  implicit_stage(plan, nrhs, dt2, U, F, S_next, w, newton_tol, newton_max, stats, s);
  return check_launch("iif2_step launch");
}

// ---------------------------------------------------------------- fixed scratch
// iif2_step_noalloc runs iif2_step on a file-scope device array instead of a
// caller workspace.  The array exists once per device for the life of the
// process; in host code its name is not a device address, so the address
// comes from hipGetSymbolAddress, once per device, with that device current.
constexpr size_t SGDG_SCRATCH_BYTES = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[SGDG_SCRATCH_BYTES];

namespace {
constexpr int SCRATCH_MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[SCRATCH_MAX_DEVICES] = {};
}  // namespace

static sgdg_status scratch_address(int device, void** out) {
  if (device < 0 || device >= SCRATCH_MAX_DEVICES) return fail(SGDG_ERR_ARG, "iif2_step_noalloc: device index out of range");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e == hipSuccess && cur != device) e = hipSetDevice(device);
    void* p = nullptr;
    if (e == hipSuccess) e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (cur >= 0 && cur != device) (void)hipSetDevice(cur);
    if (e != hipSuccess) return hip_fail(e, "iif2_step_noalloc: hipGetSymbolAddress(scratch)");
    g_scratch_ptr[device] = p;
  }
  *out = g_scratch_ptr[device];
  return SGDG_OK;
}

extern "C" sgdg_status iif2_step_noalloc(const sgdg_plan* plan, int32_t nrhs, double dt, int32_t M, double* U,
                                         double* Fcache, const double* S_next, double newton_tol, int32_t newton_max,
                                         sgdg_stats* stats, void* stream) {
  if (!plan) return fail(SGDG_ERR_ARG, "iif2_step_noalloc: null plan");
  if (nrhs < 1 || nrhs > 65535) return fail(SGDG_ERR_ARG, "iif2_step_noalloc: nrhs must be in 1..65535");
  if (M < 1 || M > SGDG_MAX_M) return fail(SGDG_ERR_ARG, "iif2_step_noalloc: M must be in 1..48");
  const size_t need = iif2_ws_bytes(plan, M, nrhs);
  if (need > SGDG_SCRATCH_BYTES)
    return fail(SGDG_ERR_UNSUPPORTED, "iif2_step_noalloc: this plan, M and nrhs need " + std::to_string(need) +
                                          " bytes of workspace; the fixed device scratch holds " +
                                          std::to_string(SGDG_SCRATCH_BYTES) + " (call iif2_step with a workspace)");
  void* ws = nullptr;
  const sgdg_status st = scratch_address(plan->device, &ws);
  if (st != SGDG_OK) return st;
  // every kernel of the step writes its part of the workspace before reading
  // it (as with a caller workspace from an uninitialised allocation), so
  // nothing needs clearing between calls
  return iif2_step(plan, nrhs, dt, M, U, Fcache, S_next, newton_tol, newton_max, ws, SGDG_SCRATCH_BYTES, stats,
                   stream);
}

extern "C" sgdg_status iif3_step(const sgdg_plan* plan, int32_t nrhs, double dt, int32_t M, double* U, double* Fcur,
                                 double* Fprev, const double* S_next, double newton_tol, int32_t newton_max,
                                 void* workspace, size_t workspace_bytes, sgdg_stats* stats, void* stream) {
  if (!plan) return fail(SGDG_ERR_ARG, "iif3_step: null plan");
  if (nrhs < 1 || nrhs > 65535) return fail(SGDG_ERR_ARG, "iif3_step: nrhs must be in 1..65535");
  if (M < 1 || M > SGDG_MAX_M) return fail(SGDG_ERR_ARG, "iif3_step: M must be in 1..48");
  if (!(dt > 0.0) || !std::isfinite(dt)) return fail(SGDG_ERR_ARG, "iif3_step: dt must be positive");
  if (!(newton_tol >= 0.0)) return fail(SGDG_ERR_ARG, "iif3_step: newton_tol must be >= 0");
  if (newton_max < 0 || newton_max > 1000) return fail(SGDG_ERR_ARG, "iif3_step: newton_max must be in 0..1000");
  if (!U || !Fcur || !Fprev || !workspace) return fail(SGDG_ERR_ARG, "iif3_step: null device pointer");
  if (U == Fcur || U == Fprev || Fcur == Fprev) return fail(SGDG_ERR_ARG, "iif3_step: U, Fcur and Fprev must not alias");
  if (!reaction_supported(plan)) return fail(SGDG_ERR_UNSUPPORTED, "iif3_step: (k+1) 2^N above 2048 per axis (1024 with two species)");
  if (workspace_bytes < iif2_ws_bytes(plan, M, nrhs)) return fail(SGDG_ERR_ARG, "iif3_step: workspace too small");
  hipStream_t s = (hipStream_t)stream;
  IifWs w = carve(plan, M, nrhs, workspace);
  const int64_t n = plan->total * (int64_t)nrhs;
  const dim3 vg((unsigned)((n + 255) / 256)), vb(256);
  // exp(2 A dt)(-1/12 dt F^{n-1}); F^{n-1} is then replaced by F^n
  const KrylovIn vin1{w.v, nullptr, Fprev, -dt / 12.0};
  sgdg_status st = krylov_run(plan, nrhs, 2.0 * dt, M, w.v, w.W2, w.kws, stats, s, &vin1);
  if (st != SGDG_OK) return st;
  hipLaunchKernelGGL(k_copy, vg, vb, 0, s, Fprev, Fcur, n);
  // exp(A dt)(U^n + 2/3 dt F^n), plus the first term
  const KrylovIn vin2{w.v, U, Fcur, 2.0 * dt / 3.0};
  st = krylov_run(plan, nrhs, dt, M, w.v, w.W, w.kws, stats, s, &vin2);
  if (st != SGDG_OK) return st;
  hipLaunchKernelGGL(k_axpy, vg, vb, 0, s, w.W, w.W, 1.0, w.W2, n);
  implicit_stage(plan, nrhs, 5.0 * dt / 12.0, U, Fcur, S_next, w, newton_tol, newton_max, stats, s);
  return check_launch("iif3_step launch");
}

// L(V) = A V + F(V) into out (tmp: F(V)); FP64 plans
static void rk_rhs(const sgdg_plan* plan, int nrhs, const double* V, double* out, double* tmp, const IifWs& w,
                   hipStream_t s) {
  launch_apply<PrecF64>(plan, nrhs, V, out, plan->total, plan->total, s);
  RxArgs a{};
  a.rws = w.rws;
  a.U = const_cast<double*>(V);
  a.F = tmp;
  reaction_pass(plan, nrhs, RX_F, a, s);
  const int64_t n = plan->total * (int64_t)nrhs;
  hipLaunchKernelGGL(k_axpy, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, out, out, 1.0, tmp, n);
}

extern "C" sgdg_status rk_step(const sgdg_plan* plan, int32_t nrhs, double dt, int32_t order, double* U,
                               void* workspace, size_t workspace_bytes, void* stream) {
  if (!plan) return fail(SGDG_ERR_ARG, "rk_step: null plan");
  if (nrhs < 1 || nrhs > 65535) return fail(SGDG_ERR_ARG, "rk_step: nrhs must be in 1..65535");
  if (order != 2 && order != 3) return fail(SGDG_ERR_ARG, "rk_step: order must be 2 or 3");
  if (!(dt > 0.0) || !std::isfinite(dt)) return fail(SGDG_ERR_ARG, "rk_step: dt must be positive");
  if (!U || !workspace) return fail(SGDG_ERR_ARG, "rk_step: null device pointer");
  if (plan->prec != SGDG_FP64) return fail(SGDG_ERR_UNSUPPORTED, "rk_step: FP64 plans only");
  if (!reaction_supported(plan)) return fail(SGDG_ERR_UNSUPPORTED, "rk_step: (k+1) 2^N above 2048 per axis (1024 with two species)");
  if (workspace_bytes < iif2_ws_bytes(plan, 1, nrhs)) return fail(SGDG_ERR_ARG, "rk_step: workspace too small");
  hipStream_t s = (hipStream_t)stream;
  IifWs w = carve(plan, 1, nrhs, workspace);
  const int64_t n = plan->total * (int64_t)nrhs;
  const dim3 vg((unsigned)((n + 255) / 256)), vb(256);
  // stage 1: v = U + dt L(U)
  rk_rhs(plan, nrhs, U, w.G, w.F, w, s);
  hipLaunchKernelGGL(k_axpy, vg, vb, 0, s, w.v, U, dt, w.G, n);
  rk_rhs(plan, nrhs, w.v, w.G, w.F, w, s);
  if (order == 2) {
    // U = 1/2 U + 1/2 (v + dt L(v))
    hipLaunchKernelGGL(k_lin3, vg, vb, 0, s, U, 0.5, U, 0.5, w.v, 0.5 * dt, w.G, n);
  } else {
    // W = 3/4 U + 1/4 (v + dt L(v));  U = 1/3 U + 2/3 (W + dt L(W))
    hipLaunchKernelGGL(k_lin3, vg, vb, 0, s, w.W, 0.75, U, 0.25, w.v, 0.25 * dt, w.G, n);
    rk_rhs(plan, nrhs, w.W, w.G, w.F, w, s);
    hipLaunchKernelGGL(k_lin3, vg, vb, 0, s, U, 1.0 / 3.0, U, 2.0 / 3.0, w.W, 2.0 / 3.0 * dt, w.G, n);
  }
  return check_launch("rk_step launch");
}

extern "C" sgdg_status iif2_step_local(const sgdg_plan* plan, int32_t nrhs, double dt, int32_t M, double* U,
                                       double* Fcache, const double* S_next, void* workspace, size_t workspace_bytes,
                                       sgdg_stats* stats, void* stream) {
  if (!plan) return fail(SGDG_ERR_ARG, "iif2_step_local: null plan");
  if (nrhs < 1 || nrhs > 65535) return fail(SGDG_ERR_ARG, "iif2_step_local: nrhs must be in 1..65535");
  if (M < 1 || M > SGDG_MAX_M) return fail(SGDG_ERR_ARG, "iif2_step_local: M must be in 1..48");
  if (!(dt > 0.0) || !std::isfinite(dt)) return fail(SGDG_ERR_ARG, "iif2_step_local: dt must be positive");
  if (!U || !Fcache || !workspace) return fail(SGDG_ERR_ARG, "iif2_step_local: null device pointer");
  if (U == Fcache) return fail(SGDG_ERR_ARG, "iif2_step_local: U and Fcache must not alias");
  if (!reaction_supported(plan)) return fail(SGDG_ERR_UNSUPPORTED, "iif2_step_local: (k+1) 2^N above 2048 per axis (1024 with two species)");
  if (workspace_bytes < iif2_ws_bytes(plan, M, nrhs))
    return fail(SGDG_ERR_ARG, "iif2_step_local: workspace too small");
  hipStream_t s = (hipStream_t)stream;
  IifWs w = carve(plan, M, nrhs, workspace);
  const double c = 0.5 * dt;
  const int64_t n = plan->total * (int64_t)nrhs;
  const dim3 vg((unsigned)((n + 255) / 256)), vb(256);
  const KrylovIn vin{w.v, U, Fcache, c};
  sgdg_status st = krylov_run(plan, nrhs, dt, M, w.v, w.W, w.kws, stats, s, &vin);
  if (st != SGDG_OK) return st;
  if (S_next) hipLaunchKernelGGL(k_axpy, vg, vb, 0, s, w.W, w.W, c, S_next, n);
  // U = P u, u - c f(u) = R W at every Gauss point
  RxArgs a{};
  a.rws = w.rws;
  a.dt2 = c;
  a.U = w.W;
  a.Gout = U;
  reaction_pass(plan, nrhs, RX_LOCAL, a, s);
  // F of the new level
  RxArgs b{};
  b.rws = w.rws;
  b.U = U;
  b.F = Fcache;
  reaction_pass(plan, nrhs, RX_F, b, s);
  if (S_next) hipLaunchKernelGGL(k_axpy, vg, vb, 0, s, Fcache, Fcache, 1.0, S_next, n);
  return check_launch("iif2_step_local launch");
}

// ---------------------------------------------------------------- launch-shape autotuning
namespace {
// key: architecture name, compute units, K1, N, species, inputs, nrhs, lines of the class
using TuneKey = std::tuple<std::string, int64_t, int64_t, int64_t, int64_t, int64_t, int64_t, int64_t>;
std::mutex g_tune_mu;
struct TuneShape {
  int rounds, wgcu, waves;
};
std::map<TuneKey, TuneShape> g_tune_cache;
bool g_tune_file_read = false;

// The file named by SGDG_TUNE_CACHE (if set) extends the process cache: one
// line per choice, "arch cus K1 N S inputs nrhs lines rounds wgcu waves"
// (a line without the last field means waves 0); read once, appended to
// after every new choice.  (Called with g_tune_mu held.)
void tune_file_read() {
  if (g_tune_file_read) return;
  g_tune_file_read = true;
  const char* path = std::getenv("SGDG_TUNE_CACHE");
  if (!path || !*path) return;
  FILE* f = std::fopen(path, "r");
  if (!f) return;
  char line[512], arch[64];
  long long v[10];
  while (std::fgets(line, sizeof line, f)) {
    v[9] = 0;
    const int n = std::sscanf(line, "%63s %lld %lld %lld %lld %lld %lld %lld %lld %lld %lld", arch, &v[0], &v[1], &v[2],
                              &v[3], &v[4], &v[5], &v[6], &v[7], &v[8], &v[9]);
    if (n == 10 || n == 11)
      g_tune_cache[TuneKey{arch, v[0], v[1], v[2], v[3], v[4], v[5], v[6]}] = {(int)v[7], (int)v[8], (int)v[9]};
  }
  std::fclose(f);
}

void tune_file_append(const TuneKey& k, const TuneShape& t) {
  const char* path = std::getenv("SGDG_TUNE_CACHE");
  if (!path || !*path) return;
  FILE* f = std::fopen(path, "a");
  if (!f) return;
  std::fprintf(f, "%s %lld %lld %lld %lld %lld %lld %lld %d %d %d\n", std::get<0>(k).c_str(),
               (long long)std::get<1>(k), (long long)std::get<2>(k), (long long)std::get<3>(k),
               (long long)std::get<4>(k), (long long)std::get<5>(k), (long long)std::get<6>(k),
               (long long)std::get<7>(k), t.rounds, t.wgcu, t.waves);
  std::fclose(f);
}
}  // namespace

extern "C" sgdg_status sg_dg_line_shape(sgdg_plan* plan, int32_t cls, int32_t ninputs, int32_t rounds, int32_t wgcu,
                                        int32_t waves) {
  if (!plan) return fail(SGDG_ERR_ARG, "sg_dg_line_shape: null plan");
  if (!reaction_supported(plan)) return fail(SGDG_ERR_UNSUPPORTED, "sg_dg_line_shape: the plan has no reaction tables");
  // (queued work of any stream may still read the tile list being replaced)
  const hipError_t e = hipDeviceSynchronize();
  if (e != hipSuccess) return hip_fail(e, "sg_dg_line_shape: synchronise");
  return reaction_set_line_shape(plan, cls, ninputs, rounds, wgcu, waves);
}

extern "C" sgdg_status sg_dg_tune(sgdg_plan* plan, int32_t nrhs, void* workspace, size_t workspace_bytes,
                                  sgdg_tune_report* report, void* stream) {
  if (!plan) return fail(SGDG_ERR_ARG, "sg_dg_tune: null plan");
  if (nrhs < 1 || nrhs > 65535) return fail(SGDG_ERR_ARG, "sg_dg_tune: nrhs must be in 1..65535");
  if (!workspace) return fail(SGDG_ERR_ARG, "sg_dg_tune: null workspace");
  if (!reaction_supported(plan)) return fail(SGDG_ERR_UNSUPPORTED, "sg_dg_tune: the plan has no reaction tables");
  if (workspace_bytes < iif2_ws_bytes(plan, 1, nrhs)) return fail(SGDG_ERR_ARG, "sg_dg_tune: workspace too small");
  hipStream_t s = (hipStream_t)stream;
  sgdg_tune_report rep{};
  // (queued work of any stream may still read the tile lists being replaced)
  hipError_t e = hipDeviceSynchronize();
  if (e != hipSuccess) return hip_fail(e, "sg_dg_tune: synchronise");
  IifWs w = carve(plan, 1, nrhs, workspace);
  // fixed inputs for the timed launches: the reaction workspace and both input vectors zero
  const size_t tot = (size_t)plan->total * nrhs;
  e = hipMemsetAsync(w.rws, 0, (size_t)reaction_ws_doubles(plan) * nrhs * 8, s);
  if (e == hipSuccess) e = hipMemsetAsync(w.v, 0, tot * 8, s);
  if (e == hipSuccess) e = hipMemsetAsync(w.W, 0, tot * 8, s);
  if (e != hipSuccess) return hip_fail(e, "sg_dg_tune: workspace fill");
  RxArgs a{};
  a.rws = w.rws;
  a.U = w.v;
  a.G = w.W;
  a.F = w.F;
  a.Gout = w.G;
  a.W = w.W2;
  a.part = w.part;
  a.dt2 = 1e-3;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if ((e = hipEventCreate(&e0)) != hipSuccess || (e = hipEventCreate(&e1)) != hipSuccess) {
    if (e0) (void)hipEventDestroy(e0);
    return hip_fail(e, "sg_dg_tune: events");
  }
  hipDeviceProp_t prop;
  if ((e = hipGetDeviceProperties(&prop, plan->device)) != hipSuccess) {
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return hip_fail(e, "sg_dg_tune: device properties");
  }
  const std::string arch = std::string(prop.gcnArchName).substr(0, std::string(prop.gcnArchName).find(':'));
  const int64_t ncu = prop.multiProcessorCount;
  static const int kRounds[] = {1, 2, 4, 8, 16, 32};
  static const int kWgcu[] = {4, 8, 16, 32};
  constexpr int kReps = 3;
  sgdg_status st = SGDG_OK;
  const int ncls = reaction_line_classes(plan);
  for (int c = 0; c < ncls && st == SGDG_OK; ++c) {
    const LineClass& lc = reaction_line_class(plan, c);
    if (!lc.wave || rep.nclass >= SGDG_TUNE_MAXCLASS) continue;
    const int slot = rep.nclass++;
    rep.k[slot] = lc.K1 - 1;
    rep.n[slot] = lc.N;
    rep.nspecies[slot] = lc.S;
    rep.cls[slot] = c;
    int64_t lines = 0, most = 0;
    for (const WaveLines& il : lc.lines) {
      lines += il.lines;
      most = std::max(most, il.lines);
    }
    for (int nin = 1; nin <= 2 && st == SGDG_OK; ++nin) {
      const RxMode mode = nin == 1 ? RX_F : RX_CORR;
      // one launch of the class's last axis at a shape, averaged over kReps after a warm-up
      auto time_shape = [&](int r, int g, int wv, float* ms) -> sgdg_status {
        sgdg_status q = reaction_set_line_shape(plan, c, nin, r, g, wv);
        if (q != SGDG_OK) return q;
        reaction_line_stage(plan, nrhs, mode, a, s, c);
        hipError_t he = hipEventRecord(e0, s);
        for (int i = 0; i < kReps && he == hipSuccess; ++i) {
          reaction_line_stage(plan, nrhs, mode, a, s, c);
          he = hipGetLastError();
        }
        if (he == hipSuccess) he = hipEventRecord(e1, s);
        if (he == hipSuccess) he = hipEventSynchronize(e1);
        float t = 0.f;
        if (he == hipSuccess) he = hipEventElapsedTime(&t, e0, e1);
        if (he != hipSuccess) return hip_fail(he, "sg_dg_tune: timed launch");
        *ms = t / kReps;
        return SGDG_OK;
      };
      const TuneKey key{arch, ncu, lc.K1, lc.N, lc.S, nin, nrhs, lines};
      {
        std::lock_guard<std::mutex> g(g_tune_mu);
        tune_file_read();
        auto it = g_tune_cache.find(key);
        if (it != g_tune_cache.end()) {
          const TuneShape& t = it->second;
          st = reaction_set_line_shape(plan, c, nin, t.rounds, t.wgcu, t.waves);
          rep.rounds[slot][nin - 1] = t.rounds;
          rep.wgcu[slot][nin - 1] = t.wgcu;
          rep.waves[slot][nin - 1] = t.waves;
          rep.from_cache[slot][nin - 1] = 1;
          continue;
        }
      }
      const int r0 = lc.rounds[nin], g0 = lc.wgcu[nin], v0 = lc.waves[nin];
      float t0 = 0.f;
      if ((st = time_shape(r0, g0, v0, &t0)) != SGDG_OK) break;
      TuneShape b{r0, g0, v0};
      float tb = t0;
      auto trial = [&](int r, int g, int wv) -> sgdg_status {
        float t = 0.f;
        const sgdg_status q = time_shape(r, g, wv, &t);
        if (q == SGDG_OK && t < tb) {
          tb = t;
          b = {r, g, wv};
        }
        return q;
      };
      // the grid of shapes with the compiler's registers, then the capped
      // register budget at the best rounds with every workgroup count
      for (int r : kRounds) {
        if (r > 1 && (int64_t)lc.lpr * (r / 2) >= most) break;  // (no more lines per tile than the largest instance has)
        for (int g : kWgcu)
          if ((st = trial(r, g, 0)) != SGDG_OK) break;
        if (st != SGDG_OK) break;
      }
      const int rbest = b.rounds;
      for (int g : kWgcu)
        if (st == SGDG_OK) st = trial(rbest, g, 3);
      if (st != SGDG_OK) break;
      if ((st = reaction_set_line_shape(plan, c, nin, b.rounds, b.wgcu, b.waves)) != SGDG_OK) break;
      rep.rounds[slot][nin - 1] = b.rounds;
      rep.wgcu[slot][nin - 1] = b.wgcu;
      rep.waves[slot][nin - 1] = b.waves;
      rep.ms_default[slot][nin - 1] = t0;
      rep.ms_best[slot][nin - 1] = tb;
      std::lock_guard<std::mutex> g(g_tune_mu);
      g_tune_cache[key] = b;
      tune_file_append(key, b);
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (report) *report = rep;
  return st;
}
