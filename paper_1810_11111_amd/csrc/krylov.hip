// Krylov approximation of exp(h A) v (Sec. 3, eqs. 3.7-3.8).
//
// Arnoldi: v_1 = v / gamma, gamma = ||v||_2; for j = 1..M: w = A v_j,
// orthogonalise against v_1..v_j, h_{j+1,j} = ||w||, v_{j+1} = w / h_{j+1,j};
// result gamma V_m exp(h H_m) e_1 with exp(h H_m) by Pade approximation with
// scaling and squaring (Higham 2005).
//
// GPU form.  Every (right-hand side, instance, species) is an independent
// problem; all problems advance in lockstep over j.  Orthogonalisation is
// classical Gram-Schmidt applied twice (rounding-level equivalent of the
// modified form) with the second pass delayed by one step, so that a step
// needs one device-wide reduction besides the sweep; each reduction is a
// kernel boundary (cheap inside a captured graph):
//   sweep : w = A x_j (the sg_dg_apply kernels) and, in the same workgroups,
//           the per-chunk partials <v_i, w> (i < j) and <x_j, w>, where slot j
//           of the basis holds x_j, the once-orthogonalised residual of the
//           previous step
//   k_upd : reorthogonalise and normalise x_j into v_j with the partials of
//           <v_i, x_j> and |x_j|^2 left by the previous step, form
//           x_{j+1} = (A v_j minus its projection on v_0..v_j), and leave the
//           partials of <v_i, x_{j+1}> and |x_{j+1}|^2 for the next step
// A v_j is never formed: w = A x_j and x_j = V c + alpha v_j give
// A v_j = (w - A V c) / alpha, and A V c lies in the span of v_0..v_j, so only
// the Hessenberg column needs it; the per-step scalars (s, c, alpha) are
// logged and k_expm assembles H from them.  Partial sums are reduced in a
// fixed order, so every workgroup of a problem computes bit-identical scalars
// and breakdown decisions.
// Dot products, norms, H, exp(h H) and the final combination are FP64 in
// every precision mode; the basis is stored in the sweep precision.
#include <hip/hip_runtime.h>

#include <cmath>

#include "internal.h"
#include "kernels.h"
#include "krylov.h"

namespace sgdg {

constexpr int NW = CHUNK / 64;

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// maximum over the wave, returned to every lane: DPP steps within each row
// of 16 lanes (quad xor 1, quad xor 2, half-row mirror, row mirror), then the
// four row maxima read as scalars
__device__ __forceinline__ unsigned wave_max_u32(unsigned v) {
  v = max(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0xB1, 0xF, 0xF, false));
  v = max(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x4E, 0xF, 0xF, false));
  v = max(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x141, 0xF, 0xF, false));
  v = max(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x140, 0xF, 0xF, false));
  const unsigned a = (unsigned)__builtin_amdgcn_readlane((int)v, 0), b = (unsigned)__builtin_amdgcn_readlane((int)v, 16);
  const unsigned c = (unsigned)__builtin_amdgcn_readlane((int)v, 32), d = (unsigned)__builtin_amdgcn_readlane((int)v, 48);
  return max(max(a, b), max(c, d));
}

// the FP64 value of lane l (l uniform)
__device__ __forceinline__ double readlane_f64(double v, int l) {
  const long long b = __double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)b, l);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

__device__ __forceinline__ int prob_of(int rhs, int ninst, const Chunk& ch) { return (rhs * ninst + ch.inst) * 2 + ch.species; }

template <class TV>
__device__ __forceinline__ const TV* vec(const KrylovWs& ws, int i, int nrhs, int rhs, int64_t total) {
  return (const TV*)ws.V + ((int64_t)i * nrhs + rhs) * total;
}

// ||v||^2 partial per chunk; resets the per-problem state.  With vbuf, v is
// first formed as vx + va vy (vx may be null) and stored there.
__global__ __launch_bounds__(CHUNK) void k_init(DevTables T, int nchunks, int ninst, int64_t total, int M,
                                                const double* __restrict__ v, KrylovWs ws, double* __restrict__ vbuf,
                                                const double* __restrict__ vx, const double* __restrict__ vy,
                                                double va) {
  const int c = blockIdx.x, rhs = blockIdx.y, tid = threadIdx.x;
  const Chunk ch = T.chunks[c];
  double x = 0.0;
  if (tid < ch.count) {
    const int64_t i = rhs * total + ch.start + tid;
    double a;
    if (vbuf) {
      a = vx ? vx[i] + va * vy[i] : va * vy[i];
      vbuf[i] = a;
    } else {
      a = v[i];
    }
    x = a * a;
  }
  x = wave_sum(x);
  __shared__ double red[NW];
  if ((tid & 63) == 0) red[tid >> 6] = x;
  __syncthreads();
  if (tid == 0) {
    double t = 0.0;
    for (int w = 0; w < NW; ++w) t += red[w];
    ws.part1[((int64_t)rhs * nchunks + c) * (M + 2)] = t;
    if (c == ch.pc0) {
      const int p = prob_of(rhs, ninst, ch);
      ws.done[p] = 0;
      ws.m[p] = 0;
    }
  }
}

// gamma = ||v||, v_1 = v / gamma.
template <class TV>
__global__ __launch_bounds__(CHUNK) void k_norm(DevTables T, int nchunks, int ninst, int64_t total, int M,
                                                const double* __restrict__ v, KrylovWs ws) {
  const int c = blockIdx.x, rhs = blockIdx.y, tid = threadIdx.x, nrhs = gridDim.y;
  const Chunk ch = T.chunks[c];
  const int c0 = ch.pc0, nc = ch.pnc;
  __shared__ double sb;
  if (tid < 64) {
    // fixed-order sum of the nc chunk partials by one wave (lane-strided, then butterfly)
    double t = 0.0;
    for (int q = tid; q < nc; q += 64) t += ws.part1[((int64_t)rhs * nchunks + c0 + q) * (M + 2)];
    t = wave_sum(t);
    if (tid == 0) sb = sqrt(t);
  }
  __syncthreads();
  const double beta = sb;
  const int p = prob_of(rhs, ninst, ch);
  if (c == c0 && tid == 0) {
    ws.beta[p] = beta;
    if (!(beta > 0.0)) {
      ws.done[p] = 1;
      ws.m[p] = 0;
    }
  }
  if (!(beta > 0.0) || tid >= ch.count) return;
  const int64_t g = ch.start + tid;
  const double x = v[rhs * total + g] / beta;
  ((TV*)ws.V)[(int64_t)rhs * total + g] = (TV)x;
  if (ws.Vb) ws.Vb[rhs * total + g] = f_to_bf16((float)x);
  (void)nrhs;
}

// Deterministic reduction of per-chunk partials of one problem: h[i] = sum
// over its nc chunks of part[c0 + q][i], i < cols.
__device__ __forceinline__ void reduce_partials(const double* __restrict__ part, int64_t row0, int nc, int ld, int cols,
                                                double* red, double* h) {
  const int tid = threadIdx.x;
  const int S = CHUNK / cols;
  if (tid < cols * S) {
    const int i = tid / S, s = tid - i * S;
    double acc = 0.0;
    for (int q = s; q < nc; q += S) acc += part[(row0 + q) * ld + i];
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

// Arnoldi step j after the sweep (see the header).  With s'_i the reduced
// sweep partials and c_i, n the partials left by step j-1 (none for j = 0,
// where x_0 = v_0):
//   alpha = h_{j,j-1} = sqrt(n - |c|^2)  (breakdown: alpha <= rel ||A||),
//   v_j = (x_j - sum_{i<j} c_i v_i) / alpha,
//   s_i = s'_i (i < j),  s_j = <v_j, w> = (s'_j - c . s'_{0..j-1}) / alpha,
//   x_{j+1} = (w - sum_{i<=j} s_i v_i) / alpha,
// then the partials <v_i, x_{j+1}> (i <= j) and |x_{j+1}|^2 into the other
// buffer of the pair (the one read here may still be read by other
// workgroups).  The chunk's first workgroup logs (s, c, alpha).
// done[p] = 1 + the first step that no longer runs for problem p.
template <class TV, class TY, int JB>
__global__ __launch_bounds__(CHUNK) void k_upd(DevTables T, int nchunks, int ninst, int64_t total, int M, int j,
                                               KrylovWs ws) {
  const int c = blockIdx.x, rhs = blockIdx.y, tid = threadIdx.x, nrhs = gridDim.y;
  const Chunk ch = T.chunks[c];
  const int p = prob_of(rhs, ninst, ch);
  const int c0 = ch.pc0, nc = ch.pnc;
  // products v_i x_{j+1} of the chunk, column i at tp[i][.] (see the end)
  // (column stride CHUNK + 1: the slice sums read columns in the same rows,
  // and an odd stride puts them in different LDS banks)
  constexpr int TPS = CHUNK + 1;
  __shared__ double sv[SGDG_MAX_M + 1], cv[SGDG_MAX_M + 1], red[CHUNK], tp[(JB + 2) * TPS];
  __shared__ double alpha_s;
  __shared__ int stop_s;
  const double* pin = (j & 1) ? ws.part3 : ws.part2;
  double* pout = (j & 1) ? ws.part2 : ws.part3;
  // Every load of the step is issued before the first wait: this thread's
  // share of the partial sums (thread (col, slice) of a cols x S arrangement
  // takes chunks slice, slice + S, ...), then x_j, w and v_i (i < j <= JB) of
  // its element.  No load sits under a branch (indices are clamped into range
  // and unused values discarded), so the waits can count them: loads return
  // in order, and the reduction waits only for its own.
  const int na = j + 1, nb = j ? j + 1 : 0, cols = na + nb, S = CHUNK / cols;
  const int pc = min(tid / S, cols - 1), ps = tid - (tid / S) * S;
  const bool pact = tid < cols * S;
  const double* psrc = pc < na ? ws.part1 + pc : pin + (pc - na);
  const int64_t row0 = (int64_t)rhs * nchunks + c0;
  constexpr int QMAX = 8;
  const bool few = nc <= QMAX * S;
  double pq[QMAX];
#pragma unroll
  for (int q = 0; q < QMAX; ++q) pq[q] = psrc[(row0 + min(ps + q * S, nc - 1)) * (M + 2)];
  const bool act = tid < ch.count;
  const int64_t g = ch.start + min(tid, ch.count - 1);
  TV* Vj = (TV*)ws.V + ((int64_t)j * nrhs + rhs) * total;
  const double x0 = (double)Vj[g];
  const double w0 = (double)((const TY*)ws.wy)[rhs * total + g];
  double vv[JB];
#pragma unroll
  for (int i = 0; i < JB; ++i) vv[i] = (double)vec<TV>(ws, max(min(i, j - 1), 0), nrhs, rhs, total)[g];
  const int dn = ws.done[p];
  __builtin_amdgcn_sched_barrier(0);  // keep the sums below every load
  if (dn && j >= dn - 1) return;  // (the loads above are in range either way)
  {
    // terms q = ps, ps + S, ... in order (the padded terms are zeros): the
    // first QMAX from the loads above, then batches of QMAX whose loads are
    // all issued before the first is added
    double acc = 0.0;
#pragma unroll
    for (int q = 0; q < QMAX; ++q) acc += ps + q * S < nc ? pq[q] : 0.0;
    if (!few && pact)
      for (int q0 = ps + QMAX * S; q0 < nc; q0 += QMAX * S) {
        double t[QMAX];
#pragma unroll
        for (int q = 0; q < QMAX; ++q) t[q] = psrc[(row0 + min(q0 + q * S, nc - 1)) * (M + 2)];
#pragma unroll
        for (int q = 0; q < QMAX; ++q) acc += q0 + q * S < nc ? t[q] : 0.0;
      }
    if (pact) red[tid] = acc;
  }
  __syncthreads();
  if (tid < cols) {
    double t = 0.0;
    for (int q = 0; q < S; ++q) t += red[tid * S + q];
    if (tid < na)
      sv[tid] = t;
    else
      cv[tid - na] = t;
  }
  __syncthreads();
  const InstDev& I = T.inst[ch.inst];
  if (tid < 64) {
    // |c|^2 and c . s' (i < j) by one wave, fixed-order butterfly sums
    const double ci = tid < j ? cv[tid] : 0.0;
    const double cc = wave_sum(ci * ci), cs = wave_sum(ci * (tid < j ? sv[tid] : 0.0));
    if (tid == 0) {
      double a = 1.0;
      int stop = 0;
      if (j > 0) {
        a = sqrt(fmax(cv[j] - cc, 0.0));
        stop = !(a > KRYLOV_BREAKDOWN_REL * I.anorm[ch.species]);
        sv[j] = stop ? 0.0 : (sv[j] - cs) / a;
      }
      alpha_s = a;
      stop_s = stop;
    }
  }
  __syncthreads();
  const double a = alpha_s;
  const bool stop = stop_s != 0;
  const int Mp = (int)min((int64_t)M, I.ndof);
  const bool last = j + 1 >= Mp;
  if (c == c0) {
    double* L = ws.lg + ((int64_t)p * (M + 1) + j) * (2 * M + 1);
    if (tid <= j) L[tid] = sv[tid];
    if (tid < j) L[M + tid] = cv[tid];
    if (tid == 0) {
      L[2 * M] = a;
      if (stop || last) {
        ws.m[p] = stop ? j : j + 1;
        ws.done[p] = j + 2;
      }
    }
  }
  if (stop) return;
  double vr = 0.0, ur = 0.0;
  if (act) {
    double xa = x0, wa = w0;
#pragma unroll
    for (int i = 0; i < JB; ++i)
      if (i < j) {
        xa -= cv[i] * vv[i];
        wa -= sv[i] * vv[i];
      }
    const TV vt = (TV)(xa / a);
    vr = (double)vt;
    if (j > 0) Vj[g] = vt;
    const double u = (wa - sv[j] * vr) / a;
    const TV ut = (TV)u;
    ur = (double)ut;
    if (!last) {
      ((TV*)ws.V)[((int64_t)(j + 1) * nrhs + rhs) * total + g] = ut;
      if (ws.Vb) ws.Vb[rhs * total + g] = f_to_bf16((float)ut);
    }
  }
  // chunk partials <v_i, x_{j+1}> (i < j), <v_j, x_{j+1}>, |x_{j+1}|^2 from
  // the basis entries already in registers: the products go to LDS by
  // column, then thread (i, s) of a (JB + 2) x S arrangement sums elements
  // s, s + S, ... of column i in that order, and the S slices in order
#pragma unroll
  for (int i = 0; i < JB; ++i)
    if (i < j) tp[i * TPS + tid] = vv[i] * ur;
  tp[j * TPS + tid] = vr * ur;
  tp[(j + 1) * TPS + tid] = ur * ur;
  __syncthreads();
  {
    constexpr int CJ = JB + 2, S2 = CHUNK / CJ, NE = (CHUNK + S2 - 1) / S2;
    const int i = tid / S2, s2 = tid - i * S2;
    if (i < j + 2) {
      double acc = 0.0;
#pragma unroll
      for (int q = 0; q < NE; ++q) {
        const int e = s2 + q * S2;
        if (e < CHUNK) acc += tp[i * TPS + e];
      }
      red[tid] = acc;
    }
    __syncthreads();
    if (tid < j + 2) {
      double t = 0.0;
#pragma unroll
      for (int q = 0; q < S2; ++q) t += red[tid * S2 + q];
      pout[((int64_t)rhs * nchunks + c) * (M + 2) + tid] = t;
    }
  }
}

// ---- exp(h H_m) e_1: Pade approximation with scaling and squaring ---------
// Higham, "The scaling and squaring method for the matrix exponential
// revisited", SIAM J. Matrix Anal. Appl. 26 (2005): degree m in {3,5,7,9,13}
// chosen from ||A||_1 against theta_m; for degree 13, A is scaled by 2^-s with
// s = ceil(log2(||A||_1 / theta_13)) and the result squared s times.
// [m/m] Pade coefficients b_j = (2m-j)! m! / ((2m)! j! (m-j)!) from the
// ratio b_j / b_{j-1} = (m-j+1) / (j (2m-j+1)).
constexpr int MM = SGDG_MAX_M;
constexpr int LDM = MM + 1;  // odd row stride (in doubles): row-per-lane accesses spread over all LDS banks

typedef double v4d __attribute__((ext_vector_type(4)));

// C = A B for m x m matrices in LDS (row stride LDM) on the FP64 matrix
// cores: the matrices are zero-padded to mp = 16 ceil(m / 16) and every wave
// computes 16 x 16 output tiles with v_mfma_f64_16x16x4f64 (A fragment: lane l
// holds A[l % 16][l / 16], B fragment: B[l / 16][l % 16], accumulator element v
// of lane l is C[4 v + l / 16][l % 16], as measured on gfx950).  The padding of A and B must be zero;
// the padding of C is written as zero.  C must not alias A or B.
// one 16 x 16 output tile with NK = mp / 4 steps; all fragments are loaded
// before the dependent MFMA chain starts
template <int NK>
__device__ __forceinline__ void mfma_tile(double* __restrict__ C, const double* __restrict__ A,
                                          const double* __restrict__ B, int ti, int tj, int li, int lk) {
  double a[NK], b[NK];
#pragma unroll
  for (int q = 0; q < NK; ++q) {
    a[q] = A[(ti + li) * LDM + 4 * q + lk];
    b[q] = B[(4 * q + lk) * LDM + tj + li];
  }
  v4d acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int q = 0; q < NK; ++q) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a[q], b[q], acc, 0, 0, 0);
#pragma unroll
  for (int v = 0; v < 4; ++v) C[(ti + 4 * v + lk) * LDM + tj + li] = acc[v];
}

__device__ void mat_mul(double* C, const double* A, const double* B, int m) {
  const int mp = (m + 15) & ~15;
  const int nt = mp >> 4;
  const int wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const int lane = threadIdx.x & 63, li = lane & 15, lk = lane >> 4;
  for (int t = wave; t < nt * nt; t += nw) {
    const int ti = (t / nt) << 4, tj = (t % nt) << 4;
    if (nt == 1)
      mfma_tile<4>(C, A, B, ti, tj, li, lk);
    else if (nt == 2)
      mfma_tile<8>(C, A, B, ti, tj, li, lk);
    else
      mfma_tile<12>(C, A, B, ti, tj, li, lk);
  }
  __syncthreads();
}

// One Gauss-Jordan step for row r of the augmented system [P | Q] (row k and
// the pivot row trade places; the pivot row is normalised, every other row
// loses its multiple of it).  Columns c = g, g + ngrp, ... (at most U per
// thread); all loads are issued before the stores.
template <int U>
__device__ __forceinline__ void gj_row(const double* __restrict__ P0, const double* __restrict__ Q0,
                                       double* __restrict__ P1, double* __restrict__ Q1, int m, int k, int piv,
                                       double inv, int r, int g, int ngrp) {
  const int sr = r == k ? piv : (r == piv ? k : r);
  const double f = P0[sr * LDM + k];
  double pp[U], ps[U], qp[U], qs[U];
  // column indices clamped into the matrix, so that no load is conditional
  // (values past column m - 1 are loaded but never stored)
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int cp = min(k + 1 + g + u * ngrp, m - 1), cq = min(g + u * ngrp, m - 1);
    pp[u] = P0[piv * LDM + cp];
    ps[u] = P0[sr * LDM + cp];
    qp[u] = Q0[piv * LDM + cq];
    qs[u] = Q0[sr * LDM + cq];
  }
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int cp = k + 1 + g + u * ngrp, cq = g + u * ngrp;
    const double vp = pp[u] * inv, vq = qp[u] * inv;
    if (cp < m) P1[r * LDM + cp] = r == k ? vp : ps[u] - f * vp;
    if (cq < m) Q1[r * LDM + cq] = r == k ? vq : qs[u] - f * vq;
  }
}

__device__ void pade_coeffs(int deg, double* b) {
  b[0] = 1.0;
  for (int jj = 1; jj <= deg; ++jj) b[jj] = b[jj - 1] * (double)(deg - jj + 1) / ((double)jj * (double)(2 * deg - jj + 1));
}

// Row i of H = G R^{-1} by forward substitution, the row held in registers
// (NB >= m unrolls every index to a constant; no loads are conditional: S and
// R are zero-padded and R[j][j] = 1 for j >= m, so the columns past m - 1 hold
// harmless values that are never used):
//   H[i][j] = (G[i][j] - sum_{k<j} H[i][k] R[k][j]) / R[j][j],
//   G[i][j] = S[i][j] + R[j][j] R[i][j+1].
template <int NB>
__device__ __forceinline__ void hess_row(int i, const double* __restrict__ Sm, const double* __restrict__ Rm,
                                         const double* __restrict__ rinv, double* __restrict__ Hs) {
  double h[NB];
#pragma unroll
  for (int j = 0; j < NB; ++j) {
    double g = Sm[i * LDM + j] + Rm[j * LDM + j] * Rm[i * LDM + j + 1];
    double g2 = 0.0;
#pragma unroll
    for (int k = 0; k + 1 < j; k += 2) {
      g -= h[k] * Rm[k * LDM + j];
      g2 -= h[k + 1] * Rm[(k + 1) * LDM + j];
    }
    if (j & 1) g -= h[j - 1] * Rm[(j - 1) * LDM + j];
    h[j] = (g + g2) * rinv[j];
  }
#pragma unroll
  for (int j = 0; j < NB; ++j) Hs[i * LDM + j] = h[j];
}

// H_m (m x m, row stride LDM) from the per-step log of k_upd.  With x_j the
// vector swept in step j, the log gives x_j = V R[:, j] (R upper triangular:
// column j holds c^(j) above the diagonal alpha_j, alpha_0 = 1) and
// A x_j = V s^(j) + alpha_j x_{j+1}, so A V R = V G with
// G[:, j] = s^(j) + alpha_j R[:, j+1], and H = G R^{-1}: every row of H by
// forward substitution, one row per thread.  R[:, m] comes from the log of
// step m when the process broke down there, else from the partials of
// <v_i, x_m>, |x_m|^2 that step m-1 left.  Returns h_{m,m-1} = alpha_m.
__device__ __forceinline__ double hess_from_log(const DevTables& T, const KrylovWs& ws, int p, int rhs, int problem,
                                                int nchunks, int M, int m, double* __restrict__ Hs,
                                                double* __restrict__ Sm, double* __restrict__ Rm,
                                                double* __restrict__ rinv, double* red, double* hv) {
  const int tid = threadIdx.x;
  const int ldl = 2 * M + 1;
  const double* L = ws.lg + (int64_t)p * (M + 1) * ldl;
  const int Mp = (int)min((int64_t)M, T.inst[problem >> 1].ndof);
  const bool brk = m < Mp;
  __shared__ double hn_s;
  const int mp = (m + 15) & ~15;
  // zero S and R on mp x (mp + 1), unit diagonal of R past m - 1
  for (int e = tid; e < mp * (mp + 1); e += blockDim.x) {
    const int r = e / (mp + 1), c = e - r * (mp + 1);
    Sm[r * LDM + c] = 0.0;
    Rm[r * LDM + c] = (r == c && r >= m) ? 1.0 : 0.0;
  }
  __syncthreads();
  const int n = (brk ? m + 1 : m) * ldl;
  // all loads of the log (and of the partials below) in flight before any is used
  constexpr int LOGQ = ((SGDG_MAX_M + 1) * (2 * SGDG_MAX_M + 1) + 255) / 256;
  double xs[LOGQ];
#pragma unroll
  for (int q = 0; q < LOGQ; ++q) {
    const int e = tid + q * 256;
    xs[q] = e < n ? L[e] : 0.0;
  }
  if (!brk) {
    const double* part = (m & 1) ? ws.part3 : ws.part2;
    reduce_partials(part, (int64_t)rhs * nchunks + T.pchunk0[problem], T.pnchunk[problem], M + 2, m + 1, red, hv);
    if (tid < m) Rm[tid * LDM + m] = hv[tid];
    if (tid == 0) {
      double n2 = hv[m];
      for (int i = 0; i < m; ++i) n2 -= hv[i] * hv[i];
      hn_s = sqrt(fmax(n2, 0.0));
    }
  }
#pragma unroll
  for (int q = 0; q < LOGQ; ++q) {
    const int e = tid + q * 256;
    if (e >= n) break;
    const int j = e / ldl, i = e - j * ldl;
    const double x = xs[q];
    if (j == m) {
      if (i >= M && i < M + m) Rm[(i - M) * LDM + m] = x;
      if (i == 2 * M) hn_s = x;
    } else if (i < M) {
      if (i <= j) Sm[i * LDM + j] = x;
    } else if (i < 2 * M) {
      if (i - M < j) Rm[(i - M) * LDM + j] = x;
    } else {
      Rm[j * LDM + j] = j ? x : 1.0;
    }
  }
  // the diagonal of R was scattered by other waves' threads
  __syncthreads();
  if (tid < mp) rinv[tid] = tid < m ? 1.0 / (tid ? Rm[tid * LDM + tid] : 1.0) : 1.0;
  __syncthreads();
  if (tid < m) {
    if (mp == 16)
      hess_row<16>(tid, Sm, Rm, rinv, Hs);
    else if (mp == 32)
      hess_row<32>(tid, Sm, Rm, rinv, Hs);
    else
      hess_row<48>(tid, Sm, Rm, rinv, Hs);
  }
  __syncthreads();
  return hn_s;
}

// H is assembled from the step log of the k_upd launches.
__global__ __launch_bounds__(256) void k_expm(DevTables T, int ninst, int nchunks, int M, double hstep, KrylovWs ws,
                                              sgdg_stats* __restrict__ stats) {
  const int p = blockIdx.x;
  const int species = p & 1;
  const int inst = (p >> 1) % ninst;
  const int rhs = (p >> 1) / ninst;
  const int tid = threadIdx.x;
  if (species >= T.inst[inst].S) return;
  const int m = ws.m[p];
  const double beta = ws.beta[p];
  __shared__ __align__(16) double Am[MM * LDM], A2[MM * LDM], A4[MM * LDM], A6[MM * LDM], Tm[MM * LDM],
      Um[MM * LDM], Vm[MM * LDM];
  __shared__ double b[14], fac[MM];
  __shared__ int deg_s, s_s, piv_s;
  __shared__ double nrm_s;
  if (m == 0) {
    for (int i = tid; i < M; i += blockDim.x) ws.y[(int64_t)p * M + i] = 0.0;
    if (stats && tid == 0) {
      stats[p].krylov_m = 0;
      stats[p].h_next = 0.0;
      stats[p].status = isfinite(beta) ? SGDG_OK : SGDG_ERR_NONFINITE;
    }
    return;
  }
  // only the Hessenberg part of H is ever written (rows <= column + 1); every
  // work matrix starts zero on the padded square used by mat_mul
  const double hnext = hess_from_log(T, ws, p, rhs, inst * 2 + species, nchunks, M, m, Tm, A2, A4, fac, Vm, Um);
  const int mp = (m + 15) & ~15;
  for (int e = tid; e < mp * mp; e += blockDim.x) {
    const int r = e / mp, c = e - r * mp, q = r * LDM + c;
    const bool in = r < m && c < m && r <= c + 1;
    Am[q] = in ? hstep * Tm[q] : 0.0;
    A2[q] = A4[q] = A6[q] = Tm[q] = Um[q] = Vm[q] = 0.0;
  }
  __syncthreads();
  // ||A||_1: column sums in parallel, maximum by thread 0
  if (tid < m) {
    double cs = 0.0;
    for (int r = 0; r < m; ++r) cs += fabs(Am[r * LDM + tid]);
    fac[tid] = cs;
  }
  __syncthreads();
  if (tid == 0) {
    double nrm = 0.0;
    for (int c = 0; c < m; ++c) nrm = fmax(nrm, fac[c]);
    const double th[5] = {1.495585217958292e-2, 2.539398330063230e-1, 9.504178996162932e-1, 2.097847961257068e0,
                          5.371920351148152e0};
    const int dg[5] = {3, 5, 7, 9, 13};
    int deg = 13, s = 0;
    for (int q = 0; q < 4; ++q)
      if (nrm <= th[q]) {
        deg = dg[q];
        break;
      }
    if (deg == 13 && nrm > th[4]) s = (int)ceil(log2(nrm / th[4]));
    if (!isfinite(nrm)) s = 0;
    deg_s = deg;
    s_s = s;
    nrm_s = nrm;
    pade_coeffs(deg, b);
  }
  __syncthreads();
  const int deg = deg_s, s = s_s;
  if (s > 0) {
    const double sc = ldexp(1.0, -s);
    for (int e = tid; e < m * m; e += blockDim.x) Am[(e / m) * LDM + e % m] *= sc;
    __syncthreads();
  }
  mat_mul(A2, Am, Am, m);
  if (deg >= 5) mat_mul(A4, A2, A2, m);
  if (deg >= 7) mat_mul(A6, A4, A2, m);
  if (deg == 13) {
    // U = A [A6 (b13 A6 + b11 A4 + b9 A2) + b7 A6 + b5 A4 + b3 A2 + b1 I]
    // V =    A6 (b12 A6 + b10 A4 + b8 A2) + b6 A6 + b4 A4 + b2 A2 + b0 I
    for (int e = tid; e < m * m; e += blockDim.x) {
      const int q = (e / m) * LDM + e % m;
      Tm[q] = b[13] * A6[q] + b[11] * A4[q] + b[9] * A2[q];
    }
    __syncthreads();
    mat_mul(Um, A6, Tm, m);
    for (int e = tid; e < m * m; e += blockDim.x) {
      const int r = e / m, c = e % m, q = r * LDM + c;
      Um[q] += b[7] * A6[q] + b[5] * A4[q] + b[3] * A2[q] + (r == c ? b[1] : 0.0);
      Tm[q] = b[12] * A6[q] + b[10] * A4[q] + b[8] * A2[q];
    }
    __syncthreads();
    mat_mul(Vm, A6, Tm, m);
    for (int e = tid; e < m * m; e += blockDim.x) {
      const int r = e / m, c = e % m, q = r * LDM + c;
      Vm[q] += b[6] * A6[q] + b[4] * A4[q] + b[2] * A2[q] + (r == c ? b[0] : 0.0);
      Tm[q] = Um[q];
    }
    __syncthreads();
    mat_mul(Um, Am, Tm, m);
  } else {
    // U = A (sum over odd j of b_j A^(j-1)), V = sum over even j of b_j A^j, powers A2, A4, A6, A8 = A4 A4
    if (deg == 9) mat_mul(Vm, A4, A4, m);  // A8 kept in Vm until consumed
    for (int e = tid; e < m * m; e += blockDim.x) {
      const int r = e / m, c = e % m, q = r * LDM + c;
      const double I = (r == c) ? 1.0 : 0.0;
      double u = b[1] * I + b[3] * A2[q];
      double v = b[0] * I + b[2] * A2[q];
      if (deg >= 5) {
        u += b[5] * A4[q];
        v += b[4] * A4[q];
      }
      if (deg >= 7) {
        u += b[7] * A6[q];
        v += b[6] * A6[q];
      }
      if (deg >= 9) {
        u += b[9] * Vm[q];
        v += b[8] * Vm[q];
      }
      Tm[q] = u;
      A2[q] = v;  // A2 no longer needed after this point
    }
    __syncthreads();
    mat_mul(Um, Am, Tm, m);
    for (int e = tid; e < m * m; e += blockDim.x) {
      const int q = (e / m) * LDM + e % m;
      Vm[q] = A2[q];
    }
    __syncthreads();
  }
  // solve (V - U) R = (V + U) by Gauss-Jordan elimination with partial
  // pivoting on the augmented rows [P | Q]; one step per column, written to a
  // second buffer pair so that every step needs a single barrier.  Columns of
  // P at or left of the pivot column are not carried (they are unit vectors).
  double* P0 = A4;
  double* Q0 = A6;
  double* P1 = Tm;
  double* Q1 = A2;
  for (int e = tid; e < m * m; e += blockDim.x) {
    const int q = (e / m) * LDM + e % m;
    P0[q] = Vm[q] - Um[q];
    Q0[q] = Vm[q] + Um[q];
  }
  __syncthreads();
  // thread -> (row, column group): rows r < m in the low bits, columns
  // strided by the number of groups (no integer division in the loop)
  const int rsh = m <= 32 ? 5 : 6;
  const int my_r = tid & ((1 << rsh) - 1), my_g = tid >> rsh, ngrp = blockDim.x >> rsh;
  for (int k = 0; k < m; ++k) {
    // pivot: largest |P[r][k]| for r >= k; every wave finds it on its own (lane
    // r - k holds row r, m <= 64) with one 32-bit key per lane: the magnitude
    // rounded to FP32 with its low 6 mantissa bits replaced by 63 - lane, so the
    // maximum key is the largest magnitude and, among magnitudes equal to ~17
    // bits, the lowest row.  Every lane also forms the reciprocal of its entry
    // (inf for a zero, which is never chosen unless the system is singular);
    // the pivot's is then read from its lane.
    int piv;
    double inv;
    {
      const int lane = tid & 63, r = k + lane;
      const double x = r < m ? P0[r * LDM + k] : 0.0;
      const unsigned key = r < m ? (__float_as_uint((float)fabs(x)) & ~63u) | (unsigned)(63 - lane) : 0u;
      const double rx = 1.0 / x;
      const int pl = 63 - (int)(wave_max_u32(key) & 63u);
      piv = k + pl;
      inv = readlane_f64(rx, pl);
    }
    if (my_r < m) {
      if (rsh == 5)
        gj_row<4>(P0, Q0, P1, Q1, m, k, piv, inv, my_r, my_g, ngrp);
      else
        gj_row<12>(P0, Q0, P1, Q1, m, k, piv, inv, my_r, my_g, ngrp);
    }
    __syncthreads();
    double* t = P0;
    P0 = P1;
    P1 = t;
    t = Q0;
    Q0 = Q1;
    Q1 = t;
  }
  // square s times
  double* R = Q0;
  double* Rn = Um;
  for (int q = 0; q < s; ++q) {
    mat_mul(Rn, R, R, m);
    double* t = R;
    R = Rn;
    Rn = t;
  }
  for (int i = tid; i < M; i += blockDim.x) ws.y[(int64_t)p * M + i] = i < m ? R[i * LDM] : 0.0;
  if (stats && tid == 0) {
    bool fin = isfinite(beta);
    for (int i = 0; i < m; ++i) fin = fin && isfinite(R[i * LDM]);
    stats[p].krylov_m = m;
    stats[p].h_next = hnext;
    stats[p].status = fin ? SGDG_OK : SGDG_ERR_NONFINITE;
  }
}

// w = gamma V_m y
template <class TV>
__global__ __launch_bounds__(CHUNK) void k_comb(DevTables T, int ninst, int64_t total, int M, KrylovWs ws,
                                                double* __restrict__ w) {
  const int c = blockIdx.x, rhs = blockIdx.y, tid = threadIdx.x, nrhs = gridDim.y;
  const Chunk ch = T.chunks[c];
  const int p = prob_of(rhs, ninst, ch);
  __shared__ double ys[SGDG_MAX_M];
  const int m = ws.m[p];
  const double beta = ws.beta[p];
  if (tid < m) ys[tid] = ws.y[(int64_t)p * M + tid];
  __syncthreads();
  if (tid >= ch.count) return;
  const int64_t g = ch.start + tid;
  double acc = 0.0;
  for (int i = 0; i < m; ++i) acc += ys[i] * (double)vec<TV>(ws, i, nrhs, rhs, total)[g];
  w[rhs * total + g] = m == 0 ? beta * 0.0 : beta * acc;
}

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

static size_t sweep_bytes(int prec) { return prec == SGDG_FP64 ? 8 : 4; }

size_t krylov_ws_bytes(const sgdg_plan* plan, int M, int nrhs) {
  const size_t tot = (size_t)plan->total * nrhs;
  const size_t np = (size_t)nrhs * plan->ninst * 2;
  size_t b = 0;
  b += align256((size_t)(M + 1) * tot * sweep_bytes(plan->prec));        // V
  b += align256(plan->prec == SGDG_BF16_SWEEP ? tot * 2 : 0);             // Vb
  b += align256(tot * sweep_bytes(plan->prec));                           // wy
  b += 3 * align256((size_t)nrhs * plan->nchunks * (M + 2) * 8);          // part1, part2, part3
  b += align256(np * (M + 1) * (2 * M + 1) * 8);                          // step log
  b += align256(np * M * 8);                                              // y
  b += align256(np * 8);                                                  // beta
  b += 2 * align256(np * 4);                                              // m, done
  return b;
}

KrylovWs krylov_carve(const sgdg_plan* plan, int M, int nrhs, void* base) {
  const size_t tot = (size_t)plan->total * nrhs;
  const size_t np = (size_t)nrhs * plan->ninst * 2;
  char* p = (char*)base;
  auto take = [&](size_t bytes) {
    char* r = p;
    p += align256(bytes);
    return (void*)r;
  };
  KrylovWs ws{};
  ws.V = take((size_t)(M + 1) * tot * sweep_bytes(plan->prec));
  void* vb = take(plan->prec == SGDG_BF16_SWEEP ? tot * 2 : 0);
  ws.Vb = plan->prec == SGDG_BF16_SWEEP ? (uint16_t*)vb : nullptr;
  ws.wy = take(tot * sweep_bytes(plan->prec));
  ws.part1 = (double*)take((size_t)nrhs * plan->nchunks * (M + 2) * 8);
  ws.part2 = (double*)take((size_t)nrhs * plan->nchunks * (M + 2) * 8);
  ws.part3 = (double*)take((size_t)nrhs * plan->nchunks * (M + 2) * 8);
  ws.lg = (double*)take(np * (M + 1) * (2 * M + 1) * 8);
  ws.y = (double*)take(np * M * 8);
  ws.beta = (double*)take(np * 8);
  ws.m = (int32_t*)take(np * 4);
  ws.done = (int32_t*)take(np * 4);
  return ws;
}

template <class P, class TV, class TY>
static void run_typed(const sgdg_plan* plan, int nrhs, double h, int M, const double* v, double* w,
                      const KrylovWs& ws, sgdg_stats* stats, hipStream_t s, const KrylovIn* in) {
  const dim3 grid((unsigned)plan->nchunks, (unsigned)nrhs), blk(CHUNK);
  if (in) v = in->vbuf;
  hipLaunchKernelGGL(k_init, grid, blk, 0, s, plan->dev, plan->nchunks, plan->ninst, plan->total, M, v, ws,
                     in ? in->vbuf : nullptr, in ? in->x : nullptr, in ? in->y : nullptr, in ? in->a : 0.0);
  hipLaunchKernelGGL((k_norm<TV>), grid, blk, 0, s, plan->dev, plan->nchunks, plan->ninst, plan->total, M, v, ws);
  {
    for (int j = 0; j < M; ++j) {
      const void* xin = ws.Vb ? (const void*)ws.Vb : (const void*)((const TV*)ws.V + (size_t)j * nrhs * plan->total);
      // sweep w = A x_j fused with the chunk partials <v_i, w>, i < j, and <x_j, w>
      const DotArgs da{ws.V, ws.part1, j, M + 2, plan->nchunks, nrhs, plan->total};
      launch_apply_dots<P, TV>(plan, nrhs, xin, ws.wy, da, s);
      // the smallest bucket JB > j: the kernel loads and multiplies JB basis
      // entries per element (measured per launch: 6.0 / 6.5 / 8.6 us at
      // JB = 8 / 16 / 32 for the 2 x 5184-DOF plan)
#define SGDG_UPD(JB)                                                                                               \
  hipLaunchKernelGGL((k_upd<TV, TY, JB>), grid, blk, 0, s, plan->dev, plan->nchunks, plan->ninst, plan->total, M, j, \
                     ws)
      if (j < 8)
        SGDG_UPD(8);
      else if (j < 16)
        SGDG_UPD(16);
      else if (j < 20)
        SGDG_UPD(20);
      else if (j < 24)
        SGDG_UPD(24);
      else if (j < 28)
        SGDG_UPD(28);
      else if (j < 32)
        SGDG_UPD(32);
      else if (j < 40)
        SGDG_UPD(40);
      else
        SGDG_UPD(SGDG_MAX_M);
#undef SGDG_UPD
    }
  }
  hipLaunchKernelGGL(k_expm, dim3((unsigned)(nrhs * plan->ninst * 2)), dim3(256), 0, s, plan->dev, plan->ninst,
                     plan->nchunks, M, h, ws, stats);
  hipLaunchKernelGGL((k_comb<TV>), grid, blk, 0, s, plan->dev, plan->ninst, plan->total, M, ws, w);
}

sgdg_status krylov_run(const sgdg_plan* plan, int nrhs, double h, int M, const double* v, double* w,
                       const KrylovWs& ws, sgdg_stats* stats, hipStream_t s, const KrylovIn* in) {
  switch (plan->prec) {
    case SGDG_FP64: run_typed<PrecF64, double, double>(plan, nrhs, h, M, v, w, ws, stats, s, in); break;
    case SGDG_FP32_SWEEP: run_typed<PrecF32, float, float>(plan, nrhs, h, M, v, w, ws, stats, s, in); break;
    default: run_typed<PrecBF16, float, float>(plan, nrhs, h, M, v, w, ws, stats, s, in); break;
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "krylov_expv launch");
  return SGDG_OK;
}

}  // namespace sgdg

using namespace sgdg;

extern "C" sgdg_status krylov_expv(const sgdg_plan* plan, int32_t nrhs, double h, int32_t M, const double* v, double* w,
                                   void* workspace, size_t workspace_bytes, sgdg_stats* stats, void* stream) {
  if (!plan) return fail(SGDG_ERR_ARG, "krylov_expv: null plan");
  if (nrhs < 1 || nrhs > 65535) return fail(SGDG_ERR_ARG, "krylov_expv: nrhs must be in 1..65535");
  if (M < 1 || M > SGDG_MAX_M) return fail(SGDG_ERR_ARG, "krylov_expv: M must be in 1..48");
  if (!std::isfinite(h)) return fail(SGDG_ERR_ARG, "krylov_expv: h must be finite");
  if (!v || !w || !workspace) return fail(SGDG_ERR_ARG, "krylov_expv: null device pointer");
  if (workspace_bytes < krylov_ws_bytes(plan, M, nrhs)) return fail(SGDG_ERR_ARG, "krylov_expv: workspace too small");
  KrylovWs ws = krylov_carve(plan, M, nrhs, workspace);
  return krylov_run(plan, nrhs, h, M, v, w, ws, stats, (hipStream_t)stream);
}
