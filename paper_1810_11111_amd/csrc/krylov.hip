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
// modified form), which needs three device-wide reductions per step instead
// of j+1; each reduction is a kernel boundary (cheap inside a captured graph):
//   sweep   : w = A v_j (the sg_dg_apply kernels) and, in the same
//             workgroups, the per-chunk partials <v_i, w>
//   k_upd1  : h1 = sum of partials, w1 = w - V h1, per-chunk <v_i, w1>, |w1|^2
//   k_upd2  : h2, w2 = w1 - V h2, |w2|^2 = |w1|^2 - |h2|^2, v_{j+1} = w2 / |w2|
// Partial sums are reduced in a fixed order, so every workgroup of a problem
// computes bit-identical Hessenberg entries and breakdown decisions.
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

__device__ __forceinline__ int prob_of(int rhs, int ninst, const Chunk& ch) { return (rhs * ninst + ch.inst) * 2 + ch.species; }

template <class TV>
__device__ __forceinline__ const TV* vec(const KrylovWs& ws, int i, int nrhs, int rhs, int64_t total) {
  return (const TV*)ws.V + ((int64_t)i * nrhs + rhs) * total;
}

// ||v||^2 partial per chunk; resets the per-problem state.
__global__ __launch_bounds__(CHUNK) void k_init(DevTables T, int nchunks, int ninst, int64_t total, int M,
                                                const double* __restrict__ v, KrylovWs ws) {
  const int c = blockIdx.x, rhs = blockIdx.y, tid = threadIdx.x;
  const Chunk ch = T.chunks[c];
  double x = 0.0;
  if (tid < ch.count) {
    double a = v[rhs * total + ch.start + tid];
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
    if (c == 0 && rhs == 0) {
      ws.bar[0] = 0u;
      ws.bar[2] = 0u;
    }
    if (c == T.pchunk0[ch.problem]) {
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
  const int c0 = T.pchunk0[ch.problem], nc = T.pnchunk[ch.problem];
  __shared__ double sb;
  if (tid == 0) {
    double t = 0.0;
    for (int q = 0; q < nc; ++q) t += ws.part1[((int64_t)rhs * nchunks + c0 + q) * (M + 2)];
    sb = sqrt(t);
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

// Deterministic chunk-level multi-dot: out[i] = sum over the chunk of
// V_i[e] * wl[e] for i < J, plus out[J] = sum wl[e]^2 when with_norm.
// Thread (i, s) of a J x S arrangement sums the elements e = s, s+S, ... so
// the loads of one column are coalesced across slices.
template <class TV>
__device__ __forceinline__ void chunk_dots(const KrylovWs& ws, int J, bool with_norm, int nrhs, int rhs,
                                           int64_t total, int64_t g0, int count, const double* wl, double* red,
                                           double* out) {
  const int tid = threadIdx.x;
  const int cols = J + (with_norm ? 1 : 0);
  const int S = CHUNK / cols;
  if (tid < cols * S) {
    const int i = tid / S, s = tid - i * S;
    double acc = 0.0;
    if (i < J) {
      const TV* v = vec<TV>(ws, i, nrhs, rhs, total) + g0;
      for (int e = s; e < count; e += S) acc += (double)v[e] * wl[e];
    } else {
      for (int e = s; e < count; e += S) acc += wl[e] * wl[e];
    }
    red[tid] = acc;
  }
  __syncthreads();
  if (tid < cols) {
    double t = 0.0;
    for (int q = 0; q < S; ++q) t += red[tid * S + q];
    out[tid] = t;
  }
  __syncthreads();
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

// h1 = <V, w>;  w1 = w - V h1;  partials <v_i, w1> and |w1|^2.
template <class TV, class TY>
__global__ __launch_bounds__(CHUNK) void k_upd1(DevTables T, int nchunks, int ninst, int64_t total, int M, int j,
                                                KrylovWs ws) {
  const int c = blockIdx.x, rhs = blockIdx.y, tid = threadIdx.x, nrhs = gridDim.y;
  const Chunk ch = T.chunks[c];
  const int p = prob_of(rhs, ninst, ch);
  if (ws.done[p]) return;
  const int c0 = T.pchunk0[ch.problem], nc = T.pnchunk[ch.problem];
  __shared__ double h[SGDG_MAX_M + 2], wl[CHUNK], red[CHUNK], out[SGDG_MAX_M + 2];
  reduce_partials(ws.part1, (int64_t)rhs * nchunks + c0, nc, M + 2, j + 1, red, h);
  if (c == c0 && tid <= j) ws.H[(int64_t)p * (M + 1) * M + tid * M + j] = h[tid];
  const int64_t g = ch.start + tid;
  double w1 = 0.0;
  if (tid < ch.count) {
    double acc = (double)((const TY*)ws.wy)[rhs * total + g];
    for (int i = 0; i <= j; ++i) acc -= h[i] * (double)vec<TV>(ws, i, nrhs, rhs, total)[g];
    w1 = acc;
    ws.w1[rhs * total + g] = w1;
  }
  wl[tid] = w1;
  __syncthreads();
  chunk_dots<TV>(ws, j + 1, true, nrhs, rhs, total, ch.start, ch.count, wl, red, out);
  if (tid <= j + 1) ws.part2[((int64_t)rhs * nchunks + c) * (M + 2) + tid] = out[tid];
}

// h2 = <V, w1>;  w2 = w1 - V h2;  h_{j+1,j} = |w2|;  v_{j+1} = w2 / h_{j+1,j}.
template <class TV>
__global__ __launch_bounds__(CHUNK) void k_upd2(DevTables T, int nchunks, int ninst, int64_t total, int M, int j,
                                                KrylovWs ws) {
  const int c = blockIdx.x, rhs = blockIdx.y, tid = threadIdx.x, nrhs = gridDim.y;
  const Chunk ch = T.chunks[c];
  const int p = prob_of(rhs, ninst, ch);
  if (ws.done[p]) return;
  const int c0 = T.pchunk0[ch.problem], nc = T.pnchunk[ch.problem];
  __shared__ double h[SGDG_MAX_M + 2], red[CHUNK];
  __shared__ double hn_s;
  reduce_partials(ws.part2, (int64_t)rhs * nchunks + c0, nc, M + 2, j + 2, red, h);
  if (tid == 0) {
    double n2 = h[j + 1];
    for (int i = 0; i <= j; ++i) n2 -= h[i] * h[i];
    hn_s = sqrt(fmax(n2, 0.0));
  }
  __syncthreads();
  const double hn = hn_s;
  double* Hp = ws.H + (int64_t)p * (M + 1) * M;
  if (c == c0 && tid <= j) Hp[tid * M + j] += h[tid];
  if (c == c0 && tid == 0) Hp[(j + 1) * M + j] = hn;
  const InstDev& I = T.inst[ch.inst];
  const int Mp = (int)min((int64_t)M, I.ndof);
  const bool stop = !(hn > KRYLOV_BREAKDOWN_REL * I.anorm[ch.species]) || (j + 1 >= Mp);
  if (stop) {
    if (c == c0 && tid == 0) {
      ws.m[p] = j + 1;
      ws.done[p] = 1;
    }
    return;
  }
  if (tid >= ch.count) return;
  const int64_t g = ch.start + tid;
  double acc = ws.w1[rhs * total + g];
  for (int i = 0; i <= j; ++i) acc -= h[i] * (double)vec<TV>(ws, i, nrhs, rhs, total)[g];
  const double x = acc / hn;
  ((TV*)ws.V)[((int64_t)(j + 1) * nrhs + rhs) * total + g] = (TV)x;
  if (ws.Vb) ws.Vb[rhs * total + g] = f_to_bf16((float)x);
}

// ---- exp(h H_m) e_1: Pade approximation with scaling and squaring ---------
// Higham, "The scaling and squaring method for the matrix exponential
// revisited", SIAM J. Matrix Anal. Appl. 26 (2005): degree m in {3,5,7,9,13}
// chosen from ||A||_1 against theta_m; for degree 13, A is scaled by 2^-s with
// s = ceil(log2(||A||_1 / theta_13)) and the result squared s times.
// [m/m] Pade coefficients b_j = (2m-j)! m! / ((2m)! j! (m-j)!) from the
// ratio b_j / b_{j-1} = (m-j+1) / (j (2m-j+1)).
constexpr int MM = SGDG_MAX_M;
constexpr int LDM = MM + 2;  // row stride of the LDS matrices: 16 consecutive rows hit distinct banks

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
                                       int r, int g, int ngrp) {
  const int sr = r == k ? piv : (r == piv ? k : r);
  const double inv = 1.0 / P0[piv * LDM + k];
  const double f = P0[sr * LDM + k];
  double pp[U], ps[U], qp[U], qs[U];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int cp = k + 1 + g + u * ngrp, cq = g + u * ngrp;
    pp[u] = cp < m ? P0[piv * LDM + cp] : 0.0;
    ps[u] = cp < m ? P0[sr * LDM + cp] : 0.0;
    qp[u] = cq < m ? Q0[piv * LDM + cq] : 0.0;
    qs[u] = cq < m ? Q0[sr * LDM + cq] : 0.0;
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

__global__ __launch_bounds__(256) void k_expm(DevTables T, int ninst, int M, double hstep, KrylovWs ws,
                                              sgdg_stats* __restrict__ stats) {
  const int p = blockIdx.x;
  const int species = p & 1;
  const int inst = (p >> 1) % ninst;
  const int tid = threadIdx.x;
  if (species >= T.inst[inst].S) return;
  const int m = ws.m[p];
  const double beta = ws.beta[p];
  const double* Hp = ws.H + (int64_t)p * (M + 1) * M;
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
  const int mp = (m + 15) & ~15;
  for (int e = tid; e < mp * mp; e += blockDim.x) {
    const int r = e / mp, c = e - r * mp, q = r * LDM + c;
    Am[q] = (r < m && c < m && r <= c + 1) ? hstep * Hp[r * M + c] : 0.0;
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
    // bits, the lowest row
    int piv;
    {
      const int lane = tid & 63, r = k + lane;
      unsigned key = 0u;
      if (r < m) key = (__float_as_uint((float)fabs(P0[r * LDM + k])) & ~63u) | (unsigned)(63 - lane);
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) key = max(key, (unsigned)__shfl_xor((int)key, off, 64));
      piv = k + 63 - (int)(key & 63u);
    }
    if (my_r < m) {
      if (rsh == 5)
        gj_row<4>(P0, Q0, P1, Q1, m, k, piv, my_r, my_g, ngrp);
      else
        gj_row<12>(P0, Q0, P1, Q1, m, k, piv, my_r, my_g, ngrp);
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
    stats[p].h_next = Hp[m * M + (m - 1)];
    stats[p].status = ws.bar[2] ? SGDG_ERR_HIP : (fin ? SGDG_OK : SGDG_ERR_NONFINITE);
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
  b += align256(tot * 8);                                                 // w1
  b += 2 * align256((size_t)nrhs * plan->nchunks * (M + 2) * 8);          // part1, part2
  b += align256(np * (M + 1) * M * 8);                                    // H
  b += align256(np * M * 8);                                              // y
  b += align256(np * 8);                                                  // beta
  b += 2 * align256(np * 4);                                              // m, done
  b += align256(64);                                                      // barrier words
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
  ws.w1 = (double*)take(tot * 8);
  ws.part1 = (double*)take((size_t)nrhs * plan->nchunks * (M + 2) * 8);
  ws.part2 = (double*)take((size_t)nrhs * plan->nchunks * (M + 2) * 8);
  ws.H = (double*)take(np * (M + 1) * M * 8);
  ws.y = (double*)take(np * M * 8);
  ws.beta = (double*)take(np * 8);
  ws.m = (int32_t*)take(np * 4);
  ws.done = (int32_t*)take(np * 4);
  ws.bar = (uint32_t*)take(64);
  return ws;
}

template <class P, class TV, class TY>
static void run_typed(const sgdg_plan* plan, int nrhs, double h, int M, const double* v, double* w,
                      const KrylovWs& ws, sgdg_stats* stats, hipStream_t s) {
  const dim3 grid((unsigned)plan->nchunks, (unsigned)nrhs), blk(CHUNK);
  hipLaunchKernelGGL(k_init, grid, blk, 0, s, plan->dev, plan->nchunks, plan->ninst, plan->total, M, v, ws);
  hipLaunchKernelGGL((k_norm<TV>), grid, blk, 0, s, plan->dev, plan->nchunks, plan->ninst, plan->total, M, v, ws);
  if (!arnoldi_persistent(plan, nrhs, M, ws, s)) {
    for (int j = 0; j < M; ++j) {
      const void* xin = ws.Vb ? (const void*)ws.Vb : (const void*)((const TV*)ws.V + (size_t)j * nrhs * plan->total);
      // sweep w = A v_j fused with the chunk partials <v_i, w>, i <= j
      const DotArgs da{ws.V, ws.part1, j, M + 2, plan->nchunks, nrhs, plan->total};
      launch_apply_dots<P, TV>(plan, nrhs, xin, ws.wy, da, s);
      hipLaunchKernelGGL((k_upd1<TV, TY>), grid, blk, 0, s, plan->dev, plan->nchunks, plan->ninst, plan->total, M, j,
                         ws);
      hipLaunchKernelGGL((k_upd2<TV>), grid, blk, 0, s, plan->dev, plan->nchunks, plan->ninst, plan->total, M, j, ws);
    }
  }
  hipLaunchKernelGGL(k_expm, dim3((unsigned)(nrhs * plan->ninst * 2)), dim3(256), 0, s, plan->dev, plan->ninst, M, h, ws,
                     stats);
  hipLaunchKernelGGL((k_comb<TV>), grid, blk, 0, s, plan->dev, plan->ninst, plan->total, M, ws, w);
}

sgdg_status krylov_run(const sgdg_plan* plan, int nrhs, double h, int M, const double* v, double* w,
                       const KrylovWs& ws, sgdg_stats* stats, hipStream_t s) {
  switch (plan->prec) {
    case SGDG_FP64: run_typed<PrecF64, double, double>(plan, nrhs, h, M, v, w, ws, stats, s); break;
    case SGDG_FP32_SWEEP: run_typed<PrecF32, float, float>(plan, nrhs, h, M, v, w, ws, stats, s); break;
    default: run_typed<PrecBF16, float, float>(plan, nrhs, h, M, v, w, ws, stats, s); break;
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
