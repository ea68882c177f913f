// Krylov workspace layout and launchers shared by krylov.hip and iif2.hip.
#pragma once

#include "internal.h"

namespace sgdg {

// happy breakdown: h_{j+1,j} <= KRYLOV_BREAKDOWN_REL * ||A_s||_inf ends the Arnoldi process
constexpr double KRYLOV_BREAKDOWN_REL = 1e-12;

// Device-side view of a Krylov workspace (one carve-up of a caller buffer).
struct KrylovWs {
  void* V;           // (M+1) basis vectors: [i][rhs][total], FP64 or FP32
  uint16_t* Vb;      // BF16 sweep copy of the current basis vector (BF16 plans)
  void* wy;          // sweep output [rhs][total]: FP64 or FP32
  double* part1;     // per-chunk partial sums [rhs][chunk][M+2]
  double* part2;     // part2 / part3: the pair that carries <v_i, x_{j+1}> between steps
  double* part3;
  double* lg;        // [problem][M+1][2M+1]: per-step (s, c, alpha), problem = (rhs*ninst + inst)*2 + species
  double* y;         // [problem][M]: first column of exp(h H_m)
  double* beta;      // [problem]
  int32_t* m;        // [problem]: Krylov dimension reached
  int32_t* done;     // [problem]: 0, or 1 + the first Arnoldi step that no longer runs
};

size_t krylov_ws_bytes(const sgdg_plan* plan, int M, int nrhs);
KrylovWs krylov_carve(const sgdg_plan* plan, int M, int nrhs, void* base);

// Optional input combination: the first kernel forms v = x + a y (x may be
// null: v = a y) and stores it in vbuf, which then serves as v.
struct KrylovIn {
  double* vbuf;
  const double* x;
  const double* y;
  double a;
};

// w = exp(h A) v for nrhs plan vectors (v, w FP64, may alias).
sgdg_status krylov_run(const sgdg_plan* plan, int nrhs, double h, int M, const double* v, double* w,
                       const KrylovWs& ws, sgdg_stats* stats, hipStream_t s, const KrylovIn* in = nullptr);

}  // namespace sgdg
