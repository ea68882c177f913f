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
  double* H;         // [problem][(M+1) x M], problem = (rhs*ninst + inst)*2 + species (persistent form)
  double* lg;        // [problem][M+1][2M+1]: per-step (s, c, alpha) of the launch-per-step form
  double* y;         // [problem][M]: first column of exp(h H_m)
  double* beta;      // [problem]
  int32_t* m;        // [problem]: Krylov dimension reached
  int32_t* done;     // [problem]: 0, or 1 + the first Arnoldi step that no longer runs
  uint32_t* bar;     // persistent Arnoldi: [0] arrivals, [1] generation, [2] error flag
};

size_t krylov_ws_bytes(const sgdg_plan* plan, int M, int nrhs);
KrylovWs krylov_carve(const sgdg_plan* plan, int M, int nrhs, void* base);

// Persistent Arnoldi (arnoldi.hip): all M steps of every problem in one
// launch with grid-wide barriers, when enabled by SGDG_ARNOLDI=persistent,
// the plan's chunks are all in one staged sweep list and the grid fits the
// device at one workgroup per compute unit.  Returns false (and launches
// nothing) otherwise.
bool arnoldi_persistent(const sgdg_plan* plan, int nrhs, int M, const KrylovWs& ws, hipStream_t s);

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
