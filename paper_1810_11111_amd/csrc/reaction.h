// Reaction transforms: plan-level tables and launchers (reaction.hip), used by iif2.hip.
#pragma once

#include <functional>

#include "internal.h"

namespace sgdg {

// One level block of an r-dimensional sparse grid of level N (r = 1..d),
// canonical order, extents c(l)(k+1).
struct RBlk {
  int64_t start;
  int32_t size;
  int32_t lsum;
  int32_t lev[SGDG_MAX_D];
};

// Per-instance constants of the reaction transforms.
struct RInst {
  int32_t N, K1, S, nq, np1, n1, d, pad;
  int64_t seg;    // offset of the instance in a plan vector
  int64_t ndof;
  int64_t EL_off;    // into EL: [(L * np1 + q) * K1 + p] = level-L cell basis p at finest 1D Gauss point q
  int64_t EH_off;    // into EH: [(q * (N + 1) + l) * K1 + p] = hierarchical function (l, cell of q at level l, p) at point q
  int64_t w_off;     // into w1: Gauss weight times h_N of 1D point q
  int64_t mats_off;  // into mats: ML, MR, cL, cR (each 16 doubles, row length K1)
  int32_t blk_off[SGDG_MAX_D + 1];  // into rblk, r-dim grid
  int32_t nblk[SGDG_MAX_D + 1];
  int32_t id_off[SGDG_MAX_D + 1];   // into rid: (N+1)^r entries, -1 if |l|_1 > N
  int32_t ntile[SGDG_MAX_D];        // fibre tiles of stage m per (species, prefix)
  int64_t be_off[SGDG_MAX_D + 1];   // into rbe: block (index in the r-dim grid) of every element
  int64_t gdof[SGDG_MAX_D + 1];     // DOFs of the r-dim grid
  int64_t npre[SGDG_MAX_D + 1];     // np1^m
  int64_t X_off[SGDG_MAX_D];        // per-rhs workspace offsets (doubles) of expansion outputs, m = 1..d-1
  int64_t Y_off[SGDG_MAX_D];        // of contraction outputs, m = 1..d-1
  double rx[2][4][4];
};

struct RTables {
  RInst* inst = nullptr;
  RBlk* rblk = nullptr;
  int32_t* rid = nullptr;
  int32_t* rbe = nullptr;
  double* EL = nullptr;
  double* EH = nullptr;
  double* w1 = nullptr;
  double* mats = nullptr;
  int64_t* cum_x[SGDG_MAX_D] = {};  // fibre tiles of stage m per instance (prefix sums, ninst+1)
  int64_t* cum_fin = nullptr;       // workgroups of the final stage (partial residual sums)
};

// A tile of the last-axis kernel: nl consecutive lines from prefix pre0 of one instance.
struct LineTask {
  int32_t inst, nl;
  int64_t pre0;
};

// Lines of one instance in a wave-form class: lpr lines per round (one
// round: every wave of a workgroup takes its lines once).
struct WaveLines {
  int inst, lpr;
  int64_t lines;
};

// One launch of the last-axis kernel per class and number of inputs (1, 2):
// wave form, instances of the same degree and species count (N: the largest
// level); LDS-tile form, instances of the same degree, level and species
// count (one LDS layout).
struct LineClass {
  int K1 = 0, N = 0, S = 0;
  std::vector<LineTask> tasks[3];
  LineTask* dev[3] = {};
  size_t lds[3] = {};  // dynamic LDS bytes
  int threads[3] = {}; // workgroup size
  // wave form (d >= 2, N <= RX_WLINE_MAXN): a tile is `rounds` rounds of an
  // instance's lines (lpr: lines per round of the class's largest instance);
  // its grid-stride launch has wgcu workgroups per compute unit and one of
  // two register budgets.  Launch shapes only: every line is computed the
  // same way whatever the shape.
  bool wave = false;
  int lpr = 0;
  int rounds[3] = {};
  int wgcu[3] = {};
  int waves[3] = {};  // 0: the compiler's register allocation; 3: at most 168 VGPRs (three waves per SIMD)
  size_t cap_tasks[3] = {};                     // room in dev[nin] (tiles of one round)
  std::vector<WaveLines> lines;                 // every instance's lines of its last axis
};

struct RHost {
  RTables dev;
  std::vector<std::vector<int64_t>> cum_x;
  std::vector<int64_t> cum_fin;
  std::vector<LineClass> lclass;
  int lam[SGDG_MAX_D] = {};    // stage m splits each fibre's points into 2^lam chunks (lam <= 8)
  int llane[SGDG_MAX_D] = {};  // of which the low llane chunk bits are lane bits (lam - llane <= 2)
  int xs_lds[SGDG_MAX_D] = {};  // stage m stages each tile's hierarchical block in LDS (bytes; 0: it does not)
  int lm[5] = {};               // [K1]: levels held per fibre by the expansion / contraction kernels (7, 9, 11)
  int64_t rws = 0;           // doubles of reaction workspace per right-hand side
  int max_n1 = 0, max_np1 = 0;
  int k1mask = 0;  // bit K1 set when an instance has degree K1 - 1
  int ncu = 0;  // compute units of the plan's device
  bool supported = true;
};

bool reaction_supported(const sgdg_plan* plan);
int64_t reaction_final_fibres(const sgdg_plan* plan);

enum RxMode { RX_F = 0, RX_RESID = 1, RX_CORR = 2, RX_LOCAL = 3 };

// local implicit stage: per-point Newton on u - dt2 f(u) = w
constexpr double RX_LOCAL_TOL = 1e-15;
constexpr int RX_LOCAL_MAX_ITER = 30;

// One reaction pass over nrhs right-hand sides.
//   RX_F    : F = P f(R U)
//   RX_RESID: F = P f(R U), G = U - dt2 F - W, per-final-workgroup |G|^2 into part
//   RX_CORR : U <- U - P[(I - dt2 J_f(R U))^{-1} R G]
//   RX_LOCAL: Gout = P u, u solving u - dt2 f(u) = R U at every point (U holds W)
// Instances with conv[rhs * ninst + inst] != 0 are skipped (conv may be null);
// conv[nprob] counts the flags set (nprob = ninst * nrhs), and a launch
// returns at once when all are.
struct RxArgs {
  double* U;
  const double* G;
  double* F;
  double* Gout;
  const double* W;
  double* part;  // [rhs][final workgroup]
  const int32_t* conv;
  int32_t nprob;
  double dt2;
  double* rws;  // reaction workspace base
};
// mark (optional) is called before every kernel launch with its stage (0
// expansion, 1 last axis, 2 contraction) and once after the last with -1.
void reaction_pass(const sgdg_plan* plan, int nrhs, RxMode mode, const RxArgs& a, hipStream_t s,
                   const std::function<void(int)>* mark = nullptr);
int64_t reaction_ws_doubles(const sgdg_plan* plan);

// Launch shapes of the last-axis kernels (autotuning).  Classes are the plan's
// (degree, level, species) groups of instances.
int reaction_line_classes(const sgdg_plan* plan);
const LineClass& reaction_line_class(const sgdg_plan* plan, int c);
sgdg_status reaction_set_line_shape(sgdg_plan* plan, int c, int nin, int rounds, int wgcu, int waves);
// Only the last-axis launch of class c of a pass (inputs: the reaction workspace).
void reaction_line_stage(const sgdg_plan* plan, int nrhs, RxMode mode, const RxArgs& a, hipStream_t s, int c);

}  // namespace sgdg
