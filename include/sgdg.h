/*
 * sgdg.h -- C ABI of the sparse-grid Krylov IIF discontinuous Galerkin library
 * for AMD MI355X (gfx950).
 *
 * Method: Liu, Cheng, Chen, Zhang, "Krylov implicit integration factor
 * discontinuous Galerkin methods on sparse grids for high dimensional
 * reaction-diffusion equations" (arXiv:1810.11111).
 *
 * Problem (Sec. 1, eq. 1.1 on the periodic unit cube, diagonal diffusion):
 *     u_t = div(K(x) grad u) + f(u),   K = diag(D_s k_ii(x_i)),  x in [0,1]^d,
 * discretised in space by the symmetric interior-penalty DG method on the
 * sparse multiwavelet space V_N^k (Sec. 2.1, eqs. 2.6-2.11) -- giving
 * dU/dt = A U + F(U) (Sec. 3, eq. 3.1) -- and in time by the Krylov IIF2 scheme
 * (Sec. 3, eqs. 3.5, 3.7, 3.8).
 *
 * Conventions for every call
 *   - Every function returns an sgdg_status.  No C++ exception crosses the ABI.
 *   - Argument errors are detected on the host before any device work is
 *     queued; nothing is written in that case.  sgdg_last_error() returns a
 *     message for the calling thread's last failure.
 *   - "device pointer" arguments are HIP device allocations owned by the
 *     caller; "host pointer" arguments are ordinary memory owned by the caller.
 *     The library never frees caller memory.
 *   - Device work is queued asynchronously on `stream` (a hipStream_t passed as
 *     void*; NULL means the default stream).  Results are valid after the
 *     caller synchronises that stream.
 *   - A plan is immutable after sg_dg_build and may be used from several
 *     threads; calls that share a workspace must not overlap in time.
 *
 * Vector layout ("plan vector")
 *   A plan holds `ninst` independent instances.  Instance i contributes
 *   nspecies_i * ndof_i consecutive entries starting at offset_i (see
 *   sg_dg_info); inside an instance the species are consecutive blocks of
 *   ndof_i entries.  Inside a species the DOFs are in the canonical order:
 *     - level blocks l in N_0^d with |l|_1 <= N (eq. 2.9), sorted by |l|_1 and
 *       then lexicographically in (l_1, ..., l_d);
 *     - inside a block a row-major d-dimensional array, axis m of extent
 *       c(l_m)(k+1) with c(0) = 1, c(l) = 2^(l-1), index j_m (k+1) + p_m for
 *       cell j_m and 0-based wavelet/Legendre index p_m (eqs. 2.6, 2.8).
 *   Calls that take `nrhs` operate on nrhs plan vectors stored one after the
 *   other (right-hand side r starts at r * total, total from sg_dg_total).
 *
 * Basis (eq. 2.6): level 0 is sqrt(2p+1) P_p(2x-1); level n >= 1, cell j is
 * 2^((n-1)/2) psi_p(2^(n-1) x - j) with psi_p the Alpert multiwavelets on [0,1],
 * fixed by vanishing moments of order k+p and a sign rule (the highest nonzero
 * Legendre coefficient on the right half is positive).
 */
#ifndef SGDG_H
#define SGDG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  SGDG_OK = 0,
  SGDG_ERR_ARG = 1,         /* invalid argument (nothing was done)                  */
  SGDG_ERR_ALLOC = 2,       /* device or host allocation failed                     */
  SGDG_ERR_HIP = 3,         /* a HIP runtime call failed                            */
  SGDG_ERR_UNSUPPORTED = 4, /* valid request outside what the library implements   */
  SGDG_ERR_NOCONV = 5,      /* implicit stage did not reach its tolerance (stats)   */
  SGDG_ERR_NONFINITE = 6    /* a NaN/Inf was produced or consumed (stats)           */
} sgdg_status;

/* Precision of the operator sweeps (the matrix-free products A x).  Inner
 * products, norms, the Hessenberg exponential, the Krylov combination and the
 * implicit-stage residual are always FP64 (FP64 accumulation).            */
typedef enum {
  SGDG_FP64 = 0,       /* sweeps, Krylov basis and state in FP64                 */
  SGDG_FP32_SWEEP = 1, /* sweep input/output and Krylov basis in FP32, FP32 sums  */
  SGDG_BF16_SWEEP = 2  /* sweep input BF16, output and Krylov basis FP32, FP32 sums */
} sgdg_precision;

/* Diagonal diffusion factor of one axis: k_ii(x) = a0 + a1 sin(2 pi freq x + phase).
 * Must be positive on [0,1] (eq. 1.2 bounds).                               */
typedef struct {
  double a0, a1, freq, phase;
} sgdg_kdiag;

/* One instance (Sec. 2.1 scheme on [0,1]^d). */
typedef struct {
  int32_t d;          /* space dimension, 1..6                                  */
  int32_t n;          /* sparse-grid level N >= 0 (|l|_1 <= N), 2^N finest cells */
  int32_t k;          /* polynomial degree, 1..3 (the scheme needs k >= 1)       */
  int32_t nspecies;   /* 1 or 2                                                 */
  double sigma;       /* interior penalty sigma (<= 0 selects 20); penalty sigma/h_N */
  double D[2];        /* per-species diffusion multiplier D_s > 0                */
  const sgdg_kdiag* kdiag; /* NULL: k_ii = 1; else d entries, read during build only */
  /* Reaction f_s(u0, u1) = sum_{a,b=0..3} rx[s][a][b] u0^a u1^b (degree <= 3 used). */
  double rx[2][4][4];
  /* Boundary: 0 periodic; 1 zero Dirichlet on every face (boundary faces take
   * the one-sided trace times the outward normal as jump and the one-sided
   * flux as average, the convention stated after eq. 2.11).                */
  int32_t bc;
  int32_t pad;
} sgdg_desc;

/* A separable 1D factor of initial data, for sg_dg_project. */
typedef struct {
  int32_t kind;   /* 0: cos(2 pi a x + b);  1: indicator of [a, b)              */
  int32_t pad;
  double a, b;
} sgdg_factor1d;

/* Per-problem statistics written on the device (one entry per right-hand
 * side, instance and species slot: index (r * ninst + i) * 2 + s).          */
typedef struct {
  int32_t krylov_m;     /* Krylov dimension reached (< M after a breakdown)     */
  int32_t newton_iters; /* corrections applied by the implicit stage            */
  double h_next;        /* h_{m+1,m}: a-posteriori Krylov size estimate         */
  double residual;      /* final ||G||_2 of the implicit stage (per instance)    */
  int32_t status;       /* SGDG_OK, SGDG_ERR_NOCONV or SGDG_ERR_NONFINITE         */
  int32_t pad;
} sgdg_stats;

typedef struct sgdg_plan sgdg_plan;

/* Message for the calling thread's last non-OK status (static storage). */
const char* sgdg_last_error(void);

/* ------------------------------------------------------------------------ */
/* Plan construction (host; uploads tables once -- the paper notes the 1D
 * integrals are assembled once before the time evolution, Sec. 4 intro).
 * descs: host array of ninst descriptors; every instance must have the same
 * d.  prec: sweep precision of the plan.  *out receives the plan.
 * Builds the 1D hierarchical SIPG operators (eq. 2.10 bilinear form, faces of
 * Omega_N, penalty sigma/h_N), the level-block tables and the Gauss tables
 * (k+1 points per axis in every finest cell) used by the reaction transforms,
 * on the current HIP device.  Errors: SGDG_ERR_ARG, _ALLOC, _HIP.           */
sgdg_status sg_dg_build(const sgdg_desc* descs, int32_t ninst, int32_t prec, sgdg_plan** out);

/* Frees the plan and its device tables (synchronises the device first). */
sgdg_status sg_dg_destroy(sgdg_plan* plan);

/* Sizes of instance `inst`: DOFs per species (eq. 2.9 index set), offset of
 * the instance in a plan vector, Gauss points per species ((k+1) 2^N)^d.     */
sgdg_status sg_dg_info(const sgdg_plan* plan, int32_t inst, int64_t* ndof, int64_t* offset,
                       int64_t* npoints);

/* Entries of one plan vector (sum over instances of nspecies * ndof). */
sgdg_status sg_dg_total(const sgdg_plan* plan, int64_t* total);

/* Device workspace (bytes) needed by krylov_expv and by iif2_step / iif3_step for Krylov
 * dimension M (1..48) and nrhs right-hand sides.                            */
sgdg_status sg_dg_workspace_size(const sgdg_plan* plan, int32_t M, int32_t nrhs, size_t* krylov_bytes,
                                 size_t* iif2_bytes);

/* Host export of the canonical DOF order of instance `inst`: level, cell and
 * 0-based index p for every DOF and axis (host arrays of ndof*d int32,
 * row-major [dof][axis]).                                                   */
sgdg_status sg_dg_layout(const sgdg_plan* plan, int32_t inst, int32_t* lev, int32_t* cell, int32_t* p);

/* L2 projection (Sec. 2.2, u_h(0) = P u) of amp * prod_m g_m(x_m) onto the
 * sparse space of instance `inst`; factors: host array of d descriptors;
 * out: host array of ndof doubles (overwritten).  Computed on the host with a
 * 16-point Gauss rule per finest cell.                                      */
sgdg_status sg_dg_project(const sgdg_plan* plan, int32_t inst, double amp, const sgdg_factor1d* factors,
                          double* out);

/* ||A_s||_inf (max absolute row sum) of species s of instance inst (host). */
sgdg_status sg_dg_norm_inf(const sgdg_plan* plan, int32_t inst, int32_t species, double* out);

/* ------------------------------------------------------------------------ */
/* y = A x for nrhs plan vectors (Sec. 2.1, eq. 2.10 with the orthonormal
 * mass matrix; Sec. 4 "unidirectional principle"):
 *   A = - sum_i D_s (I x .. x B_i x .. x I) restricted to |l|_1 <= N,
 * applied matrix-free from the 1D hierarchical operators B_i.
 * x, y: device pointers of nrhs*total elements, not aliased.  Element type
 * by plan precision: FP64 -> double/double, FP32 -> float/float, BF16 ->
 * bfloat16 (uint16 bits)/float.  Errors: SGDG_ERR_ARG, SGDG_ERR_HIP.        */
sgdg_status sg_dg_apply(const sgdg_plan* plan, int32_t nrhs, const void* x, void* y, void* stream);

/* How sg_dg_apply (and rk_step's operator products) evaluate y = A x; the
 * Krylov products keep the chunked form (they fuse the Arnoldi inner
 * products into it).
 *   1: chunked gather -- every output walks its rows of the 1D operators.
 *   2: fibre form, FP64 plans only -- direction by direction, each fibre of
 *      the sparse grid along that direction (the DOFs sharing every other
 *      axis' level and position; it spans levels 0..b of the axis, b = N -
 *      the other levels' sum) is taken from hierarchical coefficients to the
 *      level-b cell-Legendre basis by the two-scale relation, multiplied by
 *      the block-tridiagonal level-b form of B_i (Sec. 2.1, eq. 2.10
 *      restricted to that space) and transformed back: x read once per
 *      direction, O(1) work per value.  Same operator, different rounding
 *      (agrees with form 1 to a few units of 1e-13 |A||x|).  The first
 *      selection builds its tables on the device (allocates).
 *   3: form 2 with every fibre of budget b >= 2 split at level b/2 (the
 *      two-level path that form 2 takes for fibres longer than one LDS
 *      tile: coarse levels synthesised first, subtrees as tiles, coarse
 *      levels analysed last); selectable for testing.
 *   0: automatic -- form 2 for FP64 plans of at least 2^19 DOFs whose
 *      species segments all exceed the staged sweeps' LDS, else form 1
 *      (what sg_dg_build selects).
 * Synchronises the device.  Errors: SGDG_ERR_ARG (null plan, unknown form),
 * SGDG_ERR_UNSUPPORTED (forms 2, 3 on an FP32/BF16 plan), SGDG_ERR_ALLOC /
 * SGDG_ERR_HIP (the plan then keeps form 1).                                */
sgdg_status sg_dg_sweep_form(sgdg_plan* plan, int32_t form);

/* w ~ exp(h A) v (Sec. 3, eq. 3.8): Arnoldi (eq. 3.7) with M products per
 * species, instance and right-hand side, classical Gram-Schmidt with one
 * re-orthogonalisation pass, happy breakdown when h_{j+1,j} <= 1e-12 ||A_s||_inf,
 * then gamma V_m exp(h H_m) e_1 with exp by Pade approximation with scaling
 * and squaring (Higham 2005, degrees 3..13).  M is clamped to the DOF count
 * of each species.  v, w: device FP64 plan vectors (nrhs*total), may alias.
 * workspace: device buffer of at least krylov_bytes (sg_dg_workspace_size).
 * stats: device array of nrhs*ninst*2 sgdg_stats or NULL.                  */
sgdg_status krylov_expv(const sgdg_plan* plan, int32_t nrhs, double h, int32_t M, const double* v, double* w,
                        void* workspace, size_t workspace_bytes, sgdg_stats* stats, void* stream);

/* F(U) = P f(R U) + S (Sec. 5: reconstruction at the Gauss points of the
 * finest mesh, pointwise f, Gauss quadrature back to the sparse space; S the
 * projected forcing of the time level, device plan vectors, or NULL).  U, F,
 * S: device FP64 plan vectors (nrhs*total); F must not alias U or S;
 * workspace as for iif2_step.                                              */
sgdg_status sgdg_reaction(const sgdg_plan* plan, int32_t nrhs, const double* U, double* F, const double* S,
                          void* workspace, size_t workspace_bytes, void* stream);

/* Measurement helper: the reaction pass of sgdg_reaction (F = P f(R U), no
 * source) with a HIP event recorded on `stream` before every kernel launch
 * and after the last; synchronises the stream and returns the elapsed time of
 * each launch.  stage_ms, stage_kind: host arrays of *nstage entries (in:
 * capacity, out: launches timed); stage_kind[i] is 0 for an expansion stage
 * (axes 0..d-2), 1 for the last-axis kernel (transform, pointwise f,
 * transform), 2 for a contraction stage, in launch order.  Arguments as for
 * sgdg_reaction.  Errors: SGDG_ERR_ARG, _UNSUPPORTED, _HIP.                 */
sgdg_status sgdg_reaction_timed(const sgdg_plan* plan, int32_t nrhs, const double* U, double* F, void* workspace,
                                size_t workspace_bytes, float* stage_ms, int32_t* stage_kind, int32_t* nstage,
                                void* stream);

/* One IIF2 step (Sec. 3, eq. 3.5):
 *   W = exp(A dt) (U + dt/2 F(U));  solve U' - dt/2 F(U') = W;  U <- U'.
 * The implicit stage iterates U <- U - P[(I - dt/2 J_f(u_q))^{-1} (R G)_q],
 * G = U - dt/2 F(U) - W, from U = W + dt/2 F(U^n), until
 * ||G||_2 <= newton_tol * max(1, ||W||_2) per instance and right-hand side or
 * newton_max corrections (status SGDG_ERR_NOCONV in stats; U holds the last
 * iterate).  U: device FP64 plan vectors, updated in place.  Fcache: device
 * FP64 plan vectors holding F(U) on entry (computed by sgdg_reaction for the
 * first step) and F(U') on return; NULL recomputes it every step.
 * S_next: projected forcing at the new time level (F = P f(R U) + S), device
 * plan vectors or NULL; a source needs Fcache (the old level's F includes
 * its own source).  U, Fcache and S_next must not alias (SGDG_ERR_ARG).
 * workspace: at least iif2_bytes.  stats: device array or NULL.            */
sgdg_status iif2_step(const sgdg_plan* plan, int32_t nrhs, double dt, int32_t M, double* U, double* Fcache,
                      const double* S_next, double newton_tol, int32_t newton_max, void* workspace,
                      size_t workspace_bytes, sgdg_stats* stats, void* stream);

/* iif2_step without a caller workspace and without any device allocation, for
 * callers that cannot allocate: code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc.  The workspace is a fixed 64 MiB
 * device array inside the library (one per GPU, held from library load until
 * the process ends); plans, M and nrhs whose iif2_step workspace
 * (sg_dg_workspace_size) exceeds 64 MiB return SGDG_ERR_UNSUPPORTED before any
 * device work.  Every call on a GPU shares that GPU's array: calls that
 * overlap in time on one GPU (other streams, other threads) race and must be
 * serialised by the caller.  Arguments and results as iif2_step.            */
sgdg_status iif2_step_noalloc(const sgdg_plan* plan, int32_t nrhs, double dt, int32_t M, double* U, double* Fcache,
                              const double* S_next, double newton_tol, int32_t newton_max, sgdg_stats* stats,
                              void* stream);

/* One IIF3 step (Sec. 3, eq. 3.6; coefficients 5/12, 2/3, -1/12 of eq. 3.4):
 *   W = exp(A dt)(U + 2/3 dt F(U)) + exp(2 A dt)(-1/12 dt F(U^{n-1}))
 * (each exponential by its own Krylov process of dimension M), then the
 * implicit stage of iif2_step with coefficient 5/12 dt in place of dt/2, from
 * U = W + 5/12 dt F(U).  U: device FP64 plan vectors, updated in place.
 * Fcur: F(U^n) on entry, F(U^{n+1}) on return.  Fprev: F(U^{n-1}) on entry,
 * F(U^n) on return.  The three must not alias.  A run starts with one
 * iif2_step (the scheme needs F at two earlier levels), then F(U^0) becomes
 * Fprev.  S_next: forcing at the new level as for iif2_step.  workspace: at
 * least iif2_bytes.  stats: as iif2_step (the Krylov entries describe the
 * exp(A dt) process).  Errors as iif2_step.                                 */
sgdg_status iif3_step(const sgdg_plan* plan, int32_t nrhs, double dt, int32_t M, double* U, double* Fcur, double* Fprev,
                      const double* S_next, double newton_tol, int32_t newton_max, void* workspace,
                      size_t workspace_bytes, sgdg_stats* stats, void* stream);

/* One IIF2 step with the local implicit stage (a variant, not the paper's
 * scheme: the "local implicit property" Sec. 5 names as future work).  As
 * iif2_step, except that the stage is solved independently at every Gauss
 * point of Omega_N, u - dt/2 f(u) = R W (Newton per point from u = w, at most
 * 30 corrections, |g| <= 1e-15 max(1, |w|)), and projected, U = P u; no
 * global iteration.  Equal to iif2_step for linear f.  Fcache is required.
 * stats: Krylov entries only.                                               */
sgdg_status iif2_step_local(const sgdg_plan* plan, int32_t nrhs, double dt, int32_t M, double* U, double* Fcache,
                            const double* S_next, void* workspace, size_t workspace_bytes, sgdg_stats* stats,
                            void* stream);

/* One explicit Runge-Kutta step of dU/dt = A U + F(U) (Sec. 4, Table 1: the
 * RK2 and RK3 comparators whose step limit shows the stiffness of A).  order 2:
 * U1 = U + dt L(U), U <- (U + U1 + dt L(U1)) / 2; order 3 (Shu-Osher): U1 as
 * before, U2 = 3/4 U + 1/4 (U1 + dt L(U1)), U <- 1/3 U + 2/3 (U2 + dt L(U2)),
 * L(U) = A U + F(U).  FP64 plans only (SGDG_ERR_UNSUPPORTED otherwise).  U:
 * device FP64 plan vectors, updated in place.  workspace: at least
 * iif2_bytes for M = 1.  Errors: SGDG_ERR_ARG, _UNSUPPORTED, _HIP.          */
sgdg_status rk_step(const sgdg_plan* plan, int32_t nrhs, double dt, int32_t order, double* U, void* workspace,
                    size_t workspace_bytes, void* stream);

/* ---- Launch-shape autotuning ------------------------------------------------
 * The last axis of the reaction transforms (Sec. 5: F(U) = P f(R U), applied
 * axis by axis) runs, for every class of instances with the same degree and
 * species count and N <= 8 (d >= 2), as tiles of whole lines walked by one
 * grid-stride launch.  Its shape -- lines per tile (in rounds: one round
 * gives every wave of a workgroup its lines once) and workgroups per compute
 * unit -- changes only which workgroup computes which line: every value is
 * computed the same way, so results are bit for bit the same for every
 * shape.  A shape also picks one of two builds of the kernel: the compiler's
 * register allocation (waves 0) or at most 168 VGPRs, i.e. three waves per
 * SIMD, spilling what does not fit (waves 3).  These calls change a plan's
 * launch shapes: no other call may use the plan while they run. */
#define SGDG_TUNE_MAXCLASS 16
typedef struct {
  int32_t nclass;                                  /* classes reported (wave-form last axis only)      */
  int32_t k[SGDG_TUNE_MAXCLASS], n[SGDG_TUNE_MAXCLASS], nspecies[SGDG_TUNE_MAXCLASS];  /* n: largest level */
  int32_t cls[SGDG_TUNE_MAXCLASS];                 /* class index for sg_dg_line_shape                  */
  int32_t rounds[SGDG_TUNE_MAXCLASS][2];           /* chosen rounds per tile, one and two inputs/point */
  int32_t wgcu[SGDG_TUNE_MAXCLASS][2];             /* chosen workgroups per compute unit               */
  int32_t waves[SGDG_TUNE_MAXCLASS][2];            /* chosen register budget: 0 or 3 (see above)       */
  float ms_default[SGDG_TUNE_MAXCLASS][2];         /* one launch at the shape found on entry           */
  float ms_best[SGDG_TUNE_MAXCLASS][2];            /* one launch at the chosen shape                   */
  int32_t from_cache[SGDG_TUNE_MAXCLASS][2];       /* 1: taken from this process's earlier tuning      */
} sgdg_tune_report;

/* Times every candidate shape (rounds 1, 2, 4, 8, 16, 32 x workgroups per CU
 * 4, 8, 16, 32 with waves 0, then waves 3 with each workgroup count at the
 * best rounds) of each class's last-axis launch for nrhs right-hand sides,
 * one and two inputs per point, with HIP events on `stream` (synchronising
 * it), and keeps the fastest.  Choices are cached per process by GPU
 * architecture and compute-unit count, (degree, level, species), inputs,
 * nrhs and line count; a cached class is set without timing.  If the
 * environment variable SGDG_TUNE_CACHE names a file, the cache is also read
 * from it (once per process) and every new choice is appended to it (one line
 * "arch cus K1 N species inputs nrhs lines rounds wgcu waves"; a line without
 * the last field reads as waves 0).  workspace: at least iif2_bytes for M = 1 and nrhs
 * (sg_dg_workspace_size); its contents are overwritten.  report: host
 * pointer, may be NULL.  Errors: SGDG_ERR_ARG, _UNSUPPORTED (no reaction
 * tables for this plan), _HIP.                                              */
sgdg_status sg_dg_tune(sgdg_plan* plan, int32_t nrhs, void* workspace, size_t workspace_bytes,
                       sgdg_tune_report* report, void* stream);

/* Sets the shape of class `cls`, `ninputs` (1: F and residual passes, 2: the
 * stage correction) to `rounds` rounds per tile (1..64), `wgcu` workgroups
 * per compute unit (1..64) and register budget `waves` (0 or 3).  Errors:
 * SGDG_ERR_ARG, _UNSUPPORTED (the class does not run the wave form), _HIP.   */
sgdg_status sg_dg_line_shape(sgdg_plan* plan, int32_t cls, int32_t ninputs, int32_t rounds, int32_t wgcu,
                             int32_t waves);

#ifdef __cplusplus
}
#endif

#endif /* SGDG_H */
