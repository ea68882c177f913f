// Internal declarations shared by the host plan builder and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/sgdg.h"

#define SGDG_MAX_D 6
#define SGDG_MAX_M 48
#define SGDG_MAX_K 3

namespace sgdg {

struct FibreData;  // fibre form of the operator sweep (fibre.hip)

// One level block of one species of one instance.
struct GBlock {
  int64_t start;  // first element in a plan vector
  int32_t size;
  int32_t inst;
  int32_t species;
  int32_t lsum;  // |l|_1
  int32_t lev[SGDG_MAX_D];
  int32_t ext[SGDG_MAX_D];  // c(l_m)(k+1)
};

// A contiguous piece (<= CHUNK elements) of one species segment; every
// element of a chunk belongs to blocks b0..b1 of that segment.
struct Chunk {
  int64_t start;
  int32_t count;    // <= CHUNK * APPLY_G / g
  int32_t b0, b1;
  int32_t inst;
  int32_t species;
  int32_t problem;  // inst * 2 + species
  int32_t g;        // lanes per output in the staged sweep (APPLY_G..64); g / APPLY_G in the global one
  int32_t pc0, pnc; // first chunk and number of chunks of this chunk's problem (species segment)
};

// Per-instance constants seen by the kernels.
struct InstDev {
  int32_t N, k, S, nb;
  int64_t offset, ndof;
  double D[2];
  int32_t blkid_off;              // into blkid: (N+1)^d entries, -1 where |l|_1 > N
  int32_t gblk_off;               // global index of this instance's species-0 block 0
  int32_t bcsr_off[SGDG_MAX_D];   // into BCsr table per direction
  int32_t pow[SGDG_MAX_D];        // (N+1)^(d-1-i)
  int32_t n1;                     // (k+1) 2^N
  int32_t rx_off;                 // unused placeholder for alignment
  double rx[2][4][4];
  double anorm[2];                // ||A_s||_inf
};

// Cell-block CSR of a 1D hierarchical operator: for target cell t (cell
// index c = 0 for level 0, 2^(l-1)+j for level l >= 1) the source cells
// src[cptr[t] .. cptr[t+1]) in ascending order, each with a (k+1)x(k+1)
// block val[e][pt][ps] of B(v_source, v_target).
struct BCsr {
  int64_t cptr_off;  // into cptr (ncell + 1 entries)
  int64_t src_off;   // into src (block index)
  int64_t val_off;   // into val / valf (scalar index of block 0)
  int32_t ncell;
  int32_t k;
  int32_t nnzb;      // number of cell blocks (length of src)
  int32_t pad;
};

// Rows of one direction's 1D operator that a chunk's outputs use: target
// cells tlo .. tlo + nrow - 1, i.e. CSR entries elo .. elo + nent - 1 (the
// staged sweep copies only these rows, their source cells and block values).
struct StageRange {
  int32_t tlo, nrow, elo, nent;
};

// Everything the staged sweep reads before its first copy, one record per
// entry of a staged chunk list (one scalar load round instead of a chain of
// chunk -> instance -> operator lookups).
struct SweepTask {
  int64_t start, seg, ndof;      // chunk start, species segment start, segment length
  int32_t cid, count, g, inst, species, b0, b1, ntab, blkid_off;
  uint32_t dup;                  // bit i: direction i shares an earlier direction's staged copy
  int64_t cp[SGDG_MAX_D];        // staged rows of direction i: T.cptr + cp, T.src + sp, block values + vp
  int64_t sp[SGDG_MAX_D];
  int64_t vp[SGDG_MAX_D];
  int32_t nrow[SGDG_MAX_D], nent[SGDG_MAX_D], tlo[SGDG_MAX_D], elo[SGDG_MAX_D];
};

struct DevTables {
  GBlock* gblk = nullptr;
  StageRange* srange = nullptr;  // [chunk][SGDG_MAX_D]
  Chunk* chunks = nullptr;
  InstDev* inst = nullptr;
  int32_t* blkid = nullptr;
  int64_t* lstart = nullptr;  // per (instance, local block): start inside a species segment
  BCsr* bcsr = nullptr;
  int32_t* cptr = nullptr;
  int32_t* src = nullptr;
  double* val = nullptr;
  float* valf = nullptr;
  int32_t* pchunk0 = nullptr;  // [inst*2+s]: first chunk of the species segment
  int32_t* pnchunk = nullptr;  // [inst*2+s]: its number of chunks
};

struct HostInstance {
  sgdg_desc desc;
  std::vector<sgdg_kdiag> kdiag;  // d entries (a0=1,a1=0 when none)
  int64_t ndof = 0, offset = 0, npoints = 0;
  std::vector<std::vector<int>> blocks;  // level tuples, canonical order
  std::vector<int64_t> bstart;           // start inside a species segment
  std::vector<int32_t> bsize;
  // 1D operator per direction (cell-block CSR, host copy)
  std::vector<int> dir_tab;  // index into plan's op tables per direction
  double anorm[2] = {0, 0};
};

struct Op1D {  // host cell-block CSR
  int N, k;
  std::vector<int32_t> cptr, src;
  std::vector<double> val;  // nnzb * (k+1)^2
  std::vector<double> kd;   // kdiag descriptor used (a0,a1,freq,phase), for sharing
  double sigma;
  int bc;                   // 0 periodic, 1 zero Dirichlet
};

}  // namespace sgdg

struct sgdg_plan {
  int32_t ninst = 0, d = 0, prec = 0;
  int32_t device = 0;
  int64_t total = 0;
  int32_t nchunks = 0, nblocks = 0;
  std::vector<sgdg::HostInstance> inst;
  std::vector<sgdg::Op1D> ops;
  std::vector<sgdg::GBlock> gblk;
  std::vector<sgdg::Chunk> chunks;
  // chunk ids grouped by sweep kind: index k * SWEEP_TIERS + tier, tier 0 =
  // gathers from global memory, 1 = x segment and row tables staged in LDS,
  // 2 = block values staged as well
  std::vector<std::vector<int32_t>> chunk_lists;
  std::vector<int32_t*> dev_chunk_lists;
  std::vector<sgdg::SweepTask*> dev_tasks;  // staged lists: per entry, its SweepTask
  std::vector<int> list_lds;    // dynamic LDS bytes of the staged lists
  std::vector<sgdg::InstDev> instdev;
  std::vector<int32_t> pchunk0, pnchunk;  // host copies of the per-species chunk ranges
  sgdg::DevTables dev;
  std::vector<void*> allocations;
  // reaction tables (filled by the reaction module)
  void* rdata = nullptr;
  // fibre form of the operator sweep: tables (built on first selection) and
  // whether sg_dg_apply takes it
  sgdg::FibreData* fdata = nullptr;
  bool fibre_on = false;
};

namespace sgdg {

constexpr int CHUNK = 256;
constexpr int APPLY_LDS_BYTES_HOST = 160 * 1024;  // same budget as the staged sweep kernels
constexpr int SWEEP_TIERS = 3;
constexpr int APPLY_G = 4;  // lanes per output element in the staged sweeps (the least; rows with more work get more)
constexpr int APPLY_GMAX = 64;

// fibre form of the operator sweep (fibre.hip)
bool fibre_auto(const sgdg_plan* p);
sgdg_status fibre_build(sgdg_plan* p, bool test_split);
void fibre_destroy(sgdg_plan* p);
void launch_fibre(const sgdg_plan* p, int nrhs, const double* x, double* y, int64_t xs, int64_t ys, hipStream_t s);

// error reporting
sgdg_status fail(sgdg_status st, const std::string& msg);
sgdg_status hip_fail(hipError_t e, const char* what);

// host basis construction (host_basis.cpp)
void gauss01(int n, std::vector<double>& x, std::vector<double>& w);
void legendre01_all(int n, double x, double* val, double* der);  // orthonormal on [0,1], degrees 0..n
struct Basis1D {
  int k;
  std::vector<double> cL, cR;  // psi_p halves: (k+1)x(k+1), [p][q]
  std::vector<double> ML, MR;  // child coefficients from parent: [q_child][i_parent]
};
const Basis1D& basis1d(int k);
double hier_value(const Basis1D& b, int level, int j, int p, double x, bool deriv);

// 1D operator (host_operator.cpp)
struct CellMats {  // full-grid SIPG matrices on the finest cells
  bool constk = true;
  std::vector<double> kvol;      // per cell (one when k is constant): K1 x K1
  std::vector<double> face;      // per face e between cells e-1 and e (one when k is constant): 2K1 x 2K1
  std::vector<double> FB0, FB1;  // zero-Dirichlet faces at x = 0 (on cell 0) and x = 1 (on the last cell)
};
CellMats cell_mats(int N, int k, double sigma, const sgdg_kdiag& kd);
Op1D build_op1d(int N, int k, double sigma, const sgdg_kdiag& kd, int bc);
std::vector<double> build_ss_levels(const Op1D& op, std::vector<int64_t>& off, bool& uniform);

// enumeration helpers
__host__ __device__ inline int level_count(int l) { return l == 0 ? 1 : (1 << (l - 1)); }

}  // namespace sgdg
