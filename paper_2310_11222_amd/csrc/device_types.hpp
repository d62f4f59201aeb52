// Types and constants the device kernels share: solver limits, per-column
// solver state, the grid-reduction scratch and the split-row work list.
// Host-only declarations (graph handle, workspace, entry points) are in
// nvd_internal.hpp, which includes this file.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/nvd.h"

namespace nvd {

// ---------------------------------------------------------------------------
// limits and tuning constants
// ---------------------------------------------------------------------------
constexpr int kMaxTile = 64;        // columns per SpMM pass / solver tile
constexpr int kBS = 256;            // threads per block for the streaming kernels
constexpr int kGrp = 32;            // blocks per first-level reduction group
#ifndef NVD_MAX_BLOCKS
#define NVD_MAX_BLOCKS 8192
#endif
constexpr int kMaxBlocks = NVD_MAX_BLOCKS;   // grid cap for kernels that reduce
constexpr int kMaxDots = 6;         // dot products reduced by one kernel
constexpr int kRedStride = kMaxDots * 64;  // doubles per block in the reduction scratch
constexpr int kLongRow = 128;       // rows with more neighbours take the split-row path
constexpr int kSeg = 2048;          // neighbours per split-row segment

// per-column status codes (match nvd_status)
constexpr int kStOk = NVD_OK;
constexpr int kStNoconv = NVD_E_NOCONV;
constexpr int kStBreak = NVD_E_BREAKDOWN;

// ---------------------------------------------------------------------------
// per-column solver state for one tile (device memory)
// ---------------------------------------------------------------------------
struct ColState {
  double rho[kMaxTile];     // r^T z of the running CG
  double alpha[kMaxTile];
  double beta[kMaxTile];
  double bnorm2[kMaxTile];  // ||rhs||^2 of the running CG
  double obnorm2[kMaxTile]; // ||delta_bar||^2 (outer right-hand side)
  double orr[kMaxTile];     // latest outer ||r||^2 (projected, FP64)
  double mean[kMaxTile];    // mean removed by the last projection (1 component)
  double itol2[kMaxTile];   // stop threshold of the running CG: ||r||^2 <= itol2 * bnorm2
  double dots[kMaxDots][kMaxTile];  // dots of the last residual pass
  int active[kMaxTile];     // running CG still iterating
  int oactive[kMaxTile];    // pair not yet converged (outer level)
  int iters[kMaxTile];      // CG iterations, summed over inner solves
  int it_cur[kMaxTile];     // iterations of the running CG
  int status[kMaxTile];
  int refine[kMaxTile];
  int stall[kMaxTile];      // mixed: consecutive outer steps that stalled
  int fb[kMaxTile];         // mixed: handed to the FP64 solver, not yet run
  int fbdone[kMaxTile];     // mixed: finished by the FP64 solver (info flag)
  int n_active;             // count of active[] (host polls these five words)
  int n_oactive;
  int it_max;               // largest it_cur[] over the tile
  int n_fb;                 // count of fb[]
  double worst;             // largest rr / (rtol^2 bnorm2) over active columns
  // x += alpha p is applied by the direction kernel, for the iteration whose
  // update kernel ran: that kernel's last block advances xseq, and an update
  // kernel that found nothing active sets xdone = xseq instead.
  int xseq;
  int xdone;
};

// Two-level, fixed-order grid reduction scratch.
struct GridRed {
  double* part1;     // [kMaxBlocks][kMaxDots*kMaxTile]
  double* part2;     // [kMaxBlocks/kGrp][kMaxDots*kMaxTile]
  unsigned* tick1;   // [kMaxBlocks/kGrp]
  unsigned* tick2;   // [1]
};

// Split-row (long row) work list for the SpMM.
struct LongRows {
  int n_seg = 0;         // total segments (one block each)
  const int* seg_row = nullptr;    // row of segment s
  const int* seg_lo = nullptr;     // nnz range [lo, hi) of segment s
  const int* seg_hi = nullptr;
  const int* seg_first = nullptr;  // first segment of that row
  const int* seg_cnt = nullptr;    // segments of that row
  double* seg_part = nullptr;      // [n_seg][kMaxTile] partial sums
  unsigned* row_tick = nullptr;    // [n_seg] arrival counters (indexed by first seg)
};

}  // namespace nvd
