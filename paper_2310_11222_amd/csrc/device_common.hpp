// Device building blocks: column-wise block reductions and a deterministic
// two-level grid reduction (fixed summation order, so FP64 results repeat
// bit for bit run to run).
#pragma once

#include <hip/hip_runtime.h>

#include "nvd_internal.hpp"

namespace nvd {

__device__ __forceinline__ void st_agent(double* p, double v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double ld_agent(const double* p) {
  return __hip_atomic_load(const_cast<double*>(p), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
}

// Sum the per-thread values of ND dot products by column.  Thread t holds
// NE entries per dot; entry e = t*NE + v belongs to column e % T (T a power of
// two, T <= BS*NE).  On return sh[d*BS*NE + c], c < T, holds the block's sum
// for dot d and column c.  sh must hold ND*BS*NE doubles.
template <int BS, int ND, int NE>
__device__ __forceinline__ void block_reduce_cols(const double (&acc)[ND][NE],
                                                  int T, double* sh) {
  constexpr int M = BS * NE;
  const int t = threadIdx.x;
#pragma unroll
  for (int d = 0; d < ND; ++d)
#pragma unroll
    for (int v = 0; v < NE; ++v) sh[d * M + t * NE + v] = acc[d][v];
  __syncthreads();
  for (int half = M / 2; half >= T; half >>= 1) {
    for (int i = t; i < half; i += BS) {
#pragma unroll
      for (int d = 0; d < ND; ++d) sh[d * M + i] += sh[d * M + i + half];
    }
    __syncthreads();
  }
}

// Grid-wide reduction of ndt = ND*T values per block (vals, in LDS).  Blocks
// form groups of kGrp; the last block to arrive in a group sums the group's
// partials in block order, and the last group to finish sums the group
// results in group order.  Returns true in exactly one block, whose vals then
// hold the grid totals.  Every block of the grid must call it.
template <int BS>
__device__ bool grid_reduce(double* vals, int ndt, const GridRed& red) {
  __shared__ int s_last;
  const int b = blockIdx.x;
  const int nb = gridDim.x;
  const int grp = b / kGrp;
  const int ngrp = (nb + kGrp - 1) / kGrp;
  const int gsz = min(kGrp, nb - grp * kGrp);
  const int stride = kMaxDots * kMaxTile;
  for (int i = threadIdx.x; i < ndt; i += BS) st_agent(&red.part1[(size_t)b * stride + i], vals[i]);
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned t = atomicAdd(&red.tick1[grp], 1u);
    s_last = (t == (unsigned)(gsz - 1));
  }
  __syncthreads();
  if (!s_last) return false;
  __threadfence();
  for (int i = threadIdx.x; i < ndt; i += BS) {
    double s = 0.0;
    const double* p = red.part1 + (size_t)grp * kGrp * stride + i;
    for (int j = 0; j < gsz; ++j) s += ld_agent(p + (size_t)j * stride);
    st_agent(&red.part2[(size_t)grp * stride + i], s);
  }
  if (threadIdx.x == 0) red.tick1[grp] = 0u;
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned t = atomicAdd(red.tick2, 1u);
    s_last = (t == (unsigned)(ngrp - 1));
  }
  __syncthreads();
  if (!s_last) return false;
  __threadfence();
  for (int i = threadIdx.x; i < ndt; i += BS) {
    double s = 0.0;
    const double* p = red.part2 + i;
    for (int j = 0; j < ngrp; ++j) s += ld_agent(p + (size_t)j * stride);
    vals[i] = s;
  }
  if (threadIdx.x == 0) *red.tick2 = 0u;
  __syncthreads();
  return true;
}

// Recount the active flags (called by one block after it changed them).
__device__ __forceinline__ void recount_active(ColState* cs, int T) {
  __syncthreads();
  if (threadIdx.x == 0) {
    int a = 0, o = 0;
    for (int c = 0; c < T; ++c) {
      a += cs->active[c];
      o += cs->oactive[c];
    }
    cs->n_active = a;
    cs->n_oactive = o;
  }
}

template <typename V>
struct Vec16;
template <>
struct Vec16<double> {
  using type = double2;
  static constexpr int N = 2;
};
template <>
struct Vec16<float> {
  using type = float4;
  static constexpr int N = 4;
};

}  // namespace nvd
