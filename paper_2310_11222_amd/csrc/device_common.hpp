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

// Wait until this thread's outstanding memory operations have completed.
// Partials are written with agent-scope (coherent) stores; once they have
// completed they are visible to every XCD, so publishing them needs no L2
// write-back fence -- a full agent-scope fence per block would write back the
// whole L2 of the XCD, including the kernel's streaming output.
__device__ __forceinline__ void wait_stores() { __builtin_amdgcn_s_waitcnt(0); }

__device__ __forceinline__ unsigned ticket(unsigned* p) {
  return __hip_atomic_fetch_add(p, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Sum `count` rows (row stride `stride`) of ndt values from src into
// dst[ndt] in a fixed order that does not depend on timing: thread t takes
// entry i = t % ndt of rows s, s + ns, ... (s = t / ndt, ns slices), then the
// slices are added in slice order.  Loads are agent-scope (coherent) loads.
template <int BS>
__device__ __forceinline__ void sum_rows_fixed(const double* src, int count, int ndt,
                                               double* red /* LDS [BS] */, double* dst,
                                               size_t stride = kRedStride) {
  const int t = threadIdx.x;
  if (ndt * 2 <= BS) {
    int ns = BS / ndt;
    if (ns > count) ns = count;
    const int s = t / ndt;
    const int i = t - s * ndt;
    if (s < ns) {
      double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
      int j = s;
      for (; j + 3 * ns < count; j += 4 * ns) {
        a0 += ld_agent(src + (size_t)j * stride + i);
        a1 += ld_agent(src + (size_t)(j + ns) * stride + i);
        a2 += ld_agent(src + (size_t)(j + 2 * ns) * stride + i);
        a3 += ld_agent(src + (size_t)(j + 3 * ns) * stride + i);
      }
      for (; j < count; j += ns) a0 += ld_agent(src + (size_t)j * stride + i);
      red[s * ndt + i] = (a0 + a1) + (a2 + a3);
    }
    __syncthreads();
    if (t < ndt) {
      double tot = 0.0;
      for (int q = 0; q < ns; ++q) tot += red[q * ndt + t];
      dst[t] = tot;
    }
    __syncthreads();
  } else {
    for (int i = t; i < ndt; i += BS) {
      double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
      int j = 0;
      for (; j + 3 < count; j += 4) {
        a0 += ld_agent(src + (size_t)j * stride + i);
        a1 += ld_agent(src + (size_t)(j + 1) * stride + i);
        a2 += ld_agent(src + (size_t)(j + 2) * stride + i);
        a3 += ld_agent(src + (size_t)(j + 3) * stride + i);
      }
      for (; j < count; ++j) a0 += ld_agent(src + (size_t)j * stride + i);
      dst[i] = (a0 + a1) + (a2 + a3);
    }
    __syncthreads();
  }
}

// Grid-wide reduction of ndt = ND*T values per block (vals, in LDS).  Blocks
// form groups of kGrp; the last block to arrive in a group sums the group's
// partials, and the last group to finish sums the group results, both with
// sum_rows_fixed (fixed order, so results repeat bit for bit).  Returns true
// in exactly one block, whose vals then hold the grid totals.  Every block of
// the grid must call it.
template <int BS>
__device__ bool grid_reduce(double* vals, int ndt, const GridRed& red) {
  __shared__ int s_last;
  __shared__ double s_red[BS];
  const int b = blockIdx.x;
  const int nb = gridDim.x;
  const int grp = b / kGrp;
  const int ngrp = (nb + kGrp - 1) / kGrp;
  const int gsz = min(kGrp, nb - grp * kGrp);
  for (int i = threadIdx.x; i < ndt; i += BS) st_agent(&red.part1[(size_t)b * kRedStride + i], vals[i]);
  wait_stores();
  __syncthreads();
  if (threadIdx.x == 0) s_last = (ticket(&red.tick1[grp]) == (unsigned)(gsz - 1));
  __syncthreads();
  if (!s_last) return false;
  sum_rows_fixed<BS>(red.part1 + (size_t)grp * kGrp * kRedStride, gsz, ndt, s_red, vals);
  for (int i = threadIdx.x; i < ndt; i += BS) st_agent(&red.part2[(size_t)grp * kRedStride + i], vals[i]);
  if (threadIdx.x == 0) red.tick1[grp] = 0u;
  wait_stores();
  __syncthreads();
  if (threadIdx.x == 0) s_last = (ticket(red.tick2) == (unsigned)(ngrp - 1));
  __syncthreads();
  if (!s_last) return false;
  sum_rows_fixed<BS>(red.part2, ngrp, ndt, s_red, vals);
  if (threadIdx.x == 0) *red.tick2 = 0u;
  __syncthreads();
  return true;
}

// Recount the active flags (called by one block after it changed them).
__device__ __forceinline__ void recount_active(ColState* cs, int T) {
  __syncthreads();
  if (threadIdx.x == 0) {
    int a = 0, o = 0, im = 0, f = 0;
    for (int c = 0; c < T; ++c) {
      a += cs->active[c];
      o += cs->oactive[c];
      f += cs->fb[c];
      im = cs->it_cur[c] > im ? cs->it_cur[c] : im;
    }
    cs->n_active = a;
    cs->n_oactive = o;
    cs->it_max = im;
    cs->n_fb = f;
  }
}

// Loads of the CSR (column indices, weights) in the Laplacian apply.
#ifndef NVD_NT_CSR
#define NVD_NT_CSR 0
#endif
#if NVD_NT_CSR
#define NVD_CSR_LOAD(p) __builtin_nontemporal_load(p)
#else
#define NVD_CSR_LOAD(p) (*(p))
#endif

// VW consecutive elements of a row, loaded and stored as one access.
template <typename V, int VW>
struct VecOf {
  typedef V type __attribute__((ext_vector_type(VW)));
};
template <typename V>
struct VecOf<V, 1> {
  typedef V type;
};

template <typename V, int VW>
__device__ __forceinline__ void unpack(const typename VecOf<V, VW>::type& a, V (&o)[VW]) {
  if constexpr (VW == 1) {
    o[0] = a;
  } else {
#pragma unroll
    for (int v = 0; v < VW; ++v) o[v] = a[v];
  }
}

template <typename V, int VW>
__device__ __forceinline__ typename VecOf<V, VW>::type pack(const V (&o)[VW]) {
  typename VecOf<V, VW>::type a;
  if constexpr (VW == 1) {
    a = o[0];
  } else {
#pragma unroll
    for (int v = 0; v < VW; ++v) a[v] = o[v];
  }
  return a;
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
