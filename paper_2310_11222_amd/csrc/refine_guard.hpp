// Stagnation rule of the mixed-precision refinement (plain C++, so that the
// same code is compiled into the solver's kernels and into a CPU test).
//
// Each outer step solves L c = r in FP32 to a relative residual well below
// 1/2 and adds c to x in FP64, so a healthy step shrinks the FP64 residual
// by a large factor.  FP32 cannot do that once the inner problem's
// conditioning times FP32's unit roundoff approaches 1 (a long path, a
// badly weighted graph): the outer residual then stalls.  The rule: a pair
// whose outer residual norm falls by less than a factor 2 in two
// consecutive outer steps (||r_new||^2 > ||r_old||^2 / 4 twice) is handed to
// the FP64 solver, which continues from its current x.
#pragma once

#ifndef NVD_HD
#if defined(__HIPCC__)
#define NVD_HD __host__ __device__
#else
#define NVD_HD
#endif
#endif

namespace nvd {

constexpr int kStallSteps = 2;          // consecutive stalled outer steps
constexpr double kStallRatio2 = 0.25;   // ||r_new||^2 / ||r_old||^2 above this: stalled

// Stalled-step count after an outer step from residual norm^2 rr_old to
// rr_new; the pair goes to the FP64 solver once the count reaches
// kStallSteps.  A non-finite rr_new counts as stalled.
NVD_HD inline int refine_stall_count(double rr_old, double rr_new, int count,
                                     double ratio2 = kStallRatio2) {
  const bool stalled = !__builtin_isfinite(rr_new) || !(rr_new <= ratio2 * rr_old);
  return stalled ? count + 1 : 0;
}

NVD_HD inline bool refine_hand_to_fp64(int count) { return count >= kStallSteps; }

}  // namespace nvd
