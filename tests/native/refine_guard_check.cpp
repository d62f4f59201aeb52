// CPU check of the mixed-precision stagnation rule (refine_guard.hpp), the
// same code the solver's kernels compile: prints one line per case and exits
// non-zero on the first wrong answer.
#include <cmath>
#include <cstdio>
#include <limits>

#include "refine_guard.hpp"

using namespace nvd;

static int fails = 0;
static void expect(bool ok, const char* what) {
  std::printf("%s %s\n", ok ? "ok  " : "FAIL", what);
  if (!ok) ++fails;
}

// Runs the rule over a sequence of outer residual norms^2 and returns the
// step (1-based, counting outer steps after the first) at which the pair is
// handed to FP64, or 0 if never.
static int hand_off_step(const double* rr, int n) {
  int count = 0;
  for (int i = 1; i < n; ++i) {
    count = refine_stall_count(rr[i - 1], rr[i], count);
    if (refine_hand_to_fp64(count)) return i;
  }
  return 0;
}

int main() {
  const double nan = std::numeric_limits<double>::quiet_NaN();
  const double inf = std::numeric_limits<double>::infinity();
  {
    const double rr[] = {1.0, 1e-10, 1e-20, 1e-30};         // healthy: 1e-5 per step in norm
    expect(hand_off_step(rr, 4) == 0, "healthy refinement is never handed off");
  }
  {
    const double rr[] = {1.0, 0.9, 0.8, 0.7};                // stalled from the first step
    expect(hand_off_step(rr, 4) == 2, "two stalled steps in a row hand off at the second");
  }
  {
    const double rr[] = {1.0, 0.9, 1e-10, 0.9e-10, 1e-21};   // stalled, progress, stalled once
    expect(hand_off_step(rr, 5) == 0, "a stall broken by progress restarts the count");
  }
  {
    const double rr[] = {1.0, 0.25, 0.0625};                 // exactly 2x in norm: not stalled
    expect(hand_off_step(rr, 3) == 0, "a factor of exactly 2 in norm counts as progress");
  }
  {
    const double rr[] = {1.0, 0.2500001, 0.0625001};         // just under 2x: stalled
    expect(hand_off_step(rr, 3) == 2, "just under a factor 2 in norm counts as a stall");
  }
  {
    const double rr[] = {1.0, nan, 0.5};
    expect(hand_off_step(rr, 3) == 2, "a non-finite residual counts as a stall");
  }
  {
    const double rr[] = {1.0, inf, inf};
    expect(hand_off_step(rr, 3) == 2, "an infinite residual counts as a stall");
  }
  {
    const double rr[] = {1.0, 2.0, 1e-12, 2e-12, 3e-12};     // growth is a stall too
    expect(hand_off_step(rr, 5) == 4, "growth counts as a stall; count restarts after progress");
  }
  expect(kStallSteps == 2 && kStallRatio2 == 0.25, "constants: two steps, factor 2 in norm");
  return fails ? 1 : 0;
}
