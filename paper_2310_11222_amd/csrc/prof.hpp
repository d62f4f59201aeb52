// Launch timing hooks (prof.hip).
#pragma once
#include <hip/hip_runtime.h>

namespace nvd {
enum ProfKind {
  PK_SPMM64 = 0, PK_SPMM32 = 1, PK_UPD64 = 2, PK_UPD32 = 3, PK_DIR64 = 4, PK_DIR32 = 5,
  PK_OTHER = 6
};
bool prof_enabled();
int prof_begin(hipStream_t s, int kind, double bytes);
void prof_end(hipStream_t s, int id);
int prof_last_id();            // id returned by the most recent prof_begin (-1 if none)
void prof_mark_idle(int id);   // exclude a record (a launch that found no work)
}  // namespace nvd
