// Entry points the library's translation units share beyond include/top.h.
#pragma once

#include "top.h"

namespace top {
// Where a handle's device memory comes from: the library's pool (no workspace given), a caller's
// workspace, or the static scratch of a no-allocation call (shape tables and lane map in it too,
// no pinned host memory or events created).
enum class Mem { kPool, kCallerWs, kStatic };

// top_create with the memory source made explicit.
top_status internal_create(int32_t n_traj, const int64_t* seg_offsets, const double* waypoints,
                           const double* durations, const double* bc, const double* box_lo,
                           const double* box_hi, const double* vmax, const double* rho, const top_options* opt,
                           void* workspace, size_t workspace_bytes, hipStream_t stream, top_problem** out,
                           Mem mem);
// Record `text` as the calling thread's last error and return s.
top_status internal_error(top_status s, const char* text);
}  // namespace top
