// Launchers of the distance-matrix consumers (ls_cluster.hip): average
// pairwise linkage and standardised half-distance rows. Not part of the
// public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace lsk {

// Workspace of launch_linkage for T matrices of N (per matrix: the nearest
// slot, its distance, cluster sizes and ids, a row list, occupancy flags).
size_t linkage_workspace_bytes(int32_t N, int32_t T, int is_f64);
// Average linkage of T symmetric [N][N] matrices D (overwritten): Z [T][N-1][4]
// (smaller id, larger id, distance, size), order [T][N] (may be null).
hipError_t launch_linkage(void *D, int32_t N, int32_t T, int is_f64, double *Z, int32_t *order,
                          void *ws, hipStream_t st);
// Standardise, in place, T x R rows of N half distances at E + k ts + r rs
// (recipient recips[r]).
hipError_t launch_standardise(void *E, const int32_t *recips, int32_t R, int32_t T, int32_t N,
                              int64_t ts, int64_t rs, int is_f64, hipStream_t st);

// Size of the fixed per-device scratch of the allocation-free linkage entry
// point (enough for N = 10,000 with T = 150 matrices, or N = 100,000 with
// T = 15), and the address of the current device's copy (ls_cluster.hip).
constexpr size_t kLinkageScratchBytes = (size_t)32 << 20;
hipError_t linkage_scratch(void **out);

}  // namespace lsk
