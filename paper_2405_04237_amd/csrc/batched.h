// Internal interface of the persistent batched factorisation kernel.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cqr {

constexpr int kBatchMaxPanel = 32;  // panel width limit of the batched form
constexpr int kBatchMaxN = 128;     // column limit of the batched form

// Dynamic LDS bytes of the persistent kernel, and how many of its workgroups
// fit on one compute unit at once.
size_t batched_lds_bytes();
int batched_blocks_per_cu();

// Reset the queue word, then one persistent launch of `grid` workgroups that
// factor the `count` matrices in queue order order[0..count) (mCQR2GS each).
// ms/ns/bs: per-matrix shape and panel width (device arrays, indexed by
// matrix id); dA/dlda/dQ/dR: per-matrix device pointers and leading
// dimensions (R leading dimension n); dinfo[i] receives 0 or the 1-based
// breakdown column of matrix i.
hipError_t launch_batched_mod(int grid, const int *order, const int64_t *ms, const int *ns,
                              const int *bs, int count, const double *const *dA, const int64_t *dlda,
                              double *const *dQ, double *const *dR, int *dinfo, int *queue,
                              hipStream_t s);

}  // namespace cqr
