// Internal interface of the persistent batched factorisation kernel.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cqr {

constexpr int kBatchMaxPanel = 32;  // panel width limit of the batched form
constexpr int kBatchMaxN = 128;     // column limit of the batched form
constexpr int kBatchMaxTeam = 4;    // workgroups that may share one matrix
// a small batch (at most one matrix per eight resident workgroups) splits
// each matrix over up to this many workgroups of at least kTeamMinRows rows
constexpr int kBatchMaxTeamSmall = 16;
constexpr int kTeamMinRows = 128;
constexpr int kTeamSlot = kBatchMaxPanel * kBatchMaxN;  // doubles per partial product

// One work item of the persistent kernel: member `member` of the `team`
// workgroups that factor matrix `matrix` (team == 1: the whole matrix).
// Teams split the rows; their members exchange every row-reduced product
// through team_part (offset part, 2 x team x kTeamSlot doubles) and a
// counter team_cnt[cnt].
struct BatchSlot {
  int matrix, member, team, cnt;
  int64_t part;
};

// Dynamic LDS bytes of the persistent kernel, and how many of its workgroups
// fit on one compute unit at once.
size_t batched_lds_bytes();
int batched_blocks_per_cu();

// Reset the queue word and the team counters, then one persistent launch of
// `grid` workgroups (all resident at once) that take the `nslots` work items
// slots[0..nslots) in order (mCQR2GS of a matrix, or of a team's share of
// its rows). ms/ns/bs: per-matrix shape and panel width (device arrays,
// indexed by matrix id); dA/dlda/dQ/dR: per-matrix device pointers and
// leading dimensions (R leading dimension n); dinfo[i] receives 0, the
// 1-based breakdown column of matrix i, or -1 if a team member waited for
// its partners past the spin limit (the matrix's outputs are then invalid).
hipError_t launch_batched_mod(int grid, const BatchSlot *slots, int nslots, const int64_t *ms,
                              const int *ns, const int *bs, const double *const *dA,
                              const int64_t *dlda, double *const *dQ, double *const *dR,
                              int *dinfo, int *queue, double *team_part, int *team_cnt, int nteams,
                              hipStream_t s);

}  // namespace cqr
