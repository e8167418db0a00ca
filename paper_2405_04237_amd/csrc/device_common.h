// Device helpers shared by the libcqr kernels (gfx950).
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

namespace cqr {

typedef double d4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ d4 mfma16x16x4(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Workgroups are dispatched round-robin over the 8 XCDs (each with its own
// L2). Renumber so that each XCD receives a contiguous range of logical
// block ids: neighbouring logical blocks (which share input rows) then share
// an L2.
__device__ __forceinline__ int64_t xcd_logical(int64_t bid, int64_t nb) {
  constexpr int64_t kXcd = 8;
  const int64_t full = nb / kXcd * kXcd;
  if (bid >= full) return bid;
  return (bid % kXcd) * (full / kXcd) + bid / kXcd;
}

// Right-looking Cholesky W = U^T U of a w x w matrix held in LDS, one row of
// U per step: S holds W's upper triangle on entry and U's strict upper
// triangle on exit; U's diagonal goes to D (S's diagonal keeps the pivots'
// squares). Every thread reads the pivot itself, so the only barriers are
// after the row scaling and after the trailing update. Returns 0, or the
// 1-based column of the first pivot that is not > 0 (NaN included), the
// same value in every thread.
__device__ inline int lds_cholesky(double *S, double *D, int w) {
  const int tid = threadIdx.x, nt = blockDim.x;
  for (int k = 0; k < w; ++k) {
    const double d = S[k * w + k];
    if (!(d > 0.0)) return k + 1;
    const double piv = sqrt(d);
    if (tid == 0) D[k] = piv;
    for (int j = k + 1 + tid; j < w; j += nt) S[k * w + j] = S[k * w + j] / piv;
    __syncthreads();
    const int rem = w - k - 1;
    if (rem > 0) {
      // thread -> (column jj, rows ii, ii + step, ...) with ii <= jj
      const int per = nt / rem > 0 ? nt / rem : 1;
      if (tid < per * rem) {
        const int jj = tid % rem, i0 = tid / rem;
        const double ukj = S[k * w + k + 1 + jj];
        for (int ii = i0; ii <= jj; ii += per)
          S[(k + 1 + ii) * w + k + 1 + jj] -= S[k * w + k + 1 + ii] * ukj;
      }
    }
    __syncthreads();
  }
  return 0;
}

// Inverse X = U^{-1} of an upper triangular w x w matrix held in LDS: U in
// the upper triangle of S (diagonal included). Column sweep of back
// substitution U X = I, one row of X per step: scale row k by 1/U_kk, then
// remove it from rows i < k. X[i][c] (i < c) ends in S[c*w + i] (the strict
// lower triangle, transposed) and X[k][k] in D[k]; U is left intact.
__device__ inline void lds_upper_inverse(double *S, double *D, int w) {
  const int tid = threadIdx.x, nt = blockDim.x;
  for (int k = tid; k < w; k += nt) D[k] = 1.0;
  for (int e = tid; e < w * w; e += nt)
    if (e / w > e % w) S[e] = 0.0;
  __syncthreads();
  for (int k = w - 1; k >= 0; --k) {
    const double ukk = S[k * w + k];
    for (int c = k + tid; c < w; c += nt) {
      if (c == k)
        D[k] = D[k] / ukk;
      else
        S[c * w + k] = S[c * w + k] / ukk;
    }
    __syncthreads();
    if (k > 0) {
      const int cols = w - k;
      // thread -> (row i, columns c, c + step, ...)
      const int per = nt / k > 0 ? nt / k : 1;
      if (tid < per * k) {
        const int i = tid % k, c0 = tid / k;
        const double uik = S[i * w + k];
        for (int cc = c0; cc < cols; cc += per) {
          const int c = k + cc;
          if (c == k)
            S[k * w + i] -= uik * D[k];
          else
            S[c * w + i] -= uik * S[c * w + k];
        }
      }
    }
    __syncthreads();
  }
}

}  // namespace cqr
