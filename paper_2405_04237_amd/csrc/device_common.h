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

// ---------------------------------------------------------------------------
// Blocked forms for one workgroup of any size (>= 64 threads) on a matrix of
// order wp = 16 * 2^k (16 ... 128) held row-major in LDS with stride wp; the
// caller pads a smaller matrix with the identity. They need a handful of
// workgroup barriers per 16 columns instead of two per column.
// ---------------------------------------------------------------------------

// Ordering of LDS accesses among the lanes of one wave.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// W = U^T U in place (upper triangle of S; the strict lower part is left as
// it was), right-looking by 16-column panels: wave 0 factors the diagonal
// block, every thread then solves the panel's row block and updates the
// trailing upper triangle, each element's terms subtracted in column order
// (the order of the unblocked right-looking algorithm). Returns 0 or the
// 1-based column of the first pivot that is not > 0 (NaN included), the
// same in every thread. `flag` is one int of LDS; S needs 16 doubles of
// scratch after the wp x wp matrix (the panel's pivot reciprocals).
__device__ inline int lds_cholesky_blocked(double *S, int wp, int *flag) {
  const int tid = threadIdx.x, nt = blockDim.x, lane = tid & 63;
  double *rpiv = S + wp * wp;  // 16 doubles of scratch after the matrix
  if (tid == 0) *flag = 0;
  __syncthreads();
  for (int p0 = 0; p0 < wp; p0 += 16) {
    if (tid < 64) {  // diagonal block, one wave
      for (int k = 0; k < 16; ++k) {
        const int kk = p0 + k;
        const double d = S[kk * wp + kk];
        if (!(d > 0.0)) {
          if (lane == 0) *flag = kk + 1;
          break;
        }
        const double piv = sqrt(d);
        wave_lds_sync();
        if (lane < 16 - k) {
          const int j = kk + lane;
          S[kk * wp + j] = (lane == 0) ? piv : S[kk * wp + j] / piv;
        }
        wave_lds_sync();
        // trailing part of the block: rows kk+1.., columns >= row
        for (int e = lane; e < 16 * 16; e += 64) {
          const int i = p0 + e / 16, j = p0 + e % 16;
          if (i > kk && j >= i) S[i * wp + j] -= S[kk * wp + i] * S[kk * wp + j];
        }
        wave_lds_sync();
      }
    }
    // the panel's pivot reciprocals (scratch after the matrix): the row
    // solve multiplies by them, as LAPACK's unblocked Cholesky scales rows
    if (tid < 16 && p0 + tid < wp) rpiv[tid] = 1.0 / S[(p0 + tid) * wp + p0 + tid];
    __syncthreads();
    const int fail = *flag;
    if (fail) return fail;
    const int c0 = p0 + 16, rest = wp - c0;
    if (rest > 0) {
      // row block: column j solved by forward substitution through the panel
      // 16 lanes per column (lane k of the group holds row p0 + k): row k is
      // final at step k and is broadcast to the rows below it
      for (int e = tid; e < 16 * rest; e += nt) {
        const int j = c0 + e / 16, k = e % 16;
        double v = S[(p0 + k) * wp + j];
        for (int st = 0; st < 16; ++st) {
          const double x = __shfl(v * rpiv[st], st, 16);
          if (k == st) v = x;
          if (k > st) v -= S[(p0 + st) * wp + p0 + k] * x;
        }
        S[(p0 + k) * wp + j] = v;
      }
      __syncthreads();
      // trailing upper triangle
      for (int e = tid; e < rest * rest; e += nt) {
        const int i = c0 + e / rest, j = c0 + e % rest;
        if (j >= i) {
          double ui[16], uj[16];  // all 32 reads in flight before the products
#pragma unroll
          for (int k = 0; k < 16; ++k) {
            ui[k] = S[(p0 + k) * wp + i];
            uj[k] = S[(p0 + k) * wp + j];
          }
          __builtin_amdgcn_sched_barrier(0);
          double x = S[i * wp + j];
#pragma unroll
          for (int k = 0; k < 16; ++k) x -= ui[k] * uj[k];
          S[i * wp + j] = x;
        }
      }
      __syncthreads();
    }
  }
  return 0;
}

// U^{-1} in place of the upper triangle of S (U upper, nonzero diagonal) by
// block back substitution of U X = I, 16 rows at a time from the bottom:
// first every thread forms the right-hand sides of block row i from the
// finished rows below (into tmp, 16 x wp), then one thread per column solves
// with the 16 x 16 diagonal block (kept transposed in the block's strict
// lower triangle, the reciprocals of its diagonal in dg[16]). Each entry of X is thus a
// substitution step of U X = I, so U X - I stays at the rounding level of
// U's entries, which is what Q = A U^{-1} needs. The strict lower triangle
// of S is overwritten.
__device__ inline void lds_upper_inverse_blocked(double *S, int wp, double *tmp, double *dg) {
  const int tid = threadIdx.x, nt = blockDim.x;
  for (int o = wp - 16; o >= 0; o -= 16) {
    const int ncols = wp - o;
    for (int e = tid; e < 16 * 16; e += nt) {  // U_ii^T below the diagonal, diagonal to dg
      const int r = e / 16, t = e % 16;
      if (t > r) S[(o + t) * wp + o + r] = S[(o + r) * wp + o + t];
      if (t == r) dg[r] = 1.0 / S[(o + r) * wp + o + r];  // reciprocal of the pivot
    }
    for (int e = tid; e < 16 * ncols; e += nt) {
      const int r = e / ncols, j = o + e % ncols;
      // four partial sums over k, 16 rows of X at a time (X[k][j] = 0 for k > j)
      const double *ur = S + (o + r) * wp;
      double x0 = 0.0, x1 = 0.0, x2 = 0.0, x3 = 0.0;
      int k0 = o + 16;
      for (; k0 + 15 <= j; k0 += 16) {
        double ua[16], xb[16];  // all 32 reads in flight before the products
#pragma unroll
        for (int k = 0; k < 16; ++k) {
          ua[k] = ur[k0 + k];
          xb[k] = S[(k0 + k) * wp + j];
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int k = 0; k < 16; k += 4) {
          x0 += ua[k] * xb[k];
          x1 += ua[k + 1] * xb[k + 1];
          x2 += ua[k + 2] * xb[k + 2];
          x3 += ua[k + 3] * xb[k + 3];
        }
      }
      // the block holding row j: X[k][j] = 0 below the diagonal (k > j)
      if (k0 <= j) {
#pragma unroll
        for (int k = 0; k < 16; k += 4) {
          if (k0 + k <= j) x0 += ur[k0 + k] * S[(k0 + k) * wp + j];
          if (k0 + k + 1 <= j) x1 += ur[k0 + k + 1] * S[(k0 + k + 1) * wp + j];
          if (k0 + k + 2 <= j) x2 += ur[k0 + k + 2] * S[(k0 + k + 2) * wp + j];
          if (k0 + k + 3 <= j) x3 += ur[k0 + k + 3] * S[(k0 + k + 3) * wp + j];
        }
      }
      tmp[r * wp + j] = ((o + r == j) ? 1.0 : 0.0) - ((x0 + x1) + (x2 + x3));
    }
    __syncthreads();
    // 16 lanes per column (lane r of the group holds row r): x_r is final at
    // step r, is broadcast within the group, and leaves the rows above
    for (int e = tid; e < 16 * ncols; e += nt) {
      const int j = o + e / 16, r = e % 16;
      double v = tmp[r * wp + j];
      for (int st = 15; st >= 0; --st) {
        const double x = __shfl(v * dg[st], st, 16);
        if (r == st) v = x;
        if (r < st) v -= S[(o + st) * wp + o + r] * x;
      }
      if (o + r <= j) S[(o + r) * wp + j] = v;  // below X's diagonal: the U_ii copy
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Orders above what one workgroup's LDS holds (wp = 2h, h = 128): the padded
// matrix G lives in device memory (row-major, ld wp; a few hundred KiB that
// stay in L2) and one workgroup runs the same steps as the LDS forms above.
// S is LDS of blocked_lds_doubles(h) doubles.
// ---------------------------------------------------------------------------

// W = U^T U in place of G's upper triangle (the strict lower part must be 0
// on entry and stays 0). Right-looking by 16-column panels, as
// lds_cholesky_blocked: the panel's 16 rows are staged in LDS, where wave 0
// factors the diagonal block and every thread solves the row block; the
// panel's rows of U go back to G, and the trailing upper triangle is updated
// in G, each element's terms subtracted in column order. When the trailing
// matrix has order h it is moved to LDS and finished by lds_cholesky_blocked
// (the same steps). Returns 0 or the 1-based column of the first pivot that
// is not > 0 (NaN included), the same in every thread.
__device__ inline int wide_cholesky(double *G, int wp, double *S, int *flag) {
  const int tid = threadIdx.x, nt = blockDim.x, lane = tid & 63, h = wp / 2;
  double *P = S;               // 16 x wp: rows p0 .. p0 + 15 of the matrix
  double *rpiv = S + 16 * wp;  // the panel's pivot reciprocals
  for (int p0 = 0; p0 < h; p0 += 16) {
    if (tid == 0) *flag = 0;
    for (int e = tid; e < 16 * wp; e += nt) {
      const int k = e / wp, j = e % wp;
      P[e] = (j >= p0) ? G[(int64_t)(p0 + k) * wp + j] : 0.0;
    }
    __syncthreads();
    if (tid < 64) {  // diagonal block, one wave
      for (int k = 0; k < 16; ++k) {
        const int kk = p0 + k;
        const double d = P[k * wp + kk];
        if (!(d > 0.0)) {
          if (lane == 0) *flag = kk + 1;
          break;
        }
        const double piv = sqrt(d);
        wave_lds_sync();
        if (lane < 16 - k) {
          const int j = kk + lane;
          P[k * wp + j] = (lane == 0) ? piv : P[k * wp + j] / piv;
        }
        wave_lds_sync();
        for (int e = lane; e < 16 * 16; e += 64) {
          const int i = e / 16, j = e % 16;  // block-relative
          if (i > k && j >= i) P[i * wp + p0 + j] -= P[k * wp + p0 + i] * P[k * wp + p0 + j];
        }
        wave_lds_sync();
      }
    }
    if (tid < 16) rpiv[tid] = 1.0 / P[tid * wp + p0 + tid];
    __syncthreads();
    const int fail = *flag;
    if (fail) return fail;
    const int c0 = p0 + 16, rest = wp - c0;
    // row block: forward substitution through the panel, 16 lanes per column
    for (int e = tid; e < 16 * rest; e += nt) {
      const int j = c0 + e / 16, k = e % 16;
      double v = P[k * wp + j];
      for (int st = 0; st < 16; ++st) {
        const double x = __shfl(v * rpiv[st], st, 16);
        if (k == st) v = x;
        if (k > st) v -= P[st * wp + p0 + k] * x;
      }
      P[k * wp + j] = v;
    }
    __syncthreads();
    // the panel's rows of U are final
    for (int e = tid; e < 16 * (wp - p0); e += nt) {
      const int k = e / (wp - p0), j = p0 + e % (wp - p0);
      G[(int64_t)(p0 + k) * wp + j] = P[k * wp + j];
    }
    // trailing upper triangle, in device memory
    for (int e = tid; e < rest * rest; e += nt) {
      const int i = c0 + e / rest, j = c0 + e % rest;
      if (j >= i) {
        double ui[16], uj[16];
#pragma unroll
        for (int k = 0; k < 16; ++k) {
          ui[k] = P[k * wp + i];
          uj[k] = P[k * wp + j];
        }
        double *g = G + (int64_t)i * wp + j;
        double x = *g;
#pragma unroll
        for (int k = 0; k < 16; ++k) x -= ui[k] * uj[k];
        *g = x;
      }
    }
    __syncthreads();
  }
  // the trailing h x h block in LDS
  for (int e = tid; e < h * h; e += nt) S[e] = G[(int64_t)(h + e / h) * wp + h + e % h];
  __syncthreads();
  const int fail = lds_cholesky_blocked(S, h, flag);
  if (fail) return h + fail;
  for (int e = tid; e < h * h; e += nt) {
    const int i = e / h, j = e % h;
    if (j >= i) G[(int64_t)(h + i) * wp + h + j] = S[e];
  }
  __syncthreads();
  return 0;
}

// U^{-1} in place of G's upper triangle (U upper with a nonzero diagonal;
// the strict lower part is left as it was): the block back substitution of
// lds_upper_inverse_blocked. The bottom-right h x h block X22 = U22^{-1}
// involves U22 alone and is formed in LDS by that function; then block rows
// of 16 from row h - 16 upwards: the block's rows of U are staged in LDS,
// right-hand sides are formed from the finished rows of X below (read from
// G), and 16 lanes per column solve with the 16 x 16 diagonal block.
__device__ inline void wide_upper_inverse(double *G, int wp, double *S) {
  const int tid = threadIdx.x, nt = blockDim.x, h = wp / 2;
  for (int e = tid; e < h * h; e += nt) {
    const int i = e / h, j = e % h;
    S[e] = (j >= i) ? G[(int64_t)(h + i) * wp + h + j] : 0.0;
  }
  __syncthreads();
  lds_upper_inverse_blocked(S, h, S + h * h, S + h * h + 16 * h);
  for (int e = tid; e < h * h; e += nt) {
    const int i = e / h, j = e % h;
    if (j >= i) G[(int64_t)(h + i) * wp + h + j] = S[e];
  }
  __syncthreads();
  double *Ur = S;              // 16 x wp: the block's rows of U
  double *tmp = S + 16 * wp;   // 16 x wp: right-hand sides
  double *dg = S + 32 * wp;    // reciprocals of the block's pivots
  for (int o = h - 16; o >= 0; o -= 16) {
    const int ncols = wp - o;
    for (int e = tid; e < 16 * ncols; e += nt) {
      const int r = e / ncols, j = o + e % ncols;
      Ur[r * wp + j] = G[(int64_t)(o + r) * wp + j];
    }
    if (tid < 16) dg[tid] = 1.0 / G[(int64_t)(o + tid) * wp + o + tid];
    __syncthreads();
    for (int e = tid; e < 16 * ncols; e += nt) {
      const int r = e / ncols, j = o + e % ncols;
      // four partial sums over k, as lds_upper_inverse_blocked (X[k][j] = 0 for k > j)
      const double *ur = Ur + r * wp;
      double x0 = 0.0, x1 = 0.0, x2 = 0.0, x3 = 0.0;
      int k0 = o + 16;
      for (; k0 + 15 <= j; k0 += 16) {
        double ua[16], xb[16];
#pragma unroll
        for (int k = 0; k < 16; ++k) {
          ua[k] = ur[k0 + k];
          xb[k] = G[(int64_t)(k0 + k) * wp + j];
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int k = 0; k < 16; k += 4) {
          x0 += ua[k] * xb[k];
          x1 += ua[k + 1] * xb[k + 1];
          x2 += ua[k + 2] * xb[k + 2];
          x3 += ua[k + 3] * xb[k + 3];
        }
      }
      if (k0 <= j) {
#pragma unroll
        for (int k = 0; k < 16; k += 4) {
          if (k0 + k <= j) x0 += ur[k0 + k] * G[(int64_t)(k0 + k) * wp + j];
          if (k0 + k + 1 <= j) x1 += ur[k0 + k + 1] * G[(int64_t)(k0 + k + 1) * wp + j];
          if (k0 + k + 2 <= j) x2 += ur[k0 + k + 2] * G[(int64_t)(k0 + k + 2) * wp + j];
          if (k0 + k + 3 <= j) x3 += ur[k0 + k + 3] * G[(int64_t)(k0 + k + 3) * wp + j];
        }
      }
      tmp[r * wp + j] = ((o + r == j) ? 1.0 : 0.0) - ((x0 + x1) + (x2 + x3));
    }
    __syncthreads();
    for (int e = tid; e < 16 * ncols; e += nt) {
      const int j = o + e / 16, r = e % 16;
      double v = tmp[r * wp + j];
      for (int st = 15; st >= 0; --st) {
        const double x = __shfl(v * dg[st], st, 16);
        if (r == st) v = x;
        if (r < st) v -= Ur[r * wp + o + st] * x;
      }
      if (o + r <= j) G[(int64_t)(o + r) * wp + j] = v;
    }
    __syncthreads();
  }
}

// LDS doubles the blocked Cholesky + inverse need for padded order wp.
__host__ __device__ inline int blocked_lds_doubles(int wp) { return wp * wp + 16 * wp + 16; }

// LDS doubles the device-memory forms need for order wp = 2h: the LDS form
// of order h, which also covers the 16-row stagings (at most 32 wp + 16).
__host__ __device__ inline int wide_lds_doubles(int wp) { return blocked_lds_doubles(wp / 2); }

// Order of the padded LDS matrix used by the blocked forms for order w.
__host__ __device__ inline int blocked_order(int w) {
  int wp = 16;
  while (wp < w) wp *= 2;
  return wp;
}

}  // namespace cqr
