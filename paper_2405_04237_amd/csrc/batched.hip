// Batched factorisation of many independent tall-and-skinny matrices in one
// persistent launch (mCQR2GS, Algorithm 9 of arXiv 2405.04237, per matrix).
//
// Each 256-thread workgroup pops a matrix from an atomic queue (the host
// orders the queue longest-first) and factors it alone: its panel Grams,
// projections and updates are MFMA passes over the matrix rows in which the
// four waves share the work, the reductions over rows end in the
// workgroup's LDS in a fixed order (no cross-workgroup communication), and
// the b x b Cholesky factors and inverses stay in LDS. A workgroup exits
// when the queue is empty, so every wave reaches the end of the kernel.
//
// Limits of this form: panel width b <= kBatchMaxPanel, n <= kBatchMaxN.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "batched.h"
#include "device_common.h"
#include "kernels.h"

namespace cqr {

namespace {

constexpr int kThreads = 256;
// Row sums are accumulated on three levels so that no running sum takes more
// than a few hundred sequential additions: MFMA accumulators over kInnerRows
// rows, a second register set over kFlushRows rows, then the LDS result.
constexpr int kInnerRows = 512;
constexpr int kFlushRows = 4096;

// LDS layout (doubles)
constexpr int kYSize = kBatchMaxPanel * kBatchMaxN + 64;  // projections (+ read slack)
constexpr int kBB = kBatchMaxPanel * kBatchMaxPanel;
struct Lds {
  double *y, *w, *ua, *ub, *ui, *s, *d;
  int *flag;
};
__device__ inline Lds lds_layout(double *base) {
  Lds L;
  L.y = base;
  L.w = L.y + kYSize;
  L.ua = L.w + kBB;
  L.ub = L.ua + kBB;
  L.ui = L.ub + kBB;
  L.s = L.ui + kBB + 64;
  L.d = L.s + kBB;
  L.flag = reinterpret_cast<int *>(L.d + kBatchMaxPanel);
  return L;
}

// Global-memory writes made by one wave before the barrier are visible to
// every wave of the workgroup after it: release fence, barrier, then an
// acquire fence that drops stale vector-L1 lines (agent scope on both sides).
__device__ inline void wg_sync() {
  __threadfence();
  __syncthreads();
  __threadfence();
}

// out (LDS, row-major, ld ldo) = L^T Rt over rows [0, m); L is m x p, Rt m x q
// (column-major). upper: only 16x16 blocks on or above the diagonal. Each wave
// owns up to 4 output blocks and sweeps all rows, flushing its accumulators
// into `out` every kFlushRows rows (a fixed order). The caller guarantees at
// most 16 blocks (b <= 32 and n <= 128 give at most 2 x 8).
__device__ __forceinline__ void wg_tn(int64_t m, int p, int q, const double *L, int64_t ldl, const double *Rt,
                      int64_t ldr, bool upper, double *out, int ldo) {
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, g = lane >> 4, cl = lane & 15;
  for (int e = tid; e < p * ldo; e += kThreads) out[e] = 0.0;
  __syncthreads();
  const int nbp = (p + 15) / 16, nbq = (q + 15) / 16;
  const int total = upper ? nbp * (nbp + 1) / 2 : nbp * nbq;
  // block t of this wave is number wave + 4 t of the list (row-major over
  // (i, j), j >= i when upper); decoded without indexing registers dynamically
  int bi[4], bj[4];
  bool own[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    int lin = wave + 4 * t;
    own[t] = lin < total;
    int i = 0, j = 0;
    if (own[t]) {
      if (upper) {
        int len = nbp;
        while (lin >= len) {
          lin -= len;
          ++i;
          --len;
        }
        j = i + lin;
      } else {
        i = lin / nbq;
        j = lin % nbq;
      }
    }
    bi[t] = i;
    bj[t] = j;
  }
  const int nb = own[3] ? 4 : own[2] ? 3 : own[1] ? 2 : own[0] ? 1 : 0;
  if (nb > 0) {
    const double *pa[4];
    const double *pb[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int ca = 16 * bi[t] + cl, cb = 16 * bj[t] + cl;
      pa[t] = L + (int64_t)(ca < p ? ca : 0) * ldl + 4 * g;
      pb[t] = Rt + (int64_t)(cb < q ? cb : 0) * ldr + 4 * g;
    }
    d4 acc[4], acc2[4];
    auto fold = [&]() {  // acc2 += acc; acc = 0
#pragma unroll
      for (int t = 0; t < 4; ++t) {
#pragma unroll
        for (int e = 0; e < 4; ++e) acc2[t][e] += acc[t][e];
        acc[t] = d4{0.0, 0.0, 0.0, 0.0};
      }
    };
    auto flush = [&]() {  // out += acc2; acc2 = 0
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        if (t < nb) {
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const int I = 16 * bi[t] + g + 4 * e, J = 16 * bj[t] + cl;
            if (I < p && J < q) out[I * ldo + J] += acc2[t][e];
          }
        }
        acc2[t] = d4{0.0, 0.0, 0.0, 0.0};
      }
    };
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      acc[t] = d4{0.0, 0.0, 0.0, 0.0};
      acc2[t] = d4{0.0, 0.0, 0.0, 0.0};
    }
    const int64_t full = m / 16 * 16;
    double a[4][4], b[4][4];
    for (int64_t r0 = 0; r0 < full; r0 += kFlushRows) {
      const int64_t r1 = (r0 + kFlushRows < full) ? r0 + kFlushRows : full;
      for (int64_t ri = r0; ri < r1; ri += kInnerRows) {
        const int64_t r2 = (ri + kInnerRows < r1) ? ri + kInnerRows : r1;
        for (int64_t r = ri; r < r2; r += 16) {
#pragma unroll
          for (int t = 0; t < 4; ++t)
#pragma unroll
            for (int s = 0; s < 4; ++s) {
              a[t][s] = pa[t][r + s];
              b[t][s] = pb[t][r + s];
            }
#pragma unroll
          for (int s = 0; s < 4; ++s)
#pragma unroll
            for (int t = 0; t < 4; ++t)
              if (t < nb) acc[t] = mfma16x16x4(a[t][s], b[t][s], acc[t]);
        }
        fold();
      }
      flush();
    }
    if (full < m) {  // ragged tail
#pragma unroll
      for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          const bool ok = full + 4 * g + s < m;
          a[t][s] = ok ? pa[t][full + s] : 0.0;
          b[t][s] = ok ? pb[t][full + s] : 0.0;
        }
#pragma unroll
      for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int t = 0; t < 4; ++t)
          if (t < nb) acc[t] = mfma16x16x4(a[t][s], b[t][s], acc[t]);
      fold();
      flush();
    }
  }
  wg_sync();
}

// C = L Y (+ Cin when sub) over rows [0, m): L m x p column-major, Y p x q
// row-major in LDS (ld ldy, padded so that 4-wide reads past q stay in the Y
// region), Cin / C m x q column-major. C may alias L only when each wave's
// tile covers all of C's columns (q <= 64): a wave reads its rows of L fully
// before it writes them. 64 x 64 tiles are dealt to the waves round-robin.
__device__ __forceinline__ void wg_nn(int64_t m, int p, int q, const double *L, int64_t ldl, const double *Y, int ldy,
                      const double *Cin, int64_t ldci, double *C, int64_t ldc, bool sub) {
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, g = lane >> 4, cl = lane & 15;
  const int64_t nrt = (m + 63) / 64;
  const int nct = (q + 63) / 64;
  for (int64_t t = wave; t < nrt * nct; t += 4) {
    const int64_t r0 = (t / nct) * 64;
    const int c0 = (int)(t % nct) * 64;
    const int64_t rl = r0 + 4 * cl;
    const bool full_rows = r0 + 64 <= m;
    d4 acc[4][4];
#pragma unroll
    for (int x = 0; x < 4; ++x)
#pragma unroll
      for (int y = 0; y < 4; ++y) acc[x][y] = d4{0.0, 0.0, 0.0, 0.0};
    if (sub) {
#pragma unroll
      for (int e = 0; e < 4; ++e)
#pragma unroll
        for (int x = 0; x < 4; ++x) {
          const int col = c0 + 4 * g + 16 * e + x;
          if (col < q) {
            const double *pc = Cin + (int64_t)col * ldci + rl;
#pragma unroll
            for (int y = 0; y < 4; ++y) acc[x][y][e] = (rl + y < m) ? pc[y] : 0.0;
          }
        }
    }
    const double *yb = Y + c0 + 4 * cl;
    const double *lb = L + (full_rows ? rl : 0);
    for (int kk = 0; kk < p; kk += 4) {
      const int k = kk + g;
      const bool kok = k < p;
      const int ks = kok ? k : 0;
      double av[4], bv[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const double yv = yb[ks * ldy + u];
        av[u] = kok ? yv : 0.0;
      }
      if (full_rows) {
#pragma unroll
        for (int u = 0; u < 4; ++u) bv[u] = kok ? lb[(int64_t)ks * ldl + u] : 0.0;
      } else {
#pragma unroll
        for (int u = 0; u < 4; ++u) bv[u] = (kok && rl + u < m) ? L[(int64_t)ks * ldl + rl + u] : 0.0;
      }
#pragma unroll
      for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 4; ++y) acc[x][y] = mfma16x16x4(av[x], bv[y], acc[x][y]);
    }
#pragma unroll
    for (int e = 0; e < 4; ++e)
#pragma unroll
      for (int x = 0; x < 4; ++x) {
        const int col = c0 + 4 * g + 16 * e + x;
        if (col < q) {
          double *pc = C + (int64_t)col * ldc + rl;
#pragma unroll
          for (int y = 0; y < 4; ++y)
            if (rl + y < m) pc[y] = acc[x][y][e];
        }
      }
  }
  wg_sync();
}

// Cholesky of W (LDS, row-major w x w, upper read) into uout (row-major, ld
// w) and its inverse into ui (row-major, ld ldu). Returns the failing 1-based
// panel column or 0 (uniform over the workgroup).
__device__ __forceinline__ int wg_chol_inv(const Lds &S, int w, double *uout, int ldu) {
  const int tid = threadIdx.x;
  for (int e = tid; e < w * w; e += kThreads) {
    const int i = e / w, j = e % w;
    S.s[e] = (i <= j) ? S.w[e] : 0.0;
  }
  __syncthreads();
  const int fail = lds_cholesky(S.s, S.d, w);
  if (fail) {
    __syncthreads();
    return fail;
  }
  for (int e = tid; e < w * w; e += kThreads) {
    const int i = e / w, j = e % w;
    uout[e] = (i < j) ? S.s[e] : (i == j ? S.d[i] : 0.0);
  }
  __syncthreads();
  for (int k = tid; k < w; k += kThreads) S.s[k * w + k] = S.d[k];
  __syncthreads();
  lds_upper_inverse(S.s, S.d, w);
  for (int e = tid; e < w * ldu; e += kThreads) {
    const int i = e / ldu, c = e % ldu;
    S.ui[e] = (c < i || c >= w) ? 0.0 : (c == i ? S.d[i] : S.s[c * w + i]);
  }
  __syncthreads();
  return 0;
}

// R (column-major, ld n) block at (r0, c0), w x w: Ub * Ua (uppers, ld w)
__device__ __forceinline__ void wg_r_upper_product(double *R, int n, int r0, int w, const double *Ub,
                                   const double *Ua) {
  for (int e = threadIdx.x; e < w * w; e += kThreads) {
    const int i = e % w, c = e / w;
    double acc = 0.0;
    for (int k = i; k <= c; ++k) acc += Ub[i * w + k] * Ua[k * w + c];
    R[(r0 + i) + (int64_t)(r0 + c) * n] = (i <= c) ? acc : 0.0;
  }
}

// mCQR2GS of one matrix by one workgroup. Returns 0 or the breakdown column.
__device__ __forceinline__ int wg_mcqr2gs(const Lds &S, int64_t m, int n, int b, const double *A, int64_t lda,
                          double *Q, double *R) {
  const int tid = threadIdx.x;
  for (int e = tid; e < n * n; e += kThreads) R[e] = 0.0;
  const int w0 = n < b ? n : b;
  int ldu = (int)padded_ld(w0);
  // first panel: CholeskyQR2, reading A and writing Q
  wg_tn(m, w0, w0, A, lda, A, lda, true, S.w, w0);
  int fail = wg_chol_inv(S, w0, S.ua, ldu);
  if (fail) return fail;
  wg_nn(m, w0, w0, A, lda, S.ui, ldu, nullptr, 0, Q, lda, false);
  wg_tn(m, w0, w0, Q, lda, Q, lda, true, S.w, w0);
  fail = wg_chol_inv(S, w0, S.ub, ldu);
  if (fail) return fail;
  wg_nn(m, w0, w0, Q, lda, S.ui, ldu, nullptr, 0, Q, lda, false);
  wg_r_upper_product(R, n, 0, w0, S.ub, S.ua);
  for (int s = b; s < n; s += b) {
    const int ps = s - b, w = (n - s < b) ? n - s : b, nr = n - s;
    const double *Ar = (ps == 0) ? A + (int64_t)s * lda : Q + (int64_t)s * lda;
    double *Xj = Q + (int64_t)s * lda;
    const double *Qprev = Q + (int64_t)ps * lda;
    // Y := Q_{j-1}^T A_{:,j:k}; R_{j-1,j:k} := Y; A_{:,j:k} -= Q_{j-1} Y
    int ldy = (int)padded_ld(nr);
    wg_tn(m, b, nr, Qprev, lda, Ar, lda, false, S.y, ldy);
    for (int e = tid; e < b * nr; e += kThreads) {
      const int i = e / nr, j = e % nr;
      R[(ps + i) + (int64_t)(s + j) * n] = S.y[i * ldy + j];
      S.y[i * ldy + j] = -S.y[i * ldy + j];
    }
    __syncthreads();
    wg_nn(m, b, nr, Qprev, lda, S.y, ldy, Ar, lda, Xj, lda, true);
    // CQR of panel j: A_j = Qt Ua
    ldu = (int)padded_ld(w);
    wg_tn(m, w, w, Xj, lda, Xj, lda, true, S.w, w);
    fail = wg_chol_inv(S, w, S.ua, ldu);
    if (fail) return s + fail;
    wg_nn(m, w, w, Xj, lda, S.ui, ldu, nullptr, 0, Xj, lda, false);
    // re-orthogonalise: Z := Q_{1:j-1}^T Qt; Qt -= Q_{1:j-1} Z; R_{1:j-1,j} += Z Ua
    ldy = (int)padded_ld(w);
    wg_tn(m, s, w, Q, lda, Xj, lda, false, S.y, ldy);
    for (int e = tid; e < s * w; e += kThreads) {
      const int i = e % s, c = e / s;
      double acc = 0.0;
      for (int k = 0; k <= c; ++k) acc += S.y[i * ldy + k] * S.ua[k * w + c];
      R[i + (int64_t)(s + c) * n] += acc;
    }
    __syncthreads();
    for (int e = tid; e < s * ldy; e += kThreads) S.y[e] = -S.y[e];
    __syncthreads();
    wg_nn(m, s, w, Q, lda, S.y, ldy, Xj, lda, Xj, lda, true);
    // CQR again: Qt = Q_j Ub; R_jj = Ub Ua
    wg_tn(m, w, w, Xj, lda, Xj, lda, true, S.w, w);
    fail = wg_chol_inv(S, w, S.ub, ldu);
    if (fail) return s + fail;
    wg_nn(m, w, w, Xj, lda, S.ui, ldu, nullptr, 0, Xj, lda, false);
    wg_r_upper_product(R, n, s, w, S.ub, S.ua);
    __syncthreads();
  }
  return 0;
}

__global__ void k_set_int_batched(int *p) { *p = 0; }

__global__ __launch_bounds__(kThreads) void k_batched_mod(
    const int *__restrict__ order, const int64_t *__restrict__ ms, const int *__restrict__ ns,
    const int *__restrict__ bs, int count, const double *const *__restrict__ dA,
    const int64_t *__restrict__ dlda, double *const *__restrict__ dQ, double *const *__restrict__ dR,
    int *__restrict__ dinfo, int *queue) {
  extern __shared__ double lds[];
  const Lds S = lds_layout(lds);
  const int tid = threadIdx.x;
  for (;;) {
    if (tid == 0) *S.flag = atomicAdd(queue, 1);
    __syncthreads();
    const int slot = *S.flag;
    __syncthreads();
    if (slot >= count) break;  // uniform: every wave leaves together
    const int i = order[slot];
    const int fail = wg_mcqr2gs(S, ms[i], ns[i], bs[i], dA[i], dlda[i], dQ[i], dR[i]);
    if (tid == 0) dinfo[i] = fail;
    wg_sync();
  }
}

}  // namespace

size_t batched_lds_bytes() {
  return (size_t)(kYSize + 4 * kBB + 64 + kBB + kBatchMaxPanel) * sizeof(double) + 64;
}

hipError_t launch_batched_mod(int grid, const int *order, const int64_t *ms, const int *ns,
                              const int *bs, int count, const double *const *dA, const int64_t *dlda,
                              double *const *dQ, double *const *dR, int *dinfo, int *queue,
                              hipStream_t s) {
  static bool attr_set = false;
  const size_t lds = batched_lds_bytes();
  if (!attr_set) {
    const hipError_t e = hipFuncSetAttribute((const void *)k_batched_mod,
                                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  hipLaunchKernelGGL(k_set_int_batched, dim3(1), dim3(1), 0, s, queue);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_batched_mod, dim3((unsigned)grid), dim3(kThreads), lds, s, order, ms, ns, bs,
                     count, dA, dlda, dQ, dR, dinfo, queue);
  return hipGetLastError();
}

int batched_blocks_per_cu() {
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, (const void *)k_batched_mod, kThreads,
                                                   batched_lds_bytes()) != hipSuccess)
    return 1;
  return nb > 0 ? nb : 1;
}

}  // namespace cqr
