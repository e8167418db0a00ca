// libcqr device kernels for gfx950 (CDNA4, wave64, FP64 MFMA).
//
// The streaming steps of CholeskyQR with block Gram-Schmidt (Algorithms 1, 6,
// 8 and 9 of arXiv 2405.04237) are two shapes of FP64 matrix product:
//
//  * "TN" (k_tn): P = L^T Rt reduced over the m rows -- the panel Gram
//    W_j = A_j^T A_j and the projections Y = Q_j^T A_rest, Z = Q_{1:j-1}^T Qt.
//    The paper forms local products on each rank and sums them with an
//    Allreduce (Algorithm 2; Algorithm 8). On one GPU the row blocks are
//    chunks of rows handled by different waves; each wave writes one partial
//    and k_reduce sums the partials in a fixed order (deterministic).
//  * "NN" (k_nn): C = +-L Y (+ C) streamed over the rows -- Q_j = A_j U^{-1}
//    through an explicit triangular inverse, and the updates A_rest -= Q_j Y,
//    Qt -= Q_{1:j-1} Z.
//
// Both use v_mfma_f64_16x16x4_f64 with operands loaded straight from global
// memory into registers in the instruction's fragment layout:
//   A operand (16x4): lane l holds A[l % 16][l / 16]
//   B operand (4x16): lane l holds B[l / 16][l % 16]
//   D (16x16):        lane l, element r holds D[l / 16 + 4 r][l % 16]
// In k_tn the reduction index is the row; the four rows a lane group feeds in
// one instruction are permuted so that each lane reads 4 consecutive rows of
// one column (32 bytes), and a wave's 4 lane groups cover 16 consecutive rows
// (one 128-byte line per column). Row order inside a sum does not change the
// product; it changes only rounding, and the order is fixed.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "kernels.h"

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

// ----------------------------------------------------------------------------
// k_tn: split-m partial products. One wave per (row chunk, 64x64 tile).
// ----------------------------------------------------------------------------
template <bool GRAM, bool VEC>
__global__ __launch_bounds__(64) void k_tn(int64_t m, int p, int q, const double *__restrict__ L,
                                           int64_t ldl, const double *__restrict__ Rt, int64_t ldr,
                                           double *__restrict__ part, int64_t rc, int tp, int tq,
                                           const int *__restrict__ info) {
  if (*info) return;
  const int64_t lid = xcd_logical(blockIdx.x, gridDim.x);
  const int T = GRAM ? tp * (tp + 1) / 2 : tp * tq;
  const int64_t c = lid / T;
  int t = (int)(lid % T);
  int ti, tj;
  if (GRAM) {
    ti = 0;
    int len = tp;
    while (t >= len) {
      t -= len;
      ++ti;
      --len;
    }
    tj = ti + t;
  } else {
    ti = t / tq;
    tj = t % tq;
  }
  const int lane = threadIdx.x, g = lane >> 4, cl = lane & 15;
  const int i0 = ti * kTile, j0 = tj * kTile;
  const int64_t rb = c * rc;
  const int64_t re = (m < rb + rc) ? m : rb + rc;
  const int64_t nsteps = (re - rb) / 16;  // full 16-row steps; the rest is the tail

  // Columns past p (or q) are read from column 0 instead of being masked: a
  // lane's operand only reaches the output row (column) it indexes, and
  // those outputs are never stored. This keeps the hot loop free of selects.
  const double *pa[4];
  const double *pb[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int ca = i0 + 16 * u + cl, cb = j0 + 16 * u + cl;
    pa[u] = L + (int64_t)(ca < p ? ca : 0) * ldl + rb + 4 * g;
    pb[u] = Rt + (int64_t)(cb < q ? cb : 0) * ldr + rb + 4 * g;
  }

  d4 acc[4][4];
#pragma unroll
  for (int x = 0; x < 4; ++x)
#pragma unroll
    for (int y = 0; y < 4; ++y) acc[x][y] = d4{0.0, 0.0, 0.0, 0.0};

  auto load = [&](double (&da)[4][4], double (&db)[4][4], int64_t off) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      if (VEC) {
        const double2 *xa = reinterpret_cast<const double2 *>(pa[u] + off);
        const double2 *xb = reinterpret_cast<const double2 *>(pb[u] + off);
        const double2 a0 = xa[0], a1 = xa[1], b0 = xb[0], b1 = xb[1];
        da[u][0] = a0.x;
        da[u][1] = a0.y;
        da[u][2] = a1.x;
        da[u][3] = a1.y;
        db[u][0] = b0.x;
        db[u][1] = b0.y;
        db[u][2] = b1.x;
        db[u][3] = b1.y;
      } else {
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          da[u][s] = pa[u][off + s];
          db[u][s] = pb[u][off + s];
        }
      }
    }
  };
  auto compute = [&](const double (&da)[4][4], const double (&db)[4][4]) {
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 4; ++y) acc[x][y] = mfma16x16x4(da[x][s], db[y][s], acc[x][y]);
  };

  double a0[4][4], b0[4][4], a1[4][4], b1[4][4];
  if (nsteps > 0) {
    // Ping-pong over two register sets, the next step's loads issued before
    // this step's MFMAs (the scheduling barriers keep the compiler from
    // sinking the loads next to their uses). The prefetch offset is clamped
    // to the last full step, so every load stays inside the chunk.
    load(a0, b0, 0);
    int64_t it = 0;
    for (; it + 2 <= nsteps; it += 2) {
      load(a1, b1, 16 * (it + 1));
      __builtin_amdgcn_sched_barrier(0);
      compute(a0, b0);
      __builtin_amdgcn_sched_barrier(0);
      load(a0, b0, 16 * ((it + 2 < nsteps) ? it + 2 : nsteps - 1));
      __builtin_amdgcn_sched_barrier(0);
      compute(a1, b1);
      __builtin_amdgcn_sched_barrier(0);
    }
    if (it < nsteps) compute(a0, b0);
  }
  const int64_t rt = rb + 16 * nsteps;
  if (rt < re) {  // ragged tail: rows rt + 4g + s < re only
    const int64_t off = 16 * nsteps;
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const bool ok = (rt + 4 * g + s) < re;
        a0[u][s] = ok ? pa[u][off + s] : 0.0;
        b0[u][s] = ok ? pb[u][off + s] : 0.0;
      }
    compute(a0, b0);
  }

  double *out = part + (size_t)c * (size_t)p * (size_t)q;
#pragma unroll
  for (int x = 0; x < 4; ++x)
#pragma unroll
    for (int y = 0; y < 4; ++y)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int I = i0 + 16 * x + g + 4 * e, J = j0 + 16 * y + cl;
        if (I < p && J < q) out[(size_t)I * q + J] = acc[x][y][e];
      }
}

int64_t tn_tiles(bool gram, int p, int q) {
  const int tp = (p + kTile - 1) / kTile, tq = (q + kTile - 1) / kTile;
  return gram ? (int64_t)tp * (tp + 1) / 2 : (int64_t)tp * tq;
}

hipError_t launch_tn(bool gram, int64_t m, int p, int q, const double *L, int64_t ldl,
                     const double *Rt, int64_t ldr, double *part, int64_t rc, int64_t nch,
                     const int *info, hipStream_t s) {
  const int tp = (p + kTile - 1) / kTile, tq = (q + kTile - 1) / kTile;
  const int64_t nb = tn_tiles(gram, p, q) * nch;
  const bool vec = (ldl % 2 == 0) && (ldr % 2 == 0) && ((uintptr_t)L % 16 == 0) &&
                   ((uintptr_t)Rt % 16 == 0) && (rc % 16 == 0);
  dim3 grid((unsigned)nb), block(64);
  if (gram) {
    if (vec)
      hipLaunchKernelGGL((k_tn<true, true>), grid, block, 0, s, m, p, q, L, ldl, Rt, ldr, part, rc, tp, tq, info);
    else
      hipLaunchKernelGGL((k_tn<true, false>), grid, block, 0, s, m, p, q, L, ldl, Rt, ldr, part, rc, tp, tq, info);
  } else {
    if (vec)
      hipLaunchKernelGGL((k_tn<false, true>), grid, block, 0, s, m, p, q, L, ldl, Rt, ldr, part, rc, tp, tq, info);
    else
      hipLaunchKernelGGL((k_tn<false, false>), grid, block, 0, s, m, p, q, L, ldl, Rt, ldr, part, rc, tp, tq, info);
  }
  return hipGetLastError();
}

// ----------------------------------------------------------------------------
// k_nn: row-streaming product C = L Y (+ C), one wave per 64 x 64 tile of C.
// The trailing update C -= Q Y is run as C + Q (-Y): the reduction that
// produces Y also stores its negation, so the hot loop feeds loaded values
// straight to the MFMAs. A workgroup holds 4 waves arranged WR x WC (WR * WC = 4) over rows x
// columns, so narrow products (the b-column Q_j = X U^{-1}) still keep all
// four waves busy. Lane/element maps (cl = lane % 16, g = lane / 16):
//   B operand, block y: lane holds L[r0 + 4 cl + y][k],  k = kk + g
//   A operand, block x: lane holds Y[k][c0 + 4 cl + x]
//   D element e of block (x, y): C[r0 + 4 cl + y][c0 + 4 g + 16 e + x]
// so that every lane's L, Y and C accesses are 4 consecutive doubles (32 B)
// and 16 lanes cover 64 consecutive rows (or columns) of one line.
// ----------------------------------------------------------------------------
template <bool SUB, bool TRI, bool VEC>
__global__ __launch_bounds__(256) void k_nn(int64_t m, int p, int q, const double *L, int64_t ldl,
                                            const double *__restrict__ Y, int64_t ldy, double *C,
                                            int64_t ldc, int wr, int ncg,
                                            const int *__restrict__ info) {
  if (*info) return;
  const int64_t lid = xcd_logical(blockIdx.x, gridDim.x);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, g = lane >> 4, cl = lane & 15;
  const int wc = 4 / wr;
  const int64_t r0 = (lid / ncg * wr + wave % wr) * (int64_t)kTile;
  const int c0 = ((int)(lid % ncg) * wc + wave / wr) * kTile;
  const bool active = c0 < q && r0 < m;
  const int64_t rl = r0 + 4 * cl;  // first of this lane's 4 rows
  const int yc = c0 + 4 * cl;      // first of this lane's 4 columns

  d4 acc[4][4];  // [column block x][row block y]
  if (active) {
#pragma unroll
    for (int x = 0; x < 4; ++x)
#pragma unroll
      for (int y = 0; y < 4; ++y) acc[x][y] = d4{0.0, 0.0, 0.0, 0.0};
    if (SUB) {
#pragma unroll
      for (int e = 0; e < 4; ++e)
#pragma unroll
        for (int x = 0; x < 4; ++x) {
          const int col = c0 + 4 * g + 16 * e + x;
          if (col < q) {
            const double *pc = C + (int64_t)col * ldc + rl;
            if (VEC && rl + 4 <= m) {
              const double2 v0 = reinterpret_cast<const double2 *>(pc)[0];
              const double2 v1 = reinterpret_cast<const double2 *>(pc)[1];
              acc[x][0][e] = v0.x;
              acc[x][1][e] = v0.y;
              acc[x][2][e] = v1.x;
              acc[x][3][e] = v1.y;
            } else {
#pragma unroll
              for (int y = 0; y < 4; ++y) acc[x][y][e] = (rl + y < m) ? pc[y] : 0.0;
            }
          }
        }
    }

    // k range: all of p, or (upper-triangular Y) only k < c0 + 64
    const int kend = TRI ? ((c0 + kTile < p) ? c0 + kTile : p) : p;
    // Fast path: the wave's 64 rows all exist and each lane's 4 columns are
    // either all < q or all >= q. A lane whose columns are all >= q reads
    // column 0 instead of being masked: its operand only reaches outputs that
    // are never stored. Everything else (the last, partial row tile; q not a
    // multiple of 4 at the right edge) takes the masked loop below.
    const bool fast = (r0 + kTile <= m) && ((q % 4) == 0 || c0 + kTile <= q);
    const double *lb = L + rl;
    const double *yb = Y + (yc < q ? yc : 0);
    auto load = [&](double (&da)[4][4], double (&db)[4][4], int kk) {
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const int k = kk + 4 * s + g;
        const double *py = yb + (int64_t)k * ldy;
        const double *pl = lb + (int64_t)k * ldl;
        if (VEC) {
          const double2 y0 = reinterpret_cast<const double2 *>(py)[0];
          const double2 y1 = reinterpret_cast<const double2 *>(py)[1];
          const double2 l0 = reinterpret_cast<const double2 *>(pl)[0];
          const double2 l1 = reinterpret_cast<const double2 *>(pl)[1];
          da[s][0] = y0.x;
          da[s][1] = y0.y;
          da[s][2] = y1.x;
          da[s][3] = y1.y;
          db[s][0] = l0.x;
          db[s][1] = l0.y;
          db[s][2] = l1.x;
          db[s][3] = l1.y;
        } else {
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            da[s][u] = py[u];
            db[s][u] = pl[u];
          }
        }
      }
    };
    auto compute = [&](const double (&da)[4][4], const double (&db)[4][4]) {
#pragma unroll
      for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int x = 0; x < 4; ++x)
#pragma unroll
          for (int y = 0; y < 4; ++y) acc[x][y] = mfma16x16x4(da[s][x], db[s][y], acc[x][y]);
    };
    double a0[4][4], b0[4][4], a1[4][4], b1[4][4];
    const int nit = fast ? kend / 16 : 0;  // full 16-wide k iterations
    if (nit > 0) {
      load(a0, b0, 0);
      int it = 0;
      for (; it + 2 <= nit; it += 2) {
        load(a1, b1, 16 * (it + 1));
        __builtin_amdgcn_sched_barrier(0);
        compute(a0, b0);
        __builtin_amdgcn_sched_barrier(0);
        load(a0, b0, 16 * ((it + 2 < nit) ? it + 2 : nit - 1));
        __builtin_amdgcn_sched_barrier(0);
        compute(a1, b1);
        __builtin_amdgcn_sched_barrier(0);
      }
      if (it < nit) compute(a0, b0);
    }
    // k tail (and the whole k range off the fast path): masked element loads
    for (int kk = 16 * nit; kk < kend; kk += 16) {
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const int k = kk + 4 * s + g;
        const bool kok = k < kend;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          a0[s][u] = (kok && yc + u < q) ? Y[(int64_t)k * ldy + yc + u] : 0.0;
          b0[s][u] = (kok && rl + u < m) ? L[(int64_t)k * ldl + rl + u] : 0.0;
        }
      }
      compute(a0, b0);
    }
  }
  if (!SUB) __syncthreads();  // in-place: every read of L precedes every write of C
  if (!active) return;
#pragma unroll
  for (int e = 0; e < 4; ++e)
#pragma unroll
    for (int x = 0; x < 4; ++x) {
      const int col = c0 + 4 * g + 16 * e + x;
      if (col < q) {
        double *pc = C + (int64_t)col * ldc + rl;
        if (VEC && rl + 4 <= m) {
          reinterpret_cast<double2 *>(pc)[0] = double2{acc[x][0][e], acc[x][1][e]};
          reinterpret_cast<double2 *>(pc)[1] = double2{acc[x][2][e], acc[x][3][e]};
        } else {
#pragma unroll
          for (int y = 0; y < 4; ++y)
            if (rl + y < m) pc[y] = acc[x][y][e];
        }
      }
    }
}

hipError_t launch_nn(bool subtract, bool upper_y, int64_t m, int p, int q, const double *L,
                     int64_t ldl, const double *Y, int64_t ldy, double *C, int64_t ldc,
                     const int *info, hipStream_t s) {
  const int slabs = (q + kTile - 1) / kTile;
  const int wc = slabs >= 4 ? 4 : (slabs >= 2 ? 2 : 1);
  const int wr = 4 / wc;
  const int ncg = (slabs + wc - 1) / wc;
  if (!subtract && ncg != 1) return hipErrorInvalidValue;  // in-place needs one column group
  const int64_t rts = (m + (int64_t)kTile * wr - 1) / ((int64_t)kTile * wr);
  const bool vec = (ldl % 2 == 0) && (ldc % 2 == 0) && (ldy % 2 == 0) && ((uintptr_t)L % 16 == 0) &&
                   ((uintptr_t)C % 16 == 0) && ((uintptr_t)Y % 16 == 0);
  dim3 grid((unsigned)(rts * ncg)), block(256);
#define CQR_NN(S, T, V)                                                                          \
  hipLaunchKernelGGL((k_nn<S, T, V>), grid, block, 0, s, m, p, q, L, ldl, Y, ldy, C, ldc, wr, ncg, \
                     info)
  if (subtract) {
    if (vec) CQR_NN(true, false, true); else CQR_NN(true, false, false);
  } else if (upper_y) {
    if (vec) CQR_NN(false, true, true); else CQR_NN(false, true, false);
  } else {
    if (vec) CQR_NN(false, false, true); else CQR_NN(false, false, false);
  }
#undef CQR_NN
  return hipGetLastError();
}
// ----------------------------------------------------------------------------
// k_reduce: fixed-order sum of split-m partials (replaces the Allreduce of
// Algorithms 2 and 8). Element e of every partial is summed by one thread in
// a binary-counter pairwise order over the chunk index, so the result does
// not depend on which wave finished first.
// ----------------------------------------------------------------------------
template <bool GRAM>
__global__ __launch_bounds__(256) void k_reduce(const double *__restrict__ part, int64_t nch, int p,
                                                int q, double *__restrict__ out, int64_t ldo,
                                                double *__restrict__ rblk, int64_t ldr, bool neg,
                                                const int *__restrict__ info) {
  if (*info) return;
  const int64_t pq = (int64_t)p * q;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= pq) return;
  const int i = (int)(e / q), j = (int)(e % q);
  if (GRAM && i > j) {
    out[(int64_t)i * p + j] = 0.0;
    return;
  }
  double stk[40];
  int top = 0;
  for (int64_t c = 0; c < nch; ++c) {
    double v = part[c * pq + e];
    for (uint64_t k = (uint64_t)c + 1; (k & 1) == 0; k >>= 1) v = stk[--top] + v;
    stk[top++] = v;
  }
  double sum = stk[top - 1];
  for (int t = top - 2; t >= 0; --t) sum = stk[t] + sum;
  if (GRAM) {
    out[(int64_t)i * p + j] = sum;
  } else {
    out[(int64_t)i * ldo + j] = neg ? -sum : sum;
    if (rblk) rblk[i + (int64_t)j * ldr] = sum;
  }
}

hipError_t launch_reduce(bool gram, const double *part, int64_t nch, int p, int q, double *out,
                         int64_t ldo, double *rblk, int64_t ldr, bool neg, const int *info,
                         hipStream_t s) {
  const int64_t pq = (int64_t)p * q;
  dim3 grid((unsigned)((pq + 255) / 256)), block(256);
  if (gram)
    hipLaunchKernelGGL((k_reduce<true>), grid, block, 0, s, part, nch, p, q, out, ldo, rblk, ldr, neg,
                       info);
  else
    hipLaunchKernelGGL((k_reduce<false>), grid, block, 0, s, part, nch, p, q, out, ldo, rblk, ldr, neg,
                       info);
  return hipGetLastError();
}

// ----------------------------------------------------------------------------
// k_chol_inv: Cholesky W = U^T U of one panel's Gram matrix (Algorithm 1 /
// Algorithm 8, Cholesky step) and the inverse U^{-1}, in one workgroup with
// the whole w x w matrix in LDS. Right-looking, row-oriented (upper factor);
// the inverse by a column sweep of back substitution U X = I, with X kept in
// the (unused) strict lower triangle of the LDS matrix, transposed.
// ----------------------------------------------------------------------------
constexpr int kCholThreads = 512;

__global__ __launch_bounds__(kCholThreads) void k_chol_inv(const double *__restrict__ W, int w,
                                                           double *__restrict__ uout,
                                                           double *__restrict__ rblk, int64_t ldr,
                                                           double *__restrict__ uinv, int *info,
                                                           int col0) {
  extern __shared__ double S[];  // w*w matrix, then w diagonal entries of X
  __shared__ int fail;
  if (*info) return;
  double *D = S + w * w;
  const int tid = threadIdx.x, nt = blockDim.x;
  if (tid == 0) fail = 0;
  for (int e = tid; e < w * w; e += nt) {
    const int i = e / w, j = e % w;
    S[e] = (i <= j) ? W[e] : 0.0;
  }
  __syncthreads();
  for (int k = 0; k < w; ++k) {
    if (tid == 0) {
      const double d = S[k * w + k];
      if (d > 0.0)
        S[k * w + k] = sqrt(d);
      else
        fail = k + 1;  // also taken for NaN
    }
    __syncthreads();
    if (fail) break;
    const double piv = S[k * w + k];
    for (int j = k + 1 + tid; j < w; j += nt) S[k * w + j] = S[k * w + j] / piv;
    __syncthreads();
    const int rem = w - k - 1;
    for (int e = tid; e < rem * rem; e += nt) {
      const int i = k + 1 + e / rem, j = k + 1 + e % rem;
      if (j >= i) S[i * w + j] = S[i * w + j] - S[k * w + i] * S[k * w + j];
    }
    __syncthreads();
  }
  if (fail) {
    if (tid == 0) atomicCAS(info, 0, col0 + fail);
    return;
  }
  for (int e = tid; e < w * w; e += nt) {
    const int i = e / w, j = e % w;
    const double u = (i <= j) ? S[e] : 0.0;
    if (uout) uout[e] = u;
    if (rblk) rblk[i + (int64_t)j * ldr] = u;
  }
  // inverse: X = U^{-1}; X[i][c] (i < c) lives at S[c*w + i], X[k][k] at D[k]
  for (int k = tid; k < w; k += nt) D[k] = 1.0;
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
    const int cols = w - k;
    for (int e = tid; e < k * cols; e += nt) {
      const int i = e % k, c = k + e / k;
      const double xkc = (c == k) ? D[k] : S[c * w + k];
      if (c == k)
        S[k * w + i] = S[k * w + i] - S[i * w + k] * xkc;
      else
        S[c * w + i] = S[c * w + i] - S[i * w + k] * xkc;
    }
    __syncthreads();
  }
  const int ldu = (int)padded_ld(w);
  for (int e = tid; e < w * ldu; e += nt) {
    const int i = e / ldu, c = e % ldu;
    uinv[e] = (c < i || c >= w) ? 0.0 : (c == i ? D[i] : S[c * w + i]);
  }
}

hipError_t launch_chol_inv(const double *W, int w, double *uout, double *rblk, int64_t ldr,
                           double *uinv, int *info, int col0, hipStream_t s) {
  if (w < 1 || w > kMaxPanel) return hipErrorInvalidValue;
  const size_t lds = ((size_t)w * w + w) * sizeof(double);
  static bool attr_set = false;
  if (!attr_set) {
    const size_t most = ((size_t)kMaxPanel * kMaxPanel + kMaxPanel) * sizeof(double);
    const hipError_t e = hipFuncSetAttribute((const void *)k_chol_inv,
                                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)most);
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  hipLaunchKernelGGL(k_chol_inv, dim3(1), dim3(kCholThreads), lds, s, W, w, uout, rblk, ldr, uinv,
                     info, col0);
  return hipGetLastError();
}

// ----------------------------------------------------------------------------
// Small R-block products (mCQR2GS bookkeeping and R = R2 R1 of CQR2GS).
// ----------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_r_add_zu(int s_rows, int w, const double *__restrict__ Z,
                                                  int64_t ldz, const double *__restrict__ Ua,
                                                  double *rblk, int64_t ldr,
                                                  const int *__restrict__ info) {
  if (*info) return;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= (int64_t)s_rows * w) return;
  const int i = (int)(e % s_rows), c = (int)(e / s_rows);
  double acc = 0.0;
  for (int k = 0; k <= c; ++k) acc += Z[(int64_t)i * ldz + k] * Ua[k * w + c];
  rblk[i + (int64_t)c * ldr] -= acc;
}

hipError_t launch_r_add_zu(int s_rows, int w, const double *Z, int64_t ldz, const double *Ua,
                           double *rblk, int64_t ldr, const int *info, hipStream_t s) {
  const int64_t n = (int64_t)s_rows * w;
  hipLaunchKernelGGL(k_r_add_zu, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, s_rows, w, Z,
                     ldz, Ua, rblk, ldr, info);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_r_upper_product(int w, const double *__restrict__ Ub,
                                                         const double *__restrict__ Ua, double *rblk,
                                                         int64_t ldr, const int *__restrict__ info) {
  if (*info) return;
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= w * w) return;
  const int i = e % w, c = e / w;
  double acc = 0.0;
  for (int k = i; k <= c; ++k) acc += Ub[i * w + k] * Ua[k * w + c];
  rblk[i + (int64_t)c * ldr] = (i <= c) ? acc : 0.0;
}

hipError_t launch_r_upper_product(int w, const double *Ub, const double *Ua, double *rblk,
                                  int64_t ldr, const int *info, hipStream_t s) {
  hipLaunchKernelGGL(k_r_upper_product, dim3((unsigned)((w * w + 255) / 256)), dim3(256), 0, s, w,
                     Ub, Ua, rblk, ldr, info);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_trmm_upper(int n, const double *__restrict__ R2,
                                                    const double *__restrict__ R1,
                                                    double *__restrict__ R,
                                                    const int *__restrict__ info) {
  if (*info) return;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= (int64_t)n * n) return;
  const int i = (int)(e % n), c = (int)(e / n);
  double acc = 0.0;
  for (int k = i; k <= c; ++k) acc += R2[i + (int64_t)k * n] * R1[k + (int64_t)c * n];
  R[e] = (i <= c) ? acc : 0.0;
}

hipError_t launch_trmm_upper(int n, const double *R2, const double *R1, double *R, const int *info,
                             hipStream_t s) {
  const int64_t nn = (int64_t)n * n;
  hipLaunchKernelGGL(k_trmm_upper, dim3((unsigned)((nn + 255) / 256)), dim3(256), 0, s, n, R2, R1,
                     R, info);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_zero(double *p, int64_t count) {
  const int64_t stride = (int64_t)gridDim.x * 256;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < count; e += stride) p[e] = 0.0;
}

__global__ void k_set_int(int *p, int v) { *p = v; }

hipError_t launch_set_int(int *p, int v, hipStream_t s) {
  hipLaunchKernelGGL(k_set_int, dim3(1), dim3(1), 0, s, p, v);
  return hipGetLastError();
}

hipError_t launch_zero(double *p, int64_t count, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  int64_t blocks = (count + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_zero, dim3((unsigned)blocks), dim3(256), 0, s, p, count);
  return hipGetLastError();
}

}  // namespace cqr
