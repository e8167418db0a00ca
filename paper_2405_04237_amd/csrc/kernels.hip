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

#include <algorithm>
#include <type_traits>

#include "device_common.h"
#include "kernels.h"

namespace cqr {

// ----------------------------------------------------------------------------
// k_tn: split-m partial products. One wave per (row chunk, 64x64 tile).
// UPPER: only tiles on or above the diagonal (p == q), e.g. a Gram matrix.
// ----------------------------------------------------------------------------
template <bool UPPER, bool VEC>
__global__ __launch_bounds__(64) void k_tn(int64_t m, int p, int q, const double *__restrict__ L,
                                           int64_t ldl, const double *__restrict__ Rt, int64_t ldr,
                                           double *__restrict__ part, int64_t rc, int tp, int tq,
                                           int64_t sL, int64_t sRt, int64_t sPart,
                                           const int *__restrict__ info) {
  if (*info) return;
  L += blockIdx.y * sL;  // batch: one matrix per grid row
  Rt += blockIdx.y * sRt;
  part += blockIdx.y * sPart;
  const int64_t lid = xcd_logical(blockIdx.x, gridDim.x);
  const int T = UPPER ? tp * (tp + 1) / 2 : tp * tq;
  const int64_t c = lid / T;
  int t = (int)(lid % T);
  int ti, tj;
  if (UPPER) {
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

  // A diagonal tile of an upper product needs only the blocks on or above
  // its diagonal (the reduction reads i <= j only), and when both operands
  // are the same matrix (a Gram) its two column sets coincide: such tiles
  // issue 10 of the 16 MFMAs per step and load one column set instead of two.
  auto body = [&](auto diag_c, auto same_c) {
    constexpr bool DIAG = decltype(diag_c)::value, SAME = decltype(same_c)::value;
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
          const double2 a0 = xa[0], a1 = xa[1];
          da[u][0] = a0.x;
          da[u][1] = a0.y;
          da[u][2] = a1.x;
          da[u][3] = a1.y;
          if (!SAME) {
            const double2 *xb = reinterpret_cast<const double2 *>(pb[u] + off);
            const double2 b0 = xb[0], b1 = xb[1];
            db[u][0] = b0.x;
            db[u][1] = b0.y;
            db[u][2] = b1.x;
            db[u][3] = b1.y;
          }
        } else {
#pragma unroll
          for (int s = 0; s < 4; ++s) {
            da[u][s] = pa[u][off + s];
            if (!SAME) db[u][s] = pb[u][off + s];
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
          for (int y = 0; y < 4; ++y)
            if (!DIAG || x <= y) acc[x][y] = mfma16x16x4(da[x][s], SAME ? da[y][s] : db[y][s], acc[x][y]);
    };

    // Three register sets in a ring: while one step's MFMAs run, the loads of
    // the next two steps are in flight (about 8K cycles of cover at the FP64
    // MFMA rate). The scheduling barriers keep the compiler from sinking the
    // loads next to their uses. Prefetch offsets are clamped to the last full
    // step, so every load stays inside the chunk.
    double a0[4][4], b0[4][4], a1[4][4], b1[4][4], a2[4][4], b2[4][4];
    if (nsteps > 0) {
      auto at = [&](int64_t st) -> int64_t { return 16 * (st < nsteps ? st : nsteps - 1); };
      load(a0, b0, 0);
      load(a1, b1, at(1));
      int64_t it = 0;
      for (; it + 3 <= nsteps; it += 3) {
        load(a2, b2, at(it + 2));
        __builtin_amdgcn_sched_barrier(0);
        compute(a0, b0);
        __builtin_amdgcn_sched_barrier(0);
        load(a0, b0, at(it + 3));
        __builtin_amdgcn_sched_barrier(0);
        compute(a1, b1);
        __builtin_amdgcn_sched_barrier(0);
        load(a1, b1, at(it + 4));
        __builtin_amdgcn_sched_barrier(0);
        compute(a2, b2);
        __builtin_amdgcn_sched_barrier(0);
      }
      if (it < nsteps) compute(a0, b0);
      if (it + 1 < nsteps) compute(a1, b1);
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
          if (!SAME) b0[u][s] = ok ? pb[u][off + s] : 0.0;
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
          if ((!DIAG || x <= y) && I < p && J < q) out[(size_t)I * q + J] = acc[x][y][e];
        }
  };
  using T_ = std::true_type;
  using F_ = std::false_type;
  if (UPPER && ti == tj) {
    if (L == Rt && ldl == ldr)
      body(T_{}, T_{});
    else
      body(T_{}, F_{});
  } else {
    body(F_{}, F_{});
  }
}

// k_gram128: the Gram matrix W = X^T X of a 128-column panel, split-m as
// k_tn. Its upper triangle is 36 blocks of 16 x 16. With 64 x 64 tiles the
// two diagonal tiles carry 10 needed blocks and the off-diagonal one 16, so
// the waves that draw two off-diagonal tiles set the kernel's length. Here
// two waves share a row chunk and take 18 blocks each: block rows {0, 1, 6,
// 7} (which reach all 8 column blocks) and {2, 3, 4, 5} (column blocks 2..7).
// Every wave issues 72 MFMAs per 16-row step and loads only the column
// blocks its rows reach. Lane maps and the register ring as in k_tn.
// SAME = false: the upper part of X^T Y for two different 128-column
// operands (the adjoint's dQ^T Q): the same split, each half also loading
// its four row blocks of X.
__host__ __device__ constexpr int gram128_row(int half, int i) {
  return half ? 2 + i : (i < 2 ? i : 4 + i);
}

template <bool VEC, bool SAME>
__global__ __launch_bounds__(64) void k_gram128(int64_t m, const double *__restrict__ X, int64_t ldx,
                                                const double *__restrict__ Y, int64_t ldy,
                                                double *__restrict__ part, int64_t rc,
                                                const int *__restrict__ info) {
  if (*info) return;
  const int64_t lid = xcd_logical(blockIdx.x, gridDim.x);
  const int64_t c = lid >> 1;
  const int lane = threadIdx.x, g = lane >> 4, cl = lane & 15;
  const int64_t rb = c * rc;
  const int64_t re = (m < rb + rc) ? m : rb + rc;
  const int64_t nsteps = (re - rb) / 16;

  auto body = [&](auto half_c) {
    constexpr int H = decltype(half_c)::value;
    constexpr int CB0 = H ? 2 : 0;  // first column block this half reads
    constexpr int NCB = 8 - CB0;
    // SAME: one set of column lines serves both operands; otherwise the
    // half's four row blocks of X are loaded beside Y's column blocks
    constexpr int NA = SAME ? 0 : 4;
    const double *pc[NCB];
    const double *pr[4];
#pragma unroll
    for (int u = 0; u < NCB; ++u) pc[u] = Y + (int64_t)(16 * (CB0 + u) + cl) * ldy + rb + 4 * g;
#pragma unroll
    for (int i = 0; i < 4; ++i)
      pr[i] = X + (int64_t)(16 * gram128_row(H, i) + cl) * ldx + rb + 4 * g;

    d4 acc[4][8];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int y = 0; y < 8; ++y) acc[i][y] = d4{0.0, 0.0, 0.0, 0.0};

    auto ld4 = [&](const double *ptr, double (&v)[4]) {
      if (VEC) {
        const double2 *xa = reinterpret_cast<const double2 *>(ptr);
        const double2 a0 = xa[0], a1 = xa[1];
        v[0] = a0.x;
        v[1] = a0.y;
        v[2] = a1.x;
        v[3] = a1.y;
      } else {
#pragma unroll
        for (int s = 0; s < 4; ++s) v[s] = ptr[s];
      }
    };
    typedef double Stage[NCB + NA][4];
    auto load = [&](Stage &d, int64_t off) {
#pragma unroll
      for (int u = 0; u < NCB; ++u) ld4(pc[u] + off, d[u]);
#pragma unroll
      for (int i = 0; i < NA; ++i) ld4(pr[i] + off, d[NCB + i]);
    };
    auto compute = [&](const Stage &d) {
#pragma unroll
      for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int y = 0; y < 8; ++y) {
            const int x = gram128_row(H, i);
            if (y >= x) {
              if constexpr (SAME)
                acc[i][y] = mfma16x16x4(d[x - CB0][s], d[y - CB0][s], acc[i][y]);
              else
                acc[i][y] = mfma16x16x4(d[NCB + i][s], d[y - CB0][s], acc[i][y]);
            }
          }
    };

    // three stages in the ring for one operand, two for two (the register
    // budget); scheduling barriers as in k_tn
    if (nsteps > 0) {
      auto at = [&](int64_t st) -> int64_t { return 16 * (st < nsteps ? st : nsteps - 1); };
      if constexpr (SAME) {
        Stage d0, d1, d2;
        load(d0, 0);
        load(d1, at(1));
        int64_t it = 0;
        for (; it + 3 <= nsteps; it += 3) {
          load(d2, at(it + 2));
          __builtin_amdgcn_sched_barrier(0);
          compute(d0);
          __builtin_amdgcn_sched_barrier(0);
          load(d0, at(it + 3));
          __builtin_amdgcn_sched_barrier(0);
          compute(d1);
          __builtin_amdgcn_sched_barrier(0);
          load(d1, at(it + 4));
          __builtin_amdgcn_sched_barrier(0);
          compute(d2);
          __builtin_amdgcn_sched_barrier(0);
        }
        if (it < nsteps) compute(d0);
        if (it + 1 < nsteps) compute(d1);
      } else {
        Stage d0, d1;
        load(d0, 0);
        int64_t it = 0;
        for (; it + 2 <= nsteps; it += 2) {
          load(d1, at(it + 1));
          __builtin_amdgcn_sched_barrier(0);
          compute(d0);
          __builtin_amdgcn_sched_barrier(0);
          load(d0, at(it + 2));
          __builtin_amdgcn_sched_barrier(0);
          compute(d1);
          __builtin_amdgcn_sched_barrier(0);
        }
        if (it < nsteps) compute(d0);
      }
    }
    const int64_t rt = rb + 16 * nsteps;
    if (rt < re) {  // ragged tail: rows rt + 4g + s < re only
      const int64_t off = 16 * nsteps;
      Stage d;
#pragma unroll
      for (int u = 0; u < NCB + NA; ++u)
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          const double *ptr = (u < NCB) ? pc[u] : pr[u - NCB];
          d[u][s] = ((rt + 4 * g + s) < re) ? ptr[off + s] : 0.0;
        }
      compute(d);
    }

    double *out = part + (size_t)c * 128 * 128;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int y = 0; y < 8; ++y) {
        const int x = gram128_row(H, i);
        if (y >= x) {
#pragma unroll
          for (int e = 0; e < 4; ++e) out[(16 * x + g + 4 * e) * 128 + 16 * y + cl] = acc[i][y][e];
        }
      }
  };
  if (lid & 1)
    body(std::integral_constant<int, 1>{});
  else
    body(std::integral_constant<int, 0>{});
}

// k_tn_wide: the projection form (not a Gram) with a 64 x 128 output tile
// per wave (4 x 8 blocks: 256 accumulator registers, all in AGPRs) and a
// two-stage register ring (128 MFMAs of cover per stage). Each 16-row step
// loads 192 column segments for 128 MFMAs instead of 128 for 64, which moves
// the kernel from load- to MFMA-bound. Lane maps as in k_tn.
template <bool VEC>
__global__ __launch_bounds__(64) void k_tn_wide(int64_t m, int p, int q, const double *__restrict__ L,
                                                int64_t ldl, const double *__restrict__ Rt,
                                                int64_t ldr, double *__restrict__ part, int64_t rc,
                                                int tp, int tq, const int *__restrict__ info) {
  if (*info) return;
  const int64_t lid = xcd_logical(blockIdx.x, gridDim.x);
  const int T = tp * tq;
  const int64_t c = lid / T;
  const int t = (int)(lid % T);
  const int ti = t / tq, tj = t % tq;
  const int lane = threadIdx.x, g = lane >> 4, cl = lane & 15;
  const int i0 = ti * kTile, j0 = tj * 2 * kTile;
  const int64_t rb = c * rc;
  const int64_t re = (m < rb + rc) ? m : rb + rc;
  const int64_t nsteps = (re - rb) / 16;
  // out-of-range columns read column 0 (their outputs are never stored)
  const double *pa[4];
  const double *pb[8];
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int ca = i0 + 16 * u + cl;
    pa[u] = L + (int64_t)(ca < p ? ca : 0) * ldl + rb + 4 * g;
  }
#pragma unroll
  for (int u = 0; u < 8; ++u) {
    const int cb = j0 + 16 * u + cl;
    pb[u] = Rt + (int64_t)(cb < q ? cb : 0) * ldr + rb + 4 * g;
  }
  d4 acc[4][8];
#pragma unroll
  for (int x = 0; x < 4; ++x)
#pragma unroll
    for (int y = 0; y < 8; ++y) acc[x][y] = d4{0.0, 0.0, 0.0, 0.0};
  auto ld4 = [&](const double *ptr, double (&v)[4]) {
    if (VEC) {
      const double2 *x2 = reinterpret_cast<const double2 *>(ptr);
      const double2 a = x2[0], b = x2[1];
      v[0] = a.x;
      v[1] = a.y;
      v[2] = b.x;
      v[3] = b.y;
    } else {
#pragma unroll
      for (int s = 0; s < 4; ++s) v[s] = ptr[s];
    }
  };
  auto load = [&](double (&da)[4][4], double (&db)[8][4], int64_t off) {
#pragma unroll
    for (int u = 0; u < 4; ++u) ld4(pa[u] + off, da[u]);
#pragma unroll
    for (int u = 0; u < 8; ++u) ld4(pb[u] + off, db[u]);
  };
  auto compute = [&](const double (&da)[4][4], const double (&db)[8][4]) {
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 8; ++y) acc[x][y] = mfma16x16x4(da[x][s], db[y][s], acc[x][y]);
  };
  double a0[4][4], b0[8][4];
  if (nsteps > 0) {
    double a1[4][4], b1[8][4];
    auto at = [&](int64_t st) -> int64_t { return 16 * (st < nsteps ? st : nsteps - 1); };
    load(a0, b0, 0);
    int64_t it = 0;
    for (; it + 2 <= nsteps; it += 2) {
      load(a1, b1, at(it + 1));
      __builtin_amdgcn_sched_barrier(0);
      compute(a0, b0);
      __builtin_amdgcn_sched_barrier(0);
      load(a0, b0, at(it + 2));
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
      for (int s = 0; s < 4; ++s) a0[u][s] = ((rt + 4 * g + s) < re) ? pa[u][off + s] : 0.0;
#pragma unroll
    for (int u = 0; u < 8; ++u)
#pragma unroll
      for (int s = 0; s < 4; ++s) b0[u][s] = ((rt + 4 * g + s) < re) ? pb[u][off + s] : 0.0;
    compute(a0, b0);
  }
  double *out = part + (size_t)c * (size_t)p * (size_t)q;
#pragma unroll
  for (int x = 0; x < 4; ++x)
#pragma unroll
    for (int y = 0; y < 8; ++y)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int I = i0 + 16 * x + g + 4 * e, J = j0 + 16 * y + cl;
        if (I < p && J < q) out[(size_t)I * q + J] = acc[x][y][e];
      }
}

// the wide tile is used for single-matrix projections that fill it, unless
// the 64 x 64 tiles are asked for
static bool tn_use_wide(bool gram, int p, int q, int batch, int tile) {
  return !gram && batch == 1 && p >= kTile && q >= 2 * kTile && tile != kTileNarrow;
}

static bool tn_use_gram128(bool gram, int p, int q, int batch) {
  return gram && p == 128 && q == 128 && batch == 1;
}

int64_t tn_tiles(bool gram, int p, int q, bool same, int tile) {
  const int tp = (p + kTile - 1) / kTile, tq = (q + kTile - 1) / kTile;
  (void)same;
  if (tile != kTileNarrow && tn_use_gram128(gram, p, q, 1)) return 2;
  if (tn_use_wide(gram, p, q, 1, tile)) return (int64_t)tp * ((q + 2 * kTile - 1) / (2 * kTile));
  return gram ? (int64_t)tp * (tp + 1) / 2 : (int64_t)tp * tq;
}

hipError_t launch_tn(bool gram, int64_t m, int p, int q, const double *L, int64_t ldl,
                     const double *Rt, int64_t ldr, double *part, int64_t rc, int64_t nch,
                     const int *info, hipStream_t s, int batch, int64_t sL, int64_t sRt,
                     int64_t sPart, int tile) {
  const int tp = (p + kTile - 1) / kTile, tq = (q + kTile - 1) / kTile;
  const bool vec = (ldl % 2 == 0) && (ldr % 2 == 0) && ((uintptr_t)L % 16 == 0) &&
                   ((uintptr_t)Rt % 16 == 0) && (rc % 16 == 0) && (sL % 2 == 0) && (sRt % 2 == 0);
  if (tn_use_gram128(gram, p, q, batch)) {
    const dim3 gg((unsigned)(2 * nch));
    const bool same = L == Rt && ldl == ldr;
#define CQR_G128(V, S_) \
  hipLaunchKernelGGL((k_gram128<V, S_>), gg, dim3(64), 0, s, m, L, ldl, Rt, ldr, part, rc, info)
    if (same) {
      if (vec) CQR_G128(true, true); else CQR_G128(false, true);
    } else {
      if (vec) CQR_G128(true, false); else CQR_G128(false, false);
    }
#undef CQR_G128
    return hipGetLastError();
  }
  if (tn_use_wide(gram, p, q, batch, tile)) {
    const int tqw = (q + 2 * kTile - 1) / (2 * kTile);
    const dim3 gw((unsigned)((int64_t)tp * tqw * nch));
    if (vec)
      hipLaunchKernelGGL((k_tn_wide<true>), gw, dim3(64), 0, s, m, p, q, L, ldl, Rt, ldr, part, rc,
                         tp, tqw, info);
    else
      hipLaunchKernelGGL((k_tn_wide<false>), gw, dim3(64), 0, s, m, p, q, L, ldl, Rt, ldr, part, rc,
                         tp, tqw, info);
    return hipGetLastError();
  }
  const int64_t nb = tn_tiles(gram, p, q, false, kTileNarrow) * nch;
  dim3 grid((unsigned)nb, (unsigned)batch), block(64);
#define CQR_TN(U, V)                                                                             \
  hipLaunchKernelGGL((k_tn<U, V>), grid, block, 0, s, m, p, q, L, ldl, Rt, ldr, part, rc, tp, tq, \
                     sL, sRt, sPart, info)
  if (gram) {
    if (vec) CQR_TN(true, true); else CQR_TN(true, false);
  } else {
    if (vec) CQR_TN(false, true); else CQR_TN(false, false);
  }
#undef CQR_TN
  return hipGetLastError();
}

// ----------------------------------------------------------------------------
// k_nn: row-streaming product C = L Y (+ C), one wave per (16 RB) x 64 tile
// of C. The trailing update C -= Q Y is run as C + Q (-Y): the reduction that
// produces Y also stores its negation, so the hot loop feeds loaded values
// straight to the MFMAs. A workgroup holds 4 waves arranged WR x WC
// (WR * WC = 4) over rows x columns, so narrow products (the b-column
// Q_j = X U^{-1}) still keep all four waves busy. Lane/element maps
// (cl = lane % 16, g = lane / 16, y < RB row blocks, x < 4 column blocks):
//   B operand, block y: lane holds L[r0 + RB cl + y][k],  k = kk + g
//   A operand, block x: lane holds Y[k][c0 + 4 cl + x]
//   D element e of block (x, y): C[r0 + RB cl + y][c0 + 4 g + 16 e + x]
// so that every lane's L and C accesses are RB consecutive doubles and its Y
// accesses 4 consecutive doubles, and 16 lanes cover whole lines.
// RB = 2 (32-row tiles) halves the accumulators so that two waves fit on a
// SIMD: one wave's loads of C and its stores overlap the other's MFMAs.
// ----------------------------------------------------------------------------
template <bool SUB, bool TRI, bool VEC, int RB>
__global__ __launch_bounds__(256, (RB == 2) ? 2 : 1) void k_nn(
    int64_t m, int p, int q, const double *L, int64_t ldl, const double *L2, int64_t ldl2,
    int psplit, const double *__restrict__ Y, int64_t ldy, const double *Cin, int64_t ldci,
    double *C, int64_t ldc, int wr, int ncg, int64_t sL, int64_t sL2, int64_t sY, int64_t sCin,
    int64_t sC, double *C2, int64_t ldc2, const int *__restrict__ info,
    const int *__restrict__ skip) {
  constexpr int kRows = 16 * RB;  // rows of a wave's tile
  if (*info || (skip && *skip)) return;
  {  // batch: one matrix per grid row
    const int64_t bi = blockIdx.y;
    L += bi * sL;
    L2 += bi * sL2;
    Y += bi * sY;
    Cin += bi * sCin;
    C += bi * sC;
  }
  const int64_t lid = xcd_logical(blockIdx.x, gridDim.x);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, g = lane >> 4, cl = lane & 15;
  const int wc = 4 / wr;
  const int64_t r0 = (lid / ncg * wr + wave % wr) * (int64_t)kRows;
  const int c0 = ((int)(lid % ncg) * wc + wave / wr) * kTile;
  const bool active = c0 < q && r0 < m;
  const int64_t rl = r0 + RB * cl;  // first of this lane's RB rows
  const int yc = c0 + 4 * cl;       // first of this lane's 4 columns

  // RB consecutive doubles at p (16-byte aligned when VEC) into v[0..RB)
  auto ld_rows = [&](const double *pp, double *v) {
    if (VEC) {
#pragma unroll
      for (int h = 0; h < RB / 2; ++h) {
        const double2 t = reinterpret_cast<const double2 *>(pp)[h];
        v[2 * h] = t.x;
        v[2 * h + 1] = t.y;
      }
    } else {
#pragma unroll
      for (int u = 0; u < RB; ++u) v[u] = pp[u];
    }
  };

  d4 acc[4][RB];  // [column block x][row block y]
  if (active) {
#pragma unroll
    for (int x = 0; x < 4; ++x)
#pragma unroll
      for (int y = 0; y < RB; ++y) acc[x][y] = d4{0.0, 0.0, 0.0, 0.0};
    if (SUB) {
#pragma unroll
      for (int e = 0; e < 4; ++e)
#pragma unroll
        for (int x = 0; x < 4; ++x) {
          const int col = c0 + 4 * g + 16 * e + x;
          if (col < q) {
            const double *pc = Cin + (int64_t)col * ldci + rl;
            if (rl + RB <= m) {
              double v[RB];
              ld_rows(pc, v);
#pragma unroll
              for (int y = 0; y < RB; ++y) acc[x][y][e] = v[y];
            } else {
#pragma unroll
              for (int y = 0; y < RB; ++y) acc[x][y][e] = (rl + y < m) ? pc[y] : 0.0;
            }
          }
        }
    }

    // k range: all of p, or (upper-triangular Y) only k < c0 + 64
    const int kend = TRI ? ((c0 + kTile < p) ? c0 + kTile : p) : p;
    // Fast path: the wave's rows all exist and each lane's 4 columns are
    // either all < q or all >= q. A lane whose columns are all >= q reads
    // column 0 instead of being masked: its operand only reaches outputs that
    // are never stored. Everything else (the last, partial row tile; q not a
    // multiple of 4 at the right edge) takes the masked loop below.
    const bool fast = (r0 + kRows <= m) && ((q % 4) == 0 || c0 + kTile <= q);
    const double *lb = L + rl;
    const double *lb2 = L2 + rl;  // k >= psplit reads L2[:, k - psplit]
    const double *yb = Y + (yc < q ? yc : 0);
    auto load = [&](double (&da)[4][4], double (&db)[4][RB], int kk) {
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const int k = kk + 4 * s + g;
        const double *py = yb + (int64_t)k * ldy;
        const double *pl = (k < psplit) ? lb + (int64_t)k * ldl : lb2 + (int64_t)(k - psplit) * ldl2;
        if (VEC) {
          const double2 y0 = reinterpret_cast<const double2 *>(py)[0];
          const double2 y1 = reinterpret_cast<const double2 *>(py)[1];
          da[s][0] = y0.x;
          da[s][1] = y0.y;
          da[s][2] = y1.x;
          da[s][3] = y1.y;
        } else {
#pragma unroll
          for (int u = 0; u < 4; ++u) da[s][u] = py[u];
        }
        ld_rows(pl, db[s]);
      }
    };
    auto compute = [&](const double (&da)[4][4], const double (&db)[4][RB]) {
#pragma unroll
      for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int x = 0; x < 4; ++x)
#pragma unroll
          for (int y = 0; y < RB; ++y) acc[x][y] = mfma16x16x4(da[s][x], db[s][y], acc[x][y]);
    };
    // three-deep register ring, as in k_tn
    double a0[4][4], b0[4][RB], a1[4][4], b1[4][RB], a2[4][4], b2[4][RB];
    const int nit = fast ? kend / 16 : 0;  // full 16-wide k iterations
    if (nit > 0) {
      auto at = [&](int st) -> int { return 16 * (st < nit ? st : nit - 1); };
      load(a0, b0, 0);
      load(a1, b1, at(1));
      int it = 0;
      for (; it + 3 <= nit; it += 3) {
        load(a2, b2, at(it + 2));
        __builtin_amdgcn_sched_barrier(0);
        compute(a0, b0);
        __builtin_amdgcn_sched_barrier(0);
        load(a0, b0, at(it + 3));
        __builtin_amdgcn_sched_barrier(0);
        compute(a1, b1);
        __builtin_amdgcn_sched_barrier(0);
        load(a1, b1, at(it + 4));
        __builtin_amdgcn_sched_barrier(0);
        compute(a2, b2);
        __builtin_amdgcn_sched_barrier(0);
      }
      if (it < nit) compute(a0, b0);
      if (it + 1 < nit) compute(a1, b1);
    }
    // k tail (and the whole k range off the fast path): masked element loads
    for (int kk = 16 * nit; kk < kend; kk += 16) {
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const int k = kk + 4 * s + g;
        const bool kok = k < kend;
        const double *lk = (k < psplit) ? L + (int64_t)k * ldl : L2 + (int64_t)(k - psplit) * ldl2;
#pragma unroll
        for (int u = 0; u < 4; ++u) a0[s][u] = (kok && yc + u < q) ? Y[(int64_t)k * ldy + yc + u] : 0.0;
#pragma unroll
        for (int u = 0; u < RB; ++u) b0[s][u] = (kok && rl + u < m) ? lk[rl + u] : 0.0;
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
        double *pc2 = C2 ? C2 + (int64_t)col * ldc2 + rl : nullptr;
        if (VEC && rl + RB <= m) {
#pragma unroll
          for (int h = 0; h < RB / 2; ++h) {
            const double2 v = double2{acc[x][2 * h][e], acc[x][2 * h + 1][e]};
            reinterpret_cast<double2 *>(pc)[h] = v;
            if (pc2) reinterpret_cast<double2 *>(pc2)[h] = v;
          }
        } else {
#pragma unroll
          for (int y = 0; y < RB; ++y)
            if (rl + y < m) {
              pc[y] = acc[x][y][e];
              if (pc2) pc2[y] = acc[x][y][e];
            }
        }
      }
    }
}

// ----------------------------------------------------------------------------
// k_upd: the trailing update C = Cin + L Y for a short inner dimension
// (p <= kUpdMaxK, the panel width): Y is p x q and is re-read for every row
// tile by k_nn, which makes that kernel bound by L2 -> CU traffic. Here a
// workgroup owns one 64-column slab of C and a contiguous range of rows; it
// stages its slab of Y (zero-padded to a multiple of 16 rows) in LDS once and
// its four waves sweep 32-row tiles of the range, reading only L, Cin and C
// from global memory. Lane/element maps are those of k_nn with RB = 2.
// Consecutive logical workgroups share a row range (and so L's rows in one
// XCD's L2) and differ in the slab.
// ----------------------------------------------------------------------------
constexpr int kUpdMaxK = 128;
constexpr int kLdsPanelRows = 128;  // U^{-1} block k_trsm holds in LDS

// Position in a 64-column LDS slab row of column j (0..63): each lane of the
// update kernels reads its 4 consecutive columns 4 cl .. 4 cl + 3 as two
// 16-byte halves, so the row is stored as the first halves of all 16 lanes
// followed by the second halves. Each 16-byte read then covers consecutive
// addresses across the lanes (no bank conflicts); the plain order made every
// read a two-way conflict (lanes 32 bytes apart).
__host__ __device__ constexpr int slab_pos(int j) { return ((j >> 1) & 1) * 32 + (j >> 2) * 2 + (j & 1); }

bool nn_short_k(int p, const double *L, int64_t ldl, const double *Cin, int64_t ldci,
                const double *C, int64_t ldc) {
  return p <= kUpdMaxK && (ldl % 2 == 0) && (ldc % 2 == 0) && (ldci % 2 == 0) &&
         ((uintptr_t)L % 16 == 0) && ((uintptr_t)C % 16 == 0) && ((uintptr_t)Cin % 16 == 0);
}

__global__ __launch_bounds__(256, 2) void k_upd(int64_t m, int p, int q, const double *L,
                                                int64_t ldl, const double *__restrict__ Y,
                                                int64_t ldy, const double *Cin, int64_t ldci,
                                                double *C, int64_t ldc, int nslab,
                                                int64_t rows_per_wg, const int *__restrict__ info,
                                                const int *__restrict__ skip) {
  extern __shared__ double ys[];  // [pp][64], row-major
  if (*info || (skip && *skip)) return;
  const int64_t lid = xcd_logical(blockIdx.x, gridDim.x);
  const int c0 = (int)(lid % nslab) * kTile;
  const int64_t rb = (lid / nslab) * rows_per_wg;
  if (rb >= m) return;  // whole workgroup
  const int64_t re = (rb + rows_per_wg < m) ? rb + rows_per_wg : m;
  const int pp = (p + 15) / 16 * 16;
  for (int e = threadIdx.x; e < pp * kTile; e += 256) {
    const int k = e / kTile, c = c0 + e % kTile;
    ys[k * kTile + slab_pos(e % kTile)] = (k < p && c < q) ? Y[(int64_t)k * ldy + c] : 0.0;
  }
  __syncthreads();

  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, g = lane >> 4, cl = lane & 15;
  const double *yl = ys + 2 * cl;  // this lane's 4 columns of the slab (two halves)
  const int nit = p / 16;  // full 16-wide k steps; a ragged p adds one masked step

  for (int64_t r0 = rb + 32 * wave; r0 < re; r0 += 128) {
    const int64_t rl = r0 + 2 * cl;
    const bool full = r0 + 32 <= m;
    d4 acc[4][2];
#pragma unroll
    for (int e = 0; e < 4; ++e)
#pragma unroll
      for (int x = 0; x < 4; ++x) {
        const int col = c0 + 4 * g + 16 * e + x;
        double v0 = 0.0, v1 = 0.0;
        if (col < q) {
          const double *pc = Cin + (int64_t)col * ldci + rl;
          if (full) {
            const double2 t = *reinterpret_cast<const double2 *>(pc);
            v0 = t.x;
            v1 = t.y;
          } else {
            v0 = (rl < m) ? pc[0] : 0.0;
            v1 = (rl + 1 < m) ? pc[1] : 0.0;
          }
        }
        acc[x][0][e] = v0;
        acc[x][1][e] = v1;
      }
    auto load_y = [&](double (&da)[4][4], int kk) {
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const int k = kk + 4 * s + g;
        const double2 y0 = *reinterpret_cast<const double2 *>(yl + k * kTile);
        const double2 y1 = *reinterpret_cast<const double2 *>(yl + k * kTile + 32);
        da[s][0] = y0.x;
        da[s][1] = y0.y;
        da[s][2] = y1.x;
        da[s][3] = y1.y;
      }
    };
    auto compute = [&](const double (&da)[4][4], const double (&db)[4][2]) {
#pragma unroll
      for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int x = 0; x < 4; ++x)
#pragma unroll
          for (int y = 0; y < 2; ++y) acc[x][y] = mfma16x16x4(da[s][x], db[s][y], acc[x][y]);
    };
    // Y comes from LDS (short latency) right before its step; only L, from
    // global memory, goes through a three-deep register ring
    double a0[4][4], b0[4][2];
    const double *lb = L + (int64_t)g * ldl + rl;  // column g of this lane's rows
    if (full && nit > 0) {
      auto load = [&](double (&db)[4][2], int kk) {
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          const double2 t = *reinterpret_cast<const double2 *>(lb + (int64_t)(kk + 4 * s) * ldl);
          db[s][0] = t.x;
          db[s][1] = t.y;
        }
      };
      auto step = [&](const double (&db)[4][2], int kk) {
        load_y(a0, kk);
        compute(a0, db);
      };
      double b1[4][2], b2[4][2];
      auto at = [&](int st) -> int { return 16 * (st < nit ? st : nit - 1); };
      load(b0, 0);
      load(b1, at(1));
      int it = 0;
      for (; it + 3 <= nit; it += 3) {
        load(b2, at(it + 2));
        __builtin_amdgcn_sched_barrier(0);
        step(b0, 16 * it);
        __builtin_amdgcn_sched_barrier(0);
        load(b0, at(it + 3));
        __builtin_amdgcn_sched_barrier(0);
        step(b1, 16 * (it + 1));
        __builtin_amdgcn_sched_barrier(0);
        load(b1, at(it + 4));
        __builtin_amdgcn_sched_barrier(0);
        step(b2, 16 * (it + 2));
        __builtin_amdgcn_sched_barrier(0);
      }
      if (it < nit) step(b0, 16 * it);
      if (it + 1 < nit) step(b1, 16 * (it + 1));
    }
    // masked steps: every step of the last, partial row tile; the ragged k tail
    for (int kk = (full ? 16 * nit : 0); kk < pp; kk += 16) {
      load_y(a0, kk);
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const int k = kk + 4 * s + g;
        const double *pl = L + (int64_t)(k < p ? k : 0) * ldl + rl;
        b0[s][0] = (k < p && rl < m) ? pl[0] : 0.0;
        b0[s][1] = (k < p && rl + 1 < m) ? pl[1] : 0.0;
      }
      compute(a0, b0);
    }
#pragma unroll
    for (int e = 0; e < 4; ++e)
#pragma unroll
      for (int x = 0; x < 4; ++x) {
        const int col = c0 + 4 * g + 16 * e + x;
        if (col < q) {
          double *pc = C + (int64_t)col * ldc + rl;
          if (full) {
            *reinterpret_cast<double2 *>(pc) = double2{acc[x][0][e], acc[x][1][e]};
          } else {
            if (rl < m) pc[0] = acc[x][0][e];
            if (rl + 1 < m) pc[1] = acc[x][1][e];
          }
        }
      }
  }
}

// ----------------------------------------------------------------------------
// k_upd_lr: the same update C = Cin + L Y (inner dimension p <= kUpdMaxK,
// p % 16 == 0) with each wave's rows of L held in registers: k_upd re-reads
// L for every 64-column slab of C (q / 64 times; at 2^22 rows, 128 inner x
// 896 columns its HBM reads came to 1.38 x the compulsory bytes, at 4.6 TB/s
// of traffic), here L is read once. One persistent 4-wave workgroup per CU
// takes 128-row blocks (32 rows per wave; rows [0, mfull), mfull a multiple
// of 128) and sweeps every slab of C for them: slab s + 1 of Y is copied
// from global memory straight into the other half of a double-buffered LDS
// slab (global_load_lds) and its Cin into registers while slab s is
// multiplied, so only the first slab of a row block waits for memory. Lane
// maps, and the order of every sum (Cin first, then k ascending in groups of
// four), are those of k_upd, so the two kernels agree bit for bit.
// ----------------------------------------------------------------------------
constexpr int kLrRows = 128;  // rows per block (4 waves x 32)

__global__ __launch_bounds__(256, 1) void k_upd_lr(int64_t mfull, int p, int q, const double *L,
                                                   int64_t ldl, const double *__restrict__ Y,
                                                   int64_t ldy, const double *Cin, int64_t ldci,
                                                   double *C, int64_t ldc,
                                                   const int *__restrict__ info,
                                                   const int *__restrict__ skip) {
  // the two halves of the double-buffered Y slab ([p][64] each, row-major)
  // are separate arrays, so that the compiler can tell the copy into one from
  // the reads of the other and does not wait for the copy before reading
  __shared__ double ys0[kUpdMaxK * kTile];
  __shared__ double ys1[kUpdMaxK * kTile];
  if (*info || (skip && *skip)) return;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, g = lane >> 4, cl = lane & 15;
  const int nk = p / 16;
  const int nslab = (q + kTile - 1) / kTile;
  const int64_t nblk = mfull / kLrRows;

  // Y slab sl -> LDS: each instruction moves two 64-column rows (16 bytes
  // per lane); columns past q read column 0 (they reach only outputs that
  // are never stored)
  auto stage_y = [&](int sl, double *dst) {
    // lane position pp (16 bytes) of the slab row holds columns 4 (pp % 16)
    // + 2 (pp / 16) and the next one (the slab_pos layout)
    const int pp = lane & 31;
    const int c = sl * kTile + 4 * (pp & 15) + 2 * (pp >> 4);
    const double *src = Y + (c < q ? c : 0);
    for (int k0 = 2 * wave; k0 < p; k0 += 8) {
      const int k = k0 + (lane >> 5);
      __builtin_amdgcn_global_load_lds(
          (const void *)(src + (int64_t)k * ldy),
          (__attribute__((address_space(3))) void *)(dst + k0 * kTile), 16, 0, 0);
    }
  };
  // Cin of slab sl straight into an accumulator set (the sums start from it)
  auto load_cin = [&](int64_t rl, int sl, d4 (&acc)[4][2]) {
#pragma unroll
    for (int e = 0; e < 4; ++e)
#pragma unroll
      for (int x = 0; x < 4; ++x) {
        const int col = sl * kTile + 4 * g + 16 * e + x;
        const double2 t =
            *reinterpret_cast<const double2 *>(Cin + (int64_t)(col < q ? col : 0) * ldci + rl);
        acc[x][0][e] = t.x;
        acc[x][1][e] = t.y;
      }
  };
  double lv[kUpdMaxK / 16][4][2];  // L[rl + y][16 ks + 4 s + g]: this wave's rows of L
  auto store = [&](int64_t rl, int sl, const d4 (&acc)[4][2]) {
#pragma unroll
    for (int e = 0; e < 4; ++e)
#pragma unroll
      for (int x = 0; x < 4; ++x) {
        const int col = sl * kTile + 4 * g + 16 * e + x;
        if (col < q)
          *reinterpret_cast<double2 *>(C + (int64_t)col * ldc + rl) = double2{acc[x][0][e], acc[x][1][e]};
      }
  };

  // Slab sl of C: acc holds its Cin on entry and its result on exit; Y is
  // in `rd`. `other` holds the previous slab's result: it is stored first
  // (stores issued a whole slab before the barrier that closes this one,
  // which waits for every outstanding memory operation, have long
  // completed) and then receives the next slab's Cin, while the next slab's
  // Y is copied into `wr`. The last slab fetches itself again: unconditional
  // loads keep the compiler from moving registers, which would make it wait
  // for the loads right away.
  auto slab = [&](int64_t rl, int sl, const double *rd, double *wr, d4 (&acc)[4][2],
                  d4 (&other)[4][2]) {
    if (sl > 0) store(rl, sl - 1, other);
    const int nx = (sl + 1 < nslab) ? sl + 1 : sl;
    stage_y(nx, wr);
    load_cin(rl, nx, other);
    __builtin_amdgcn_sched_barrier(0);
    const double *yl = rd + 2 * cl;  // this lane's 4 columns (two halves)
#pragma unroll
    for (int ks = 0; ks < kUpdMaxK / 16; ++ks) {
      if (ks < nk) {
        // the k step's Y from LDS first, then its 32 MFMAs (only the first
        // read's latency is exposed)
        double ya[4][4];
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          const int k = 16 * ks + 4 * s + g;
          const double2 y0 = *reinterpret_cast<const double2 *>(yl + k * kTile);
          const double2 y1 = *reinterpret_cast<const double2 *>(yl + k * kTile + 32);
          ya[s][0] = y0.x;
          ya[s][1] = y0.y;
          ya[s][2] = y1.x;
          ya[s][3] = y1.y;
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
          for (int x = 0; x < 4; ++x)
#pragma unroll
            for (int y = 0; y < 2; ++y) acc[x][y] = mfma16x16x4(ya[s][x], lv[ks][s][y], acc[x][y]);
      }
    }
    if (sl == nslab - 1) store(rl, sl, acc);  // the row block's last slab
    __syncthreads();  // this slab's buffer is free; the next slab's copy has landed
  };

  d4 acc0[4][2], acc1[4][2];
  for (int64_t blk = blockIdx.x; blk < nblk; blk += gridDim.x) {
    const int64_t rl = blk * kLrRows + 32 * wave + 2 * cl;  // this lane's 2 rows
#pragma unroll
    for (int ks = 0; ks < kUpdMaxK / 16; ++ks)
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        if (ks < nk) {
          const double2 t =
              *reinterpret_cast<const double2 *>(L + (int64_t)(16 * ks + 4 * s + g) * ldl + rl);
          lv[ks][s][0] = t.x;
          lv[ks][s][1] = t.y;
        } else {
          lv[ks][s][0] = lv[ks][s][1] = 0.0;
        }
      }
    stage_y(0, ys0);
    load_cin(rl, 0, acc0);
    __syncthreads();  // the first slab's copy has landed (the compiler waits for it)
    for (int sl = 0; sl < nslab; sl += 2) {
      slab(rl, sl, ys0, ys1, acc0, acc1);
      if (sl + 1 < nslab) slab(rl, sl + 1, ys1, ys0, acc1, acc0);
    }
  }
}

// ----------------------------------------------------------------------------
// k_nn_wide: the update C = Cin + L Y (Y = -projection, row-major p x q) with
// one wave per 64-row x 16NX-column tile of C and the accumulators (4 x NX
// MFMA blocks: 128 doubles at NX = 8) held across the whole inner dimension.
// Each 16-wide k step loads 16 L values and 4 NX Y values per lane for 16 NX
// MFMAs (128 at NX = 8), against 8 + 16 values for 32 MFMAs in k_nn's 32 x 64
// tiles, so the operand traffic per MFMA is about a third; Y (the short,
// L2-resident side) is read from global memory directly. Lane/element maps
// (cl = lane % 16, g = lane / 16, y < 4 row blocks, x < NX column blocks):
//   B operand, block y: lane holds L[r0 + 4 cl + y][k],  k = kk + 4 s + g
//   A operand, block x: lane holds Y[k][c0 + NX cl + x]
//   D element e of block (x, y): C[r0 + 4 cl + y][c0 + NX (g + 4 e) + x]
// so a lane's L and C accesses are 4 consecutive doubles of one column and
// its Y accesses NX consecutive doubles of one row. Every element is summed
// in the order of k_nn and k_upd (Cin first, then k steps ascending with the
// same groups of four per MFMA), so the three kernels agree bit for bit.
// Fast path: the tile's rows all exist, p is a multiple of 16 and each
// lane's NX columns are all < q or all >= q (those lanes read column 0: their
// outputs are never stored); anything else takes the masked loop.
// SUB = false, TRI = true: the in-place product Q = X U^{-1} (Y = U^{-1}
// upper triangular, L = C = X, no Cin): a workgroup holds one wave per
// 128-column tile of one 64-row tile, every wave sums k < c0 + 128 only (the
// rest of U^{-1}'s column is zero) from zero, and a workgroup barrier
// separates the last read of the rows from the first write. k_trsm and
// k_nn<TRI> sum the same terms in the same order (their extra k steps only
// add exact zeros), so all three agree bit for bit. C2 (optional) receives
// the same values as C.
// ----------------------------------------------------------------------------
template <int NX, bool SUB, bool TRI, bool LFIRST = false>
__global__ __launch_bounds__(128) void k_nn_wide(int64_t m, int p, int q, const double *L,
                                                 int64_t ldl, const double *__restrict__ Y,
                                                 int64_t ldy, const double *Cin, int64_t ldci,
                                                 double *C, int64_t ldc, int nct, double *C2,
                                                 int64_t ldc2, const int *__restrict__ info,
                                                 const int *__restrict__ skip, const double *L2,
                                                 int64_t ldl2, int psplit, int64_t sL,
                                                 int64_t sL2, int64_t sY, int64_t sC) {
  if (*info || (skip && *skip)) return;
  {  // batch: matrix blockIdx.y (C2 and Cin only for single products)
    const int64_t bi = blockIdx.y;
    L += bi * sL;
    L2 += bi * sL2;
    Y += bi * sY;
    C += bi * sC;
  }
  constexpr int kCols = 16 * NX;
  const int nw = blockDim.x >> 6;  // waves (column tiles) per workgroup
  const int64_t lid = xcd_logical(blockIdx.x, gridDim.x);
  const int groups = nct / nw;  // workgroups per row tile
  const int64_t r0 = (lid / groups) * 64;
  const int c0 = ((int)(lid % groups) * nw + (int)(threadIdx.x >> 6)) * kCols;
  const int kend = TRI ? ((c0 + kCols < p) ? c0 + kCols : p) : p;
  const int lane = threadIdx.x & 63, g = lane >> 4, cl = lane & 15;
  const int64_t rl = r0 + 4 * cl;  // this lane's 4 rows
  const int yc = c0 + NX * cl;     // this lane's NX columns of Y
  // column of A-operand / D row i in column block x: NX-interleaved, or (LFIRST)
  // block x = the 16 contiguous columns c0 + 16 x .. c0 + 16 x + 15
  auto col_of = [&](int x, int i) -> int { return LFIRST ? c0 + 16 * x + i : c0 + NX * i + x; };

  // FAST: every row of the tile exists, p % 16 == 0 and each lane's NX
  // columns are all < q or all >= q. The two forms are separate code paths
  // so that the accumulators never merge across them.
  auto body = [&](auto fast_c) {
    constexpr bool FAST = decltype(fast_c)::value;
    d4 acc[NX][4];  // [column block x][row block y]
    // Cin into the accumulators, each one whole (its four columns, one row)
    // before the next is started, one column block per scheduling region:
    // building them element by element made the compiler hold all of them
    // in VGPRs at once and spill
#pragma unroll
    for (int x = 0; x < NX; ++x) {
      if (!SUB) {
#pragma unroll
        for (int y = 0; y < 4; ++y) acc[x][y] = d4{0.0, 0.0, 0.0, 0.0};
        continue;
      }
#pragma unroll
      for (int y = 0; y < 4; ++y) {
        d4 v;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int col = col_of(x, g + 4 * e);
          const double *pc = Cin + (int64_t)(col < q ? col : 0) * ldci + rl + y;
          v[e] = (FAST || (col < q && rl + y < m)) ? *pc : 0.0;
        }
        acc[x][y] = mfma16x16x4(0.0, 0.0, v);  // = v, placed as an accumulator
      }
      __builtin_amdgcn_sched_barrier(0);
    }
    // LFIRST: the first source's rows of Y (k < psplit) are lower triangular
    // (Y[k][c] = 0 for c > k), so block x gets nothing from a k step that
    // ends below column 16 x: those MFMAs would add exact zeros
    auto compute = [&](const double (&da)[4][NX], const double (&db)[4][4], int kk) {
#pragma unroll
      for (int x = 0; x < NX; ++x) {
        if (LFIRST && kk + 16 <= psplit && 16 * x > kk + 15) continue;
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
          for (int y = 0; y < 4; ++y) acc[x][y] = mfma16x16x4(da[s][x], db[s][y], acc[x][y]);
      }
    };
    if (FAST) {
      const double *yb = LFIRST ? Y + c0 + cl + (int64_t)g * ldy
                                : Y + (yc < q ? yc : 0) + (int64_t)g * ldy;
      const double *lb = L + (int64_t)g * ldl + rl;
      const double *lb2 = L2 + (int64_t)g * ldl2 + rl;  // k >= psplit: column k - psplit of L2
      auto load = [&](double (&da)[4][NX], double (&db)[4][4], int kk) {
        const bool first = kk < psplit;  // a whole k step lies in one source
        const double *lbase = first ? lb + (int64_t)kk * ldl : lb2 + (int64_t)(kk - psplit) * ldl2;
        const int64_t lld = first ? ldl : ldl2;
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          if constexpr (LFIRST) {
            const double *py = yb + (int64_t)(kk + 4 * s) * ldy;
#pragma unroll
            for (int x = 0; x < NX; ++x) da[s][x] = py[16 * x];
          } else {
            const double2 *py = reinterpret_cast<const double2 *>(yb + (int64_t)(kk + 4 * s) * ldy);
#pragma unroll
            for (int h = 0; h < NX / 2; ++h) {
              const double2 t = py[h];
              da[s][2 * h] = t.x;
              da[s][2 * h + 1] = t.y;
            }
          }
          const double2 *pl = reinterpret_cast<const double2 *>(lbase + (int64_t)(4 * s) * lld);
          const double2 l0 = pl[0], l1 = pl[1];
          db[s][0] = l0.x;
          db[s][1] = l0.y;
          db[s][2] = l1.x;
          db[s][3] = l1.y;
        }
      };
      // two register stages: while one step's MFMAs run, the next step's
      // loads are in flight (16 NX MFMAs of cover)
      const int nit = kend / 16;
      double a0[4][NX], b0[4][4], a1[4][NX], b1[4][4];
      auto at = [&](int st) -> int { return 16 * (st < nit ? st : nit - 1); };
      if (nit > 0) {
        load(a0, b0, 0);
        int it = 0;
        for (; it + 2 <= nit; it += 2) {
          load(a1, b1, at(it + 1));
          __builtin_amdgcn_sched_barrier(0);
          compute(a0, b0, 16 * it);
          __builtin_amdgcn_sched_barrier(0);
          load(a0, b0, at(it + 2));
          __builtin_amdgcn_sched_barrier(0);
          compute(a1, b1, 16 * (it + 1));
          __builtin_amdgcn_sched_barrier(0);
        }
        if (it < nit) compute(a0, b0, 16 * it);
      }
    } else {
      for (int kk = 0; kk < kend; kk += 16) {
        double da[4][NX], db[4][4];
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          const int k = kk + 4 * s + g;
          const bool kok = k < kend;
          const int kc = kok ? k : 0;
          const double *py = Y + (int64_t)kc * ldy;
          const double *pl = (kc < psplit) ? L + (int64_t)kc * ldl : L2 + (int64_t)(kc - psplit) * ldl2;
#pragma unroll
          for (int x = 0; x < NX; ++x) {
            const int col = col_of(x, cl);
            da[s][x] = (kok && col < q) ? py[col] : 0.0;
          }
#pragma unroll
          for (int y = 0; y < 4; ++y) db[s][y] = (kok && rl + y < m) ? pl[rl + y] : 0.0;
        }
        compute(da, db, kk);
      }
    }
    if (!SUB) __syncthreads();  // in place: every read of the rows precedes every write
#pragma unroll
    for (int e = 0; e < 4; ++e)
#pragma unroll
      for (int x = 0; x < NX; ++x) {
        const int col = col_of(x, g + 4 * e);
        if (col < q) {
          double *pc = C + (int64_t)col * ldc + rl;
          double *pc2 = C2 ? C2 + (int64_t)col * ldc2 + rl : nullptr;
          if (FAST) {
            const double2 v0 = double2{acc[x][0][e], acc[x][1][e]};
            const double2 v1 = double2{acc[x][2][e], acc[x][3][e]};
            reinterpret_cast<double2 *>(pc)[0] = v0;
            reinterpret_cast<double2 *>(pc)[1] = v1;
            if (pc2) {
              reinterpret_cast<double2 *>(pc2)[0] = v0;
              reinterpret_cast<double2 *>(pc2)[1] = v1;
            }
          } else {
#pragma unroll
            for (int y = 0; y < 4; ++y)
              if (rl + y < m) {
                pc[y] = acc[x][y][e];
                if (pc2) pc2[y] = acc[x][y][e];
              }
          }
        }
      }
  };
  if ((r0 + 64 <= m) && (kend % 16 == 0) && (psplit % 16 == 0) &&
      (((q % NX) == 0 && !LFIRST) || c0 + kCols <= q))
    body(std::true_type{});
  else
    body(std::false_type{});
}

// ----------------------------------------------------------------------------
// k_trsm: Q_j = X U^{-1} in place for a panel of W = 64 or 128 columns, over
// the rows [0, mfull) in blocks of 128 rows. One persistent 8-wave
// workgroup per CU keeps U^{-1} (upper triangle, zero elsewhere) in LDS and
// takes every gridDim.x-th block; each wave owns a 16-row x W tile of the
// block, so it reads and writes only its own rows (no workgroup barrier) and
// every wave does the same work. MFMA block x covers the 16 contiguous
// columns 16x..16x+15, which need k < 16(x+1) only: k step ks feeds blocks
// x >= ks, 36 of the 64 block-steps at W = 128. Lane maps (cl = lane % 16,
// g = lane / 16):
//   A operand (U^{-1}), block x, step s: lane holds U^{-1}[k][16x + cl],
//     k = 16 ks + 4 s + g
//   B operand (X): lane holds X[r + cl][k]
//   D element e of block x: Q[r + cl][16x + g + 4e]
// The k steps of consecutive blocks form one stream through a four-deep
// register ring (prefetch three steps ahead). The product reads Xs (ld
// ldxs) and writes X: Xs = X is the in-place form, any other Xs must not
// overlap X. X2 (optional) receives the same values as X.
// ----------------------------------------------------------------------------
constexpr int kTrsmRows = 128;

template <int W>
__global__ __launch_bounds__(512, 1) void k_trsm(int64_t mfull, const double *Xs, int64_t ldxs,
                                                 double *X, int64_t ldx,
                                                 const double *__restrict__ Uinv, int64_t ldu,
                                                 double *X2, int64_t ldx2,
                                                 const int *__restrict__ info,
                                                 const int *__restrict__ skip) {
  extern __shared__ double us[];  // [W][W] row-major
  if (*info || (skip && *skip)) return;
  for (int e = threadIdx.x; e < W * W; e += 512) {
    const int k = e / W, c = e % W;
    us[e] = (c >= k) ? Uinv[(int64_t)k * ldu + c] : 0.0;
  }
  __syncthreads();
  constexpr int NX = W / 16, NK = W / 16;
  static_assert(NK % 4 == 0, "the ring depth divides the k steps of a block");
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, g = lane >> 4, cl = lane & 15;
  const int64_t nblk = mfull / kTrsmRows;
  if ((int64_t)blockIdx.x >= nblk) return;  // whole workgroup
  const int64_t nmine = (nblk - blockIdx.x + gridDim.x - 1) / gridDim.x;
  const int64_t T = nmine * NK;
  const int64_t rstep = (int64_t)gridDim.x * kTrsmRows;  // rows between this workgroup's blocks
  int64_t rl = (int64_t)blockIdx.x * kTrsmRows + 16 * wave + cl;

  // load cursor: step index -> pointer to Xs[row rl][column 16 ks + g]
  int64_t lt = 0;
  const double *lp = Xs + rl + (int64_t)g * ldxs;
  auto load = [&](double (&db)[4]) {
#pragma unroll
    for (int s = 0; s < 4; ++s) db[s] = lp[(int64_t)(4 * s) * ldxs];
    if (lt + 1 < T) {  // advance; past the end the last step is re-read
      ++lt;
      lp += ((lt % NK) == 0) ? rstep - (int64_t)(NK - 1) * 16 * ldxs : 16 * ldxs;
    }
  };
  double ring[4][4];
  load(ring[0]);
  load(ring[1]);
  load(ring[2]);
  const double *ucol = us + cl;
  for (int64_t blk = 0; blk < nmine; ++blk) {
    d4 acc[NX];
#pragma unroll
    for (int x = 0; x < NX; ++x) acc[x] = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int ks = 0; ks < NK; ++ks) {
      load(ring[(ks + 3) & 3]);
      __builtin_amdgcn_sched_barrier(0);
      const double (&db)[4] = ring[ks & 3];
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const double *urow = ucol + (16 * ks + 4 * s + g) * W;
#pragma unroll
        for (int x = ks; x < NX; ++x) acc[x] = mfma16x16x4(urow[16 * x], db[s], acc[x]);
      }
      __builtin_amdgcn_sched_barrier(0);
    }
#pragma unroll
    for (int x = 0; x < NX; ++x)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int64_t off = (int64_t)(16 * x + g + 4 * e) * ldx + rl;
        X[off] = acc[x][e];
        if (X2) X2[(int64_t)(16 * x + g + 4 * e) * ldx2 + rl] = acc[x][e];
      }
    rl += rstep;
  }
}

// ----------------------------------------------------------------------------
// k_nn_ys: C = [L(:, 0:psplit) | L2] Y without an input C (the adjoint's
// second pass, dA = [dQ | Q] [R^{-T}; G]), with Y staged per 64-column slab
// in LDS as in k_upd: eight waves per workgroup (two per SIMD; one workgroup
// per CU holds a slab of up to 256 x 64 doubles) sweep 32-row tiles of an
// equal share of the rows. p and psplit are multiples of 16, so each 16-wide
// k step reads one source. Batch: matrix blockIdx.y at the given strides.
// ----------------------------------------------------------------------------
constexpr int kYsMaxK = 256;

__global__ __launch_bounds__(512, 1) void k_nn_ys(int64_t m, int p, int q, const double *L,
                                                  int64_t ldl, const double *L2, int64_t ldl2,
                                                  int psplit, const double *__restrict__ Y,
                                                  int64_t ldy, double *C, int64_t ldc, int nslab,
                                                  int64_t rows_per_wg, int64_t sL, int64_t sL2,
                                                  int64_t sY, int64_t sC,
                                                  const int *__restrict__ info) {
  extern __shared__ double ys[];  // [p][64], row-major
  if (*info) return;
  {
    const int64_t bi = blockIdx.y;
    L += bi * sL;
    L2 += bi * sL2;
    Y += bi * sY;
    C += bi * sC;
  }
  const int64_t lid = xcd_logical(blockIdx.x, gridDim.x);
  const int c0 = (int)(lid % nslab) * kTile;
  const int64_t rb = (lid / nslab) * rows_per_wg;
  if (rb >= m) return;  // whole workgroup
  const int64_t re = (rb + rows_per_wg < m) ? rb + rows_per_wg : m;
  for (int e = threadIdx.x; e < p * kTile; e += 512) {
    const int k = e / kTile, c = c0 + e % kTile;
    ys[k * kTile + slab_pos(e % kTile)] = (c < q) ? Y[(int64_t)k * ldy + c] : 0.0;
  }
  __syncthreads();
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, g = lane >> 4, cl = lane & 15;
  const double *yl = ys + 2 * cl;  // this lane's 4 columns (two halves, slab_pos layout)
  const int nit = p / 16;
  for (int64_t r0 = rb + 32 * wave; r0 < re; r0 += 256) {
    const int64_t rl = r0 + 2 * cl;
    const bool full = r0 + 32 <= m;
    d4 acc[4][2];
#pragma unroll
    for (int x = 0; x < 4; ++x)
#pragma unroll
      for (int y = 0; y < 2; ++y) acc[x][y] = d4{0.0, 0.0, 0.0, 0.0};
    auto lptr = [&](int kk) -> const double * {  // column kk + g of [L | L2], row rl
      return (kk < psplit) ? L + (int64_t)(kk + g) * ldl + rl
                           : L2 + (int64_t)(kk - psplit + g) * ldl2 + rl;
    };
    auto load = [&](double (&db)[4][2], int kk) {
      const double *pl = lptr(kk);
      const int64_t ld = (kk < psplit) ? ldl : ldl2;
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        if (full) {
          const double2 t = *reinterpret_cast<const double2 *>(pl + (int64_t)(4 * s) * ld);
          db[s][0] = t.x;
          db[s][1] = t.y;
        } else {
          db[s][0] = (rl < m) ? pl[(int64_t)(4 * s) * ld] : 0.0;
          db[s][1] = (rl + 1 < m) ? pl[(int64_t)(4 * s) * ld + 1] : 0.0;
        }
      }
    };
    double ya[4][4];
    auto step = [&](const double (&db)[4][2], int kk) {
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const int k = kk + 4 * s + g;
        const double2 y0 = *reinterpret_cast<const double2 *>(yl + k * kTile);
        const double2 y1 = *reinterpret_cast<const double2 *>(yl + k * kTile + 32);
        ya[s][0] = y0.x;
        ya[s][1] = y0.y;
        ya[s][2] = y1.x;
        ya[s][3] = y1.y;
      }
#pragma unroll
      for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int x = 0; x < 4; ++x)
#pragma unroll
          for (int y = 0; y < 2; ++y) acc[x][y] = mfma16x16x4(ya[s][x], db[s][y], acc[x][y]);
    };
    double b0[4][2], b1[4][2], b2[4][2];
    auto at = [&](int st) -> int { return 16 * (st < nit ? st : nit - 1); };
    load(b0, 0);
    load(b1, at(1));
    int it = 0;
    for (; it + 3 <= nit; it += 3) {
      load(b2, at(it + 2));
      __builtin_amdgcn_sched_barrier(0);
      step(b0, 16 * it);
      __builtin_amdgcn_sched_barrier(0);
      load(b0, at(it + 3));
      __builtin_amdgcn_sched_barrier(0);
      step(b1, 16 * (it + 1));
      __builtin_amdgcn_sched_barrier(0);
      load(b1, at(it + 4));
      __builtin_amdgcn_sched_barrier(0);
      step(b2, 16 * (it + 2));
      __builtin_amdgcn_sched_barrier(0);
    }
    if (it < nit) step(b0, 16 * it);
    if (it + 1 < nit) step(b1, 16 * (it + 1));
#pragma unroll
    for (int e = 0; e < 4; ++e)
#pragma unroll
      for (int x = 0; x < 4; ++x) {
        const int col = c0 + 4 * g + 16 * e + x;
        if (col < q) {
          double *pc = C + (int64_t)col * ldc + rl;
          if (full) {
            *reinterpret_cast<double2 *>(pc) = double2{acc[x][0][e], acc[x][1][e]};
          } else {
            if (rl < m) pc[0] = acc[x][0][e];
            if (rl + 1 < m) pc[1] = acc[x][1][e];
          }
        }
      }
  }
}

// rows of C per workgroup row-slab is 16 * RB * WR
constexpr int kNnRB = 2;

// CU count of the device current at the first call (one-time set-up through
// function-local statics, which C++ initialises once and thread-safely).
static int device_cus() {
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 256;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return 256;
  return cus > 0 ? cus : 256;
}

// The single-matrix update's kernel: the requested variant where it applies,
// else the default: the LDS-slab kernel for inner dimensions up to kUpdMaxK
// (measured at 2^22 rows, 128 inner x 896 columns: 9.5 ms against 11.6 ms
// for the wide tiles, whose C traffic per MFMA is the same but whose whole
// tile of Cin loads is exposed at the start of each short tile), the 64 x 128
// register tiles for longer ones (896 inner x 128 columns: 9.7 ms against
// 10.8 ms for the 32 x 64 tiles), the 32 x 64 tiles where neither applies.
int update_variant(int tile, bool res_ok, bool slab_ok, bool wide_ok) {
  if (!wide_ok && !slab_ok) return kTileNarrow;
  if (tile == kTileWide && wide_ok) return kTileWide;
  if (tile == kTileNarrow) return kTileNarrow;
  if (tile == kTileSlab && slab_ok) return kTileSlab;
  if (tile == kTileResident && res_ok) return kTileResident;
  return slab_ok ? kTileSlab : (wide_ok ? kTileWide : kTileNarrow);
}

hipError_t launch_nn(bool subtract, bool upper_y, int64_t m, int p, int q, const double *L,
                     int64_t ldl, const double *Y, int64_t ldy, const double *Cin, int64_t ldci,
                     double *C, int64_t ldc, const int *info, hipStream_t s, const double *L2,
                     int64_t ldl2, int psplit, int batch, int64_t sL, int64_t sL2, int64_t sY,
                     int64_t sCin, int64_t sC, double *C2, int64_t ldc2, const int *skip,
                     int tile, bool lower_first) {
  if (C2 && (subtract || batch != 1)) return hipErrorInvalidValue;
  if (!L2) {
    L2 = L;
    ldl2 = ldl;
    sL2 = sL;
    psplit = p;
  }
  if (!Cin) {
    Cin = C;
    ldci = ldc;
    sCin = sC;
  }
  const int slabs = (q + kTile - 1) / kTile;
  // a product without input C (Q = X U^{-1}, possibly in place) keeps all of
  // a row tile's columns in one workgroup: three slabs take all four
  // column waves (one idle) rather than two column groups
  const int wc = (slabs >= 4 || (!subtract && slabs == 3)) ? 4 : (slabs >= 2 ? 2 : 1);
  const int wr = 4 / wc;
  const int ncg = (slabs + wc - 1) / wc;
  if (!subtract && !upper_y && C2 == nullptr && p % 16 == 0 && psplit % 16 == 0 && q > 64 &&
      tile != kTileSlab && (ldl % 2 == 0) && (ldl2 % 2 == 0) && (ldc % 2 == 0) && (ldy % 2 == 0) &&
      ((uintptr_t)L % 16 == 0) && ((uintptr_t)L2 % 16 == 0) && ((uintptr_t)C % 16 == 0) &&
      ((uintptr_t)Y % 16 == 0) && (sL % 2 == 0) && (sL2 % 2 == 0) && (sY % 2 == 0) &&
      (sC % 2 == 0) && batch <= 65535) {
    // no input C, [L | L2] Y (the adjoint's second pass): one wave per
    // 64 x 128 tile, the accumulators held over the whole inner dimension
    const int nct = (q + 127) / 128;
    const int64_t rts = (m + 63) / 64;
    if (lower_first)
      hipLaunchKernelGGL((k_nn_wide<8, false, false, true>),
                         dim3((unsigned)(rts * nct), (unsigned)batch), dim3(64), 0, s, m, p, q, L,
                         ldl, Y, ldy, nullptr, 0, C, ldc, nct, nullptr, 0, info, skip, L2, ldl2,
                         psplit, sL, sL2, sY, sC);
    else
      hipLaunchKernelGGL((k_nn_wide<8, false, false>), dim3((unsigned)(rts * nct), (unsigned)batch),
                         dim3(64), 0, s, m, p, q, L, ldl, Y, ldy, nullptr, 0, C, ldc, nct, nullptr,
                         0, info, skip, L2, ldl2, psplit, sL, sL2, sY, sC);
    return hipGetLastError();
  }
  if (!subtract && !upper_y && C2 == nullptr && p <= kYsMaxK && p % 16 == 0 && psplit % 16 == 0 &&
      (ldl % 2 == 0) && (ldl2 % 2 == 0) && (ldc % 2 == 0) && ((uintptr_t)L % 16 == 0) &&
      ((uintptr_t)L2 % 16 == 0) && ((uintptr_t)C % 16 == 0) && (sL % 2 == 0) &&
      (sL2 % 2 == 0) && (sC % 2 == 0)) {
    // no input C, inner dimension <= 256: Y staged in LDS, one 8-wave
    // workgroup per CU, rows shared equally among a slab's workgroups
    static const hipError_t attr = hipFuncSetAttribute(
        (const void *)k_nn_ys, hipFuncAttributeMaxDynamicSharedMemorySize,
        kYsMaxK * kTile * (int)sizeof(double));
    if (attr != hipSuccess) return attr;
    static const int cus = device_cus();
    const int64_t per = std::max<int64_t>(1, (int64_t)std::max(cus, 1) / ((int64_t)slabs * batch));
    int64_t rpw = (m + per - 1) / per;
    rpw = (rpw + 31) / 32 * 32;
    const int64_t chunks = (m + rpw - 1) / rpw;
    hipLaunchKernelGGL(k_nn_ys, dim3((unsigned)(chunks * slabs), (unsigned)batch), dim3(512),
                       (size_t)p * kTile * sizeof(double), s, m, p, q, L, ldl, L2, ldl2, psplit, Y,
                       ldy, C, ldc, slabs, rpw, sL, sL2, sY, sC, info);
    return hipGetLastError();
  }
  const bool tri_wide_ok = !subtract && upper_y && batch == 1 && p == q && L2 == L &&
                           (ldl % 2 == 0) && (ldc % 2 == 0) && (ldy % 2 == 0) &&
                           ((uintptr_t)L % 16 == 0) && ((uintptr_t)C % 16 == 0) &&
                           ((uintptr_t)Y % 16 == 0) &&
                           (C2 == nullptr || ((ldc2 % 2 == 0) && ((uintptr_t)C2 % 16 == 0)));
  // Q = X U^{-1} for 256 columns: the right half [X_l X_r] [B; C] first (in
  // place: it reads the left half, which is still X), then the left half
  // X_l A by the persistent kernel with A's 128 x 128 block in LDS. Same
  // bits as one triangular product (the right half's extra k terms are the
  // zero entries below U^{-1}'s diagonal).
  if (tri_wide_ok && q == 2 * kLdsPanelRows && (L == C || ldl >= m) && Cin == C && m >= 128) {
    const int h = kLdsPanelRows;
    const int64_t rts = (m + 63) / 64;
    hipLaunchKernelGGL((k_nn_wide<8, false, false>), dim3((unsigned)rts), dim3(64), 0, s, m, p, h,
                       L, ldl, Y + h, ldy, nullptr, 0, C + (int64_t)h * ldc, ldc, 1,
                       C2 ? C2 + (int64_t)h * ldc2 : nullptr, ldc2, info, skip, L, ldl, p, 0, 0, 0,
                       0);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_nn(false, true, m, h, h, L, ldl, Y, ldy, nullptr, 0, C, ldc, info, s, nullptr, 0,
                     0, 1, 0, 0, 0, 0, 0, C2, ldc2, skip);
  }
  // Q = X U^{-1} for another panel width k_trsm does not take (ragged, or
  // between 128 and 256): one wave per 64 x 128 (64 x 64 up to 64 columns)
  // tile, the tiles of one row tile in one workgroup (reads before writes)
  if (tri_wide_ok && q <= 2 * kUpdMaxK && !(q == 64 || q == 128)) {
    const int nx = (q > 64) ? 8 : 4;
    const int nct = (q + 16 * nx - 1) / (16 * nx);  // 1 or 2 waves per workgroup
    const int64_t rts = (m + 63) / 64;
    if (nx == 8)
      hipLaunchKernelGGL((k_nn_wide<8, false, true>), dim3((unsigned)rts), dim3(64 * nct), 0, s, m,
                         p, q, L, ldl, Y, ldy, nullptr, 0, C, ldc, nct, C2, ldc2, info, skip, L, ldl,
                         p, 0, 0, 0, 0);
    else
      hipLaunchKernelGGL((k_nn_wide<4, false, true>), dim3((unsigned)rts), dim3(64 * nct), 0, s, m,
                         p, q, L, ldl, Y, ldy, nullptr, 0, C, ldc, nct, C2, ldc2, info, skip, L, ldl,
                         p, 0, 0, 0, 0);
    return hipGetLastError();
  }
  if (!subtract && ncg != 1) return hipErrorInvalidValue;  // in-place needs one column group
  if (!subtract && upper_y && batch == 1 && p == q && (q == 64 || q == 128) &&
      m >= kTrsmRows && Cin == C && (L == C || ldl >= m) && ldy >= q && L2 == L) {
    // Q = X U^{-1} (in place or from a separate X): persistent
    // U^{-1}-in-LDS kernel over the full row blocks, k_nn for the remaining
    // rows
    const int64_t mfull = m / kTrsmRows * kTrsmRows;  // > 0; the k_nn call below has m < 256
    {
      static const hipError_t attr = [] {
        const hipError_t e = hipFuncSetAttribute((const void *)k_trsm<128>,
                                                 hipFuncAttributeMaxDynamicSharedMemorySize,
                                                 kLdsPanel * kLdsPanel * (int)sizeof(double));
        if (e != hipSuccess) return e;
        return hipFuncSetAttribute((const void *)k_trsm<64>,
                                   hipFuncAttributeMaxDynamicSharedMemorySize,
                                   64 * 64 * (int)sizeof(double));
      }();
      if (attr != hipSuccess) return attr;
      static const int cus = device_cus();
      const int64_t nblk = mfull / kTrsmRows;
      const int64_t grid = std::min<int64_t>(nblk, std::max(cus, 1));
      if (q == 128)
        hipLaunchKernelGGL(k_trsm<128>, dim3((unsigned)grid), dim3(512),
                           (size_t)q * q * sizeof(double), s, mfull, L, ldl, C, ldc, Y, ldy, C2,
                           ldc2, info, skip);
      else
        hipLaunchKernelGGL(k_trsm<64>, dim3((unsigned)grid), dim3(512),
                           (size_t)q * q * sizeof(double), s, mfull, L, ldl, C, ldc, Y, ldy, C2,
                           ldc2, info, skip);
      const hipError_t e = hipGetLastError();
      if (e != hipSuccess || mfull == m) return e;
    }
    return launch_nn(false, true, m - mfull, p, q, L + mfull, ldl, Y, ldy, nullptr, 0, C + mfull,
                     ldc, info, s, nullptr, 0, 0, 1, 0, 0, 0, 0, 0, C2 ? C2 + mfull : nullptr, ldc2,
                     skip);
  }
  // single-matrix update: the kernel variant is a tuning choice (tile)
  const bool one_update = subtract && batch == 1 && psplit == p && C2 == nullptr;
  const bool wide_ok = one_update && (ldl % 2 == 0) && (ldci % 2 == 0) && (ldc % 2 == 0) &&
                       (ldy % 2 == 0) && ((uintptr_t)L % 16 == 0) && ((uintptr_t)Cin % 16 == 0) &&
                       ((uintptr_t)C % 16 == 0) && ((uintptr_t)Y % 16 == 0);
  const bool slab_ok = one_update && nn_short_k(p, L, ldl, Cin, ldci, C, ldc);
  const bool res_ok = slab_ok && p % 16 == 0 && m >= kLrRows && (ldy % 2 == 0) &&
                      ((uintptr_t)Y % 16 == 0);
  const int upd = update_variant(tile, res_ok, slab_ok, wide_ok);
  if (upd == kTileWide) {
    const int nx = (q > 64) ? 8 : 4;
    const int nct = (q + 16 * nx - 1) / (16 * nx);
    const int64_t rts = (m + 63) / 64;
    const dim3 gw((unsigned)(rts * nct));
    if (nx == 8)
      hipLaunchKernelGGL((k_nn_wide<8, true, false>), gw, dim3(64), 0, s, m, p, q, L, ldl, Y, ldy,
                         Cin, ldci, C, ldc, nct, nullptr, 0, info, skip, L, ldl, p, 0, 0, 0, 0);
    else
      hipLaunchKernelGGL((k_nn_wide<4, true, false>), gw, dim3(64), 0, s, m, p, q, L, ldl, Y, ldy,
                         Cin, ldci, C, ldc, nct, nullptr, 0, info, skip, L, ldl, p, 0, 0, 0, 0);
    return hipGetLastError();
  }
  if (upd == kTileResident) {
    // rows in whole 128-row blocks: one persistent workgroup per CU (its LDS
    // holds the two Y slabs); the remaining rows by the slab kernel below
    static const int cus = device_cus();
    const int64_t mfull = m / kLrRows * kLrRows;
    const int64_t grid = std::min<int64_t>(mfull / kLrRows, std::max(cus, 1));
    hipLaunchKernelGGL(k_upd_lr, dim3((unsigned)grid), dim3(256), 0, s, mfull, p, q, L, ldl, Y, ldy,
                       Cin, ldci, C, ldc, info, skip);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess || mfull == m) return e;
    return launch_nn(true, false, m - mfull, p, q, L + mfull, ldl, Y, ldy, Cin + mfull, ldci,
                     C + mfull, ldc, info, s, nullptr, 0, 0, 1, 0, 0, 0, 0, 0, nullptr, 0, skip,
                     kTileSlab);
  }
  if (upd == kTileSlab) {
    // one round of resident workgroups (two per CU): each slab gets an equal
    // share of them, each with an equal range of rows (a multiple of 32)
    static const hipError_t attr = hipFuncSetAttribute(
        (const void *)k_upd, hipFuncAttributeMaxDynamicSharedMemorySize,
        kUpdMaxK * kTile * (int)sizeof(double));
    if (attr != hipSuccess) return attr;
    static const int cus = device_cus();
    const int64_t per_slab = std::max<int64_t>(1, 2 * (int64_t)std::max(cus, 1) / slabs);
    int64_t rpw = (m + per_slab - 1) / per_slab;
    rpw = (rpw + 31) / 32 * 32;
    const int64_t chunks = (m + rpw - 1) / rpw;
    const size_t lds = (size_t)((p + 15) / 16 * 16) * kTile * sizeof(double);
    hipLaunchKernelGGL(k_upd, dim3((unsigned)(chunks * slabs)), dim3(256), lds, s, m, p, q, L, ldl,
                       Y, ldy, Cin, ldci, C, ldc, slabs, rpw, info, skip);
    return hipGetLastError();
  }
  const int64_t rows = 16 * kNnRB * (int64_t)wr;
  const int64_t rts = (m + rows - 1) / rows;
  const bool vec = (ldl % 2 == 0) && (ldl2 % 2 == 0) && (ldc % 2 == 0) && (ldci % 2 == 0) &&
                   (ldy % 2 == 0) && ((uintptr_t)L % 16 == 0) && ((uintptr_t)L2 % 16 == 0) &&
                   ((uintptr_t)C % 16 == 0) && ((uintptr_t)Cin % 16 == 0) &&
                   ((uintptr_t)Y % 16 == 0) && (sL % 2 == 0) && (sL2 % 2 == 0) && (sY % 2 == 0) &&
                   (sCin % 2 == 0) && (sC % 2 == 0) && (ldc2 % 2 == 0) && ((uintptr_t)C2 % 16 == 0);
  dim3 grid((unsigned)(rts * ncg), (unsigned)batch), block(256);
#define CQR_NN(S, T, V)                                                                             \
  hipLaunchKernelGGL((k_nn<S, T, V, kNnRB>), grid, block, 0, s, m, p, q, L, ldl, L2, ldl2, psplit, \
                     Y, ldy, Cin, ldci, C, ldc, wr, ncg, sL, sL2, sY, sCin, sC, C2, ldc2, info, \
                     skip)
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
// Split-m reduction: fixed-order sum of the per-chunk partials (replaces the
// Allreduce of Algorithms 2 and 8). Element e of the chunk partials is summed
// by one thread: groups of 8 consecutive chunks are loaded together (8
// independent loads in flight) and added in a fixed pairwise tree; the group
// sums go through a binary-counter pairwise accumulator held in registers.
// Large chunk counts are cut into slices of kSlice chunks summed by separate
// blocks, whose results are summed the same way by a second pass. The order
// depends only on (chunk count, element), never on which wave finished first.
// ----------------------------------------------------------------------------
constexpr int kSlice = 64;

__device__ __forceinline__ double pairwise_sum(const double *__restrict__ x, int64_t count,
                                               int64_t stride) {
  double lvl[24];
  unsigned occ = 0;
  for (int64_t c0 = 0; c0 < count; c0 += 8) {
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = (c0 + u < count) ? x[(c0 + u) * stride] : 0.0;
    double g = ((v[0] + v[1]) + (v[2] + v[3])) + ((v[4] + v[5]) + (v[6] + v[7]));
    bool placed = false;
#pragma unroll
    for (int l = 0; l < 24; ++l) {
      if (!placed) {
        if (occ & (1u << l)) {
          g = lvl[l] + g;
          occ &= ~(1u << l);
        } else {
          lvl[l] = g;
          occ |= 1u << l;
          placed = true;
        }
      }
    }
  }
  double sum = 0.0;
  bool first = true;
#pragma unroll
  for (int l = 0; l < 24; ++l)
    if (occ & (1u << l)) {
      sum = first ? lvl[l] : lvl[l] + sum;
      first = false;
    }
  return sum;
}

// pass 1: block (x, s) sums chunks [s kSlice, (s+1) kSlice) of its elements
// into the slice's first chunk slot
template <bool GRAM>
__global__ __launch_bounds__(256) void k_reduce_slices(double *part, int64_t nch, int p, int q,
                                                       int64_t sPart, const int *__restrict__ info) {
  if (*info) return;
  part += blockIdx.z * sPart;
  const int64_t pq = (int64_t)p * q;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= pq) return;
  if (GRAM && (int)(e / q) > (int)(e % q)) return;
  const int64_t c0 = (int64_t)blockIdx.y * kSlice;
  const int64_t cnt = (nch - c0 < kSlice) ? nch - c0 : kSlice;
  const double v = pairwise_sum(part + c0 * pq + e, cnt, pq);
  part[c0 * pq + e] = v;
}

// pass 2 (or the only pass): sum `count` values spaced `stride` apart
template <bool GRAM>
__global__ __launch_bounds__(256) void k_reduce(const double *__restrict__ part, int64_t count,
                                                int64_t stride, int p, int q,
                                                double *__restrict__ out, int64_t ldo,
                                                double *__restrict__ rblk, int64_t ldr, bool neg,
                                                int64_t sPart, int64_t sOut, int64_t sR,
                                                const int *__restrict__ info) {
  if (*info) return;
  part += blockIdx.z * sPart;
  out += blockIdx.z * sOut;
  if (rblk) rblk += blockIdx.z * sR;
  const int64_t pq = (int64_t)p * q;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= pq) return;
  const int i = (int)(e / q), j = (int)(e % q);
  if (GRAM && i > j) {
    out[(int64_t)i * p + j] = 0.0;
    return;
  }
  const double sum = pairwise_sum(part + e, count, stride);
  if (GRAM) {
    out[(int64_t)i * p + j] = sum;
  } else {
    out[(int64_t)i * ldo + j] = neg ? -sum : sum;
    if (rblk) rblk[i + (int64_t)j * ldr] = sum;
  }
}

hipError_t launch_reduce(bool gram, double *part, int64_t nch, int p, int q, double *out,
                         int64_t ldo, double *rblk, int64_t ldr, bool neg, const int *info,
                         hipStream_t s, int batch, int64_t sPart, int64_t sOut, int64_t sR) {
  const int64_t pq = (int64_t)p * q;
  const unsigned bx = (unsigned)((pq + 255) / 256);
  int64_t count = nch, stride = pq;
  if (nch > kSlice) {
    const unsigned ns = (unsigned)((nch + kSlice - 1) / kSlice);
    dim3 g(bx, ns, (unsigned)batch);
    if (gram)
      hipLaunchKernelGGL((k_reduce_slices<true>), g, dim3(256), 0, s, part, nch, p, q, sPart, info);
    else
      hipLaunchKernelGGL((k_reduce_slices<false>), g, dim3(256), 0, s, part, nch, p, q, sPart, info);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    count = ns;
    stride = pq * kSlice;
  }
  dim3 g(bx, 1, (unsigned)batch);
  if (gram)
    hipLaunchKernelGGL((k_reduce<true>), g, dim3(256), 0, s, part, count, stride, p, q, out, ldo, rblk,
                       ldr, neg, sPart, sOut, sR, info);
  else
    hipLaunchKernelGGL((k_reduce<false>), g, dim3(256), 0, s, part, count, stride, p, q, out, ldo,
                       rblk, ldr, neg, sPart, sOut, sR, info);
  return hipGetLastError();
}

// ----------------------------------------------------------------------------
// k_chol_inv: Cholesky W = U^T U of one panel's Gram matrix (Algorithm 1 /
// Algorithm 8, Cholesky step) and the inverse U^{-1}, in one workgroup with
// the whole matrix in LDS (padded with the identity to order 16 * 2^k).
// Right-looking Cholesky by 16-column panels, then the blocked in-place
// triangular inverse by block back substitution (device_common.h).
// ----------------------------------------------------------------------------
constexpr int kCholThreads = 512;

__global__ __launch_bounds__(kCholThreads) void k_chol_inv(const double *__restrict__ W, int w,
                                                           double *__restrict__ uout,
                                                           double *__restrict__ rblk, int64_t ldr,
                                                           double *__restrict__ uinv, int *info,
                                                           int col0, double skip_tol, int *skip) {
  extern __shared__ double S[];  // wp x wp, then the inverse's scratch
  __shared__ int flag;
  __shared__ double red[kCholThreads];
  if (*info) return;
  const int tid = threadIdx.x, nt = blockDim.x, wp = blocked_order(w);
  for (int e = tid; e < wp * wp; e += nt) {
    const int i = e / wp, j = e % wp;
    S[e] = (i < w && j < w) ? ((i <= j) ? W[i * w + j] : 0.0) : (i == j ? 1.0 : 0.0);
  }
  __syncthreads();
  if (skip) {
    // ||W - I||_F from the upper triangle, summed in a fixed order (each
    // thread its strided elements in turn, then a fixed tree); within the
    // tolerance the factor is U = I and the step it feeds is left out
    double acc = 0.0;
    for (int e = tid; e < w * w; e += nt) {
      const int i = e / w, j = e % w;
      if (i <= j) {
        const double v = S[i * wp + j] - (i == j ? 1.0 : 0.0);
        acc += (i == j ? 1.0 : 2.0) * v * v;
      }
    }
    red[tid] = acc;
    __syncthreads();
    for (int h = kCholThreads / 2; h > 0; h >>= 1) {
      if (tid < h) red[tid] += red[tid + h];
      __syncthreads();
    }
    const bool near = sqrt(red[0]) <= skip_tol;
    if (tid == 0) *skip = near ? 1 : 0;
    if (near) {
      for (int e = tid; e < w * w; e += nt) {
        const int i = e / w, j = e % w;
        const double u = (i == j) ? 1.0 : 0.0;
        if (uout) uout[e] = u;
        if (rblk) rblk[i + (int64_t)j * ldr] = u;
      }
      const int ldu = (int)padded_ld(w);
      for (int e = tid; e < w * ldu; e += nt) uinv[e] = (e / ldu == e % ldu) ? 1.0 : 0.0;
      return;
    }
  }
  const int fail = lds_cholesky_blocked(S, wp, &flag);
  if (fail) {
    if (tid == 0) atomicCAS(info, 0, col0 + fail);
    return;
  }
  for (int e = tid; e < w * w; e += nt) {
    const int i = e / w, j = e % w;
    const double u = (i <= j) ? S[i * wp + j] : 0.0;
    if (uout) uout[e] = u;
    if (rblk) rblk[i + (int64_t)j * ldr] = u;
  }
  __syncthreads();
  lds_upper_inverse_blocked(S, wp, S + wp * wp, S + wp * wp + 16 * wp);
  const int ldu = (int)padded_ld(w);
  for (int e = tid; e < w * ldu; e += nt) {
    const int i = e / ldu, c = e % ldu;
    uinv[e] = (c < i || c >= w) ? 0.0 : S[i * wp + c];
  }
}

// Panels wider than kLdsPanel: the same factorisation and inverse with the
// matrix (padded with the identity to order 256) in the device scratch G,
// one 512-thread workgroup (wide_cholesky / wide_upper_inverse).
constexpr int kWideThreads = 512;

__global__ __launch_bounds__(kWideThreads) void k_chol_inv_wide(
    const double *__restrict__ W, int w, double *__restrict__ uout, double *__restrict__ rblk,
    int64_t ldr, double *__restrict__ uinv, double *__restrict__ G, int *info, int col0,
    double skip_tol, int *skip) {
  extern __shared__ double S[];
  __shared__ int flag;
  __shared__ double red[kWideThreads];
  if (*info) return;
  const int tid = threadIdx.x, nt = blockDim.x, wp = blocked_order(w);
  if (skip) {
    // ||W - I||_F in a fixed order, as k_chol_inv
    double acc = 0.0;
    for (int e = tid; e < w * w; e += nt) {
      const int i = e / w, j = e % w;
      if (i <= j) {
        const double v = W[e] - (i == j ? 1.0 : 0.0);
        acc += (i == j ? 1.0 : 2.0) * v * v;
      }
    }
    red[tid] = acc;
    __syncthreads();
    for (int h = kWideThreads / 2; h > 0; h >>= 1) {
      if (tid < h) red[tid] += red[tid + h];
      __syncthreads();
    }
    const bool near = sqrt(red[0]) <= skip_tol;
    if (tid == 0) *skip = near ? 1 : 0;
    if (near) {
      for (int e = tid; e < w * w; e += nt) {
        const int i = e / w, j = e % w;
        const double u = (i == j) ? 1.0 : 0.0;
        if (uout) uout[e] = u;
        if (rblk) rblk[i + (int64_t)j * ldr] = u;
      }
      const int ldu = (int)padded_ld(w);
      for (int e = tid; e < w * ldu; e += nt) uinv[e] = (e / ldu == e % ldu) ? 1.0 : 0.0;
      return;
    }
  }
  for (int e = tid; e < wp * wp; e += nt) {
    const int i = e / wp, j = e % wp;
    G[e] = (i < w && j < w) ? ((i <= j) ? W[i * w + j] : 0.0) : (i == j ? 1.0 : 0.0);
  }
  __syncthreads();
  const int fail = wide_cholesky(G, wp, S, &flag);
  if (fail) {
    if (tid == 0) atomicCAS(info, 0, col0 + fail);
    return;
  }
  for (int e = tid; e < w * w; e += nt) {
    const int i = e / w, j = e % w;
    const double u = (i <= j) ? G[(int64_t)i * wp + j] : 0.0;
    if (uout) uout[e] = u;
    if (rblk) rblk[i + (int64_t)j * ldr] = u;
  }
  __syncthreads();
  wide_upper_inverse(G, wp, S);
  const int ldu = (int)padded_ld(w);
  for (int e = tid; e < w * ldu; e += nt) {
    const int i = e / ldu, c = e % ldu;
    uinv[e] = (c < i || c >= w) ? 0.0 : G[(int64_t)i * wp + c];
  }
}

hipError_t launch_chol_inv(const double *W, int w, double *uout, double *rblk, int64_t ldr,
                           double *uinv, int *info, int col0, hipStream_t s, double skip_tol,
                           int *skip, double *gwork) {
  if (w < 1 || w > kMaxPanel) return hipErrorInvalidValue;
  const int wp = blocked_order(w);
  if (w > kLdsPanel) {
    if (!gwork) return hipErrorInvalidValue;
    const size_t lds = (size_t)wide_lds_doubles(wp) * sizeof(double);
    static const hipError_t attr = hipFuncSetAttribute(
        (const void *)k_chol_inv_wide, hipFuncAttributeMaxDynamicSharedMemorySize,
        (int)((size_t)wide_lds_doubles(kMaxPanel) * sizeof(double)));
    if (attr != hipSuccess) return attr;
    hipLaunchKernelGGL(k_chol_inv_wide, dim3(1), dim3(kWideThreads), lds, s, W, w, uout, rblk,
                       ldr, uinv, gwork, info, col0, skip_tol, skip);
    return hipGetLastError();
  }
  const size_t lds = (size_t)blocked_lds_doubles(wp) * sizeof(double);
  static const hipError_t attr = hipFuncSetAttribute(
      (const void *)k_chol_inv, hipFuncAttributeMaxDynamicSharedMemorySize,
      (int)((size_t)blocked_lds_doubles(kLdsPanel) * sizeof(double)));
  if (attr != hipSuccess) return attr;
  hipLaunchKernelGGL(k_chol_inv, dim3(1), dim3(kCholThreads), lds, s, W, w, uout, rblk, ldr, uinv,
                     info, col0, skip_tol, skip);
  return hipGetLastError();
}

// ----------------------------------------------------------------------------
// Small n x n kernels of the QR adjoint dA = (dQ + Q copyltu(M)) R^{-T},
// M = R dR^T - dQ^T Q. One matrix per blockIdx.y (batched), n <= kMaxPanel.
// ----------------------------------------------------------------------------
// Rinv = R^{-1} (R column-major, ld n; Rinv row-major, ld n) one column per wave: column j solves R x = e_j by back
// substitution, sweeping the columns of R from the right (x_k = x_k / R_kk,
// applied as a multiply by the pivot's reciprocal, then x_i -= R_ik x_k for
// i < k: column k of R is read contiguously, and the columns eight steps
// ahead are in flight meanwhile). Lane l holds
// x_l, x_{l+64}, ... (n <= 256). Every column is independent, so a batch of
// n x n inverses is n x batch waves: a 128 x 128 inverse takes a few
// microseconds where one workgroup doing the whole matrix took ~0.1 ms (the
// adjoint's critical path waited for it).
__global__ __launch_bounds__(64) void k_tri_inv_cols(const double *__restrict__ R, int n,
                                                     int64_t sR, double *__restrict__ Rinv,
                                                     int64_t sRi, double *__restrict__ RinvT) {
  constexpr int D = 8;  // columns of R in flight ahead of the sweep
  R += blockIdx.y * sR;
  Rinv += blockIdx.y * sRi;
  if (RinvT) RinvT += blockIdx.y * sRi;
  const int j = blockIdx.x, lane = threadIdx.x;
  double x[4], rb[D][4];
  auto load_col = [&](double (&v)[4], int k) {  // rows of column k (zeros when k < 0)
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int i = lane + 64 * t;
      v[t] = (k >= 0 && i <= k && i < n) ? R[i + (int64_t)k * n] : 0.0;
    }
  };
  // the pivots' reciprocals (one IEEE division each, as LAPACK's unblocked
  // inverse scales by them), so that the sweep's dependency chain per column
  // is two shuffles, a multiply and an FMA
  double dinv[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int i = lane + 64 * t;
    x[t] = (i == j) ? 1.0 : 0.0;
    dinv[t] = (i <= j) ? 1.0 / R[i + (int64_t)i * n] : 0.0;
  }
#pragma unroll
  for (int u = 0; u < D; ++u) load_col(rb[u], j - u);
  for (int kb = j; kb >= 0; kb -= D) {
#pragma unroll
    for (int u = 0; u < D; ++u) {
      const int k = kb - u;
      if (k >= 0) {
        const int tk = k >> 6, lk = k & 63;
        double xs = x[0], ds = dinv[0];
#pragma unroll
        for (int t = 1; t < 4; ++t)
          if (tk == t) {
            xs = x[t];
            ds = dinv[t];
          }
        const double xk = __shfl(xs, lk) * __shfl(ds, lk);
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          const int i = lane + 64 * t;
          if (i == k) x[t] = xk;
          else if (i < k) x[t] -= rb[u][t] * xk;
        }
        load_col(rb[u], k - D);
      }
    }
  }
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int i = lane + 64 * t;
    if (i < n) {
      Rinv[(int64_t)i * n + j] = (i <= j) ? x[t] : 0.0;
      if (RinvT) RinvT[(int64_t)j * n + i] = (i <= j) ? x[t] : 0.0;  // R^{-T}, row-major
    }
  }
}

hipError_t launch_tri_inv(const double *R, int n, int64_t sR, double *Rinv, int64_t sRi, int batch,
                          hipStream_t s, double *RinvT) {
  if (n < 1 || n > kMaxPanel) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_tri_inv_cols, dim3((unsigned)n, (unsigned)batch), dim3(64), 0, s, R, n, sR,
                     Rinv, sRi, RinvT);
  return hipGetLastError();
}

// C = copyltu(M), M = R dR^T - P on and below the diagonal (row-major C).
// P = dQ^T Q from T = S^T dQ (upper triangle valid, row-major, ld n):
//   Q given:    P[i][j] = T[j][i]
//   recompute:  S = A and Q = A R^{-1}, so P[i][j] = sum_{k<=j} T[k][i] Rinv[k][j]
// dR == nullptr or has_p == 0 drop the corresponding term.
__global__ __launch_bounds__(256) void k_adj_c(int n, const double *__restrict__ T, int64_t sT,
                                               const double *__restrict__ R,
                                               const double *__restrict__ dR, int64_t sRn,
                                               const double *__restrict__ Rinv, int64_t sRi,
                                               int has_p, int recompute, double *__restrict__ C,
                                               int64_t sC) {
  const int64_t bi = blockIdx.y;
  T += bi * sT;
  R += bi * sRn;
  if (dR) dR += bi * sRn;
  Rinv += bi * sRi;
  C += bi * sC;
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= n * n) return;
  const int i = e / n, j = e % n;
  if (i < j) return;
  // the sums run in order of k; unrolling lets each thread keep several
  // loads in flight (the loops are latency-bound, not arithmetic-bound)
  double rdr = 0.0;
  if (dR) {
#pragma unroll 8
    for (int k = i; k < n; ++k) rdr += R[i + (int64_t)k * n] * dR[j + (int64_t)k * n];
  }
  double pv = 0.0;
  if (has_p) {
    if (recompute) {
#pragma unroll 8
      for (int k = 0; k <= j; ++k) pv += T[k * n + i] * Rinv[k * n + j];
    } else {
      pv = T[j * n + i];
    }
  }
  const double mv = rdr - pv;
  C[i * n + j] = mv;
  C[j * n + i] = mv;
}

// G = C R^{-T}: G[k][c] = sum_{l >= c} C[k][l] Rinv[c][l]   (row-major)
__global__ __launch_bounds__(256) void k_adj_g(int n, const double *__restrict__ C, int64_t sC,
                                               const double *__restrict__ RinvT, int64_t sRi,
                                               double *__restrict__ G, int64_t sG) {
  const int64_t bi = blockIdx.y;
  C += bi * sC;
  RinvT += bi * sRi;
  G += bi * sG;
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= n * n) return;
  const int k = e / n, c = e % n;
  // G[k][c] = sum_l C[k][l] R^{-T}[l][c]: the lanes of a wave read one row
  // of R^{-T} (row-major) contiguously
  double acc = 0.0;
#pragma unroll 8
  for (int l = c; l < n; ++l) acc += C[k * n + l] * RinvT[(int64_t)l * n + c];
  G[e] = acc;
}

// G = C R^{-T} as k_adj_g, written straight into the streaming pass's right
// operand (rows [off, off + n) of Y; rows [0, n) get R^{-T} when with_rt):
// the form used when Q is given, where Y's lower block is G itself.
__global__ __launch_bounds__(256) void k_adj_gy(int n, const double *__restrict__ C, int64_t sC,
                                                const double *__restrict__ RinvT, int64_t sRi,
                                                int with_rt, double *__restrict__ Y, int64_t ldy,
                                                int64_t sY) {
  const int64_t bi = blockIdx.y;
  C += bi * sC;
  RinvT += bi * sRi;
  Y += bi * sY;
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= n * n) return;
  const int k = e / n, c = e % n;
  double acc = 0.0;
#pragma unroll 8
  for (int l = c; l < n; ++l) acc += C[k * n + l] * RinvT[(int64_t)l * n + c];
  const int off = with_rt ? n : 0;
  if (with_rt) Y[(int64_t)k * ldy + c] = RinvT[(int64_t)k * n + c];
  Y[(int64_t)(off + k) * ldy + c] = acc;
}

// The right operand of the streaming pass, row-major with leading dim ldy:
//   rows [0, n) (only if with_rt): R^{-T};  rows [off, off + n): G, or
//   R^{-1} G when Q is recomputed from A (the pass then multiplies A).
__global__ __launch_bounds__(256) void k_adj_y(int n, const double *__restrict__ G, int64_t sG,
                                               const double *__restrict__ Rinv,
                                               const double *__restrict__ RinvT, int64_t sRi,
                                               int with_rt, int recompute, double *__restrict__ Y,
                                               int64_t ldy, int64_t sY) {
  const int64_t bi = blockIdx.y;
  G += bi * sG;
  Rinv += bi * sRi;
  RinvT += bi * sRi;
  Y += bi * sY;
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= n * n) return;
  const int k = e / n, c = e % n;
  const int off = with_rt ? n : 0;
  if (with_rt) Y[(int64_t)k * ldy + c] = RinvT[(int64_t)k * n + c];  // R^{-T}: zero above the diagonal
  double g;
  if (recompute) {
    g = 0.0;
    for (int j = k; j < n; ++j) g += Rinv[k * n + j] * G[j * n + c];
  } else {
    g = G[e];
  }
  Y[(int64_t)(off + k) * ldy + c] = g;
}

hipError_t launch_adj_small(int n, const double *T, int64_t sT, const double *R, const double *dR,
                            int64_t sRn, const double *Rinv, const double *RinvT, int64_t sRi,
                            int has_p, int recompute, double *C, double *G, int64_t sCG, double *Y,
                            int64_t ldy, int64_t sY, int with_rt, int batch, hipStream_t s) {
  dim3 g((unsigned)((n * n + 255) / 256), (unsigned)batch), blk(256);
  hipLaunchKernelGGL(k_adj_c, g, blk, 0, s, n, T, sT, R, dR, sRn, Rinv, sRi, has_p, recompute, C, sCG);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (!recompute) {
    hipLaunchKernelGGL(k_adj_gy, g, blk, 0, s, n, C, sCG, RinvT, sRi, with_rt, Y, ldy, sY);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(k_adj_g, g, blk, 0, s, n, C, sCG, RinvT, sRi, G, sCG);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_adj_y, g, blk, 0, s, n, G, sCG, Rinv, RinvT, sRi, with_rt, recompute, Y, ldy,
                     sY);
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

__global__ __launch_bounds__(256) void k_shift_diag(double *W, int w, double sqrt_m_u,
                                                    const int *__restrict__ info) {
  if (*info) return;
  __shared__ double shift;
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int i = 0; i < w; ++i) t += W[i + (int64_t)i * w];
    shift = sqrt_m_u * t;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < w; i += 256) W[i + (int64_t)i * w] += shift;
}

hipError_t launch_shift_diag(double *W, int w, double sqrt_m_u, const int *info, hipStream_t s) {
  if (w < 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_shift_diag, dim3(1), dim3(256), 0, s, W, w, sqrt_m_u, info);
  return hipGetLastError();
}

// Adaptive re-orthogonalisation: ||Z||_F of the rows x cols row-major Z
// (leading dim ldz) in a fixed order; within tol, Z := 0 and *skip = 1 (the
// update that would apply Z is then left out), else *skip = 0.
__global__ __launch_bounds__(512) void k_zskip(double *Z, int rows, int cols, int64_t ldz,
                                               double tol, int *skip, const int *__restrict__ info) {
  __shared__ double red[512];
  __shared__ int near;
  if (*info) return;
  const int tid = threadIdx.x;
  const int64_t count = (int64_t)rows * cols;
  double acc = 0.0;
  for (int64_t e = tid; e < count; e += 512) {
    const double v = Z[(e / cols) * ldz + e % cols];
    acc += v * v;
  }
  red[tid] = acc;
  __syncthreads();
  for (int h = 256; h > 0; h >>= 1) {
    if (tid < h) red[tid] += red[tid + h];
    __syncthreads();
  }
  if (tid == 0) {
    near = sqrt(red[0]) <= tol ? 1 : 0;
    *skip = near;
  }
  __syncthreads();
  if (near)
    for (int64_t e = tid; e < count; e += 512) Z[(e / cols) * ldz + e % cols] = 0.0;
}

hipError_t launch_zskip(double *Z, int rows, int cols, int64_t ldz, double tol, int *skip,
                        const int *info, hipStream_t s) {
  if (rows < 1 || cols < 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_zskip, dim3(1), dim3(512), 0, s, Z, rows, cols, ldz, tol, skip, info);
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

__global__ __launch_bounds__(256) void k_zero2d(double *p, int64_t rows, int64_t cols, int64_t ld,
                                                int64_t sb) {
  double *base = p + blockIdx.y * sb;
  const int64_t count = rows * cols;
  const int64_t stride = (int64_t)gridDim.x * 256;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < count; e += stride)
    base[(e / rows) * ld + e % rows] = 0.0;
}

hipError_t launch_zero2d(double *p, int64_t rows, int64_t cols, int64_t ld, int64_t sb, int batch,
                         hipStream_t s) {
  const int64_t count = rows * cols;
  if (count <= 0) return hipSuccess;
  int64_t blocks = (count + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_zero2d, dim3((unsigned)blocks, (unsigned)batch), dim3(256), 0, s, p, rows, cols,
                     ld, sb);
  return hipGetLastError();
}

__global__ void k_set_int(int *p, int v) { *p = v; }

// dst[:, c] = src[:, c] for the n columns of an m-row column-major block.
// A block copies 4096-row segments of one column; each thread moves 4 runs
// of 4 consecutive doubles, all loads issued before the stores.
template <bool VEC>
__global__ __launch_bounds__(256) void k_copy_cols(int64_t m, int64_t n, const double *__restrict__ src,
                                                   int64_t lds, double *__restrict__ dst, int64_t ldd) {
  const int64_t segs = (m + 4095) / 4096;
  for (int64_t t = blockIdx.x; t < segs * n; t += gridDim.x) {
    const int64_t c = t / segs, r0 = (t % segs) * 4096;
    const double *s = src + c * lds;
    double *d = dst + c * ldd;
    if (VEC && r0 + 4096 <= m) {
      double2 v[8];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int64_t i = r0 + 1024 * u + 4 * threadIdx.x;
        v[2 * u] = reinterpret_cast<const double2 *>(s + i)[0];
        v[2 * u + 1] = reinterpret_cast<const double2 *>(s + i)[1];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int64_t i = r0 + 1024 * u + 4 * threadIdx.x;
        reinterpret_cast<double2 *>(d + i)[0] = v[2 * u];
        reinterpret_cast<double2 *>(d + i)[1] = v[2 * u + 1];
      }
    } else {
      const int64_t r1 = (r0 + 4096 < m) ? r0 + 4096 : m;
      for (int64_t i = r0 + threadIdx.x; i < r1; i += 256) d[i] = s[i];
    }
  }
}

hipError_t launch_copy_cols(int64_t m, int64_t n, const double *src, int64_t lds, double *dst,
                            int64_t ldd, hipStream_t s) {
  if (m <= 0 || n <= 0) return hipSuccess;
  const int64_t work = (m + 4095) / 4096 * n;
  const int64_t bx = std::min<int64_t>(work, 16384);
  const bool vec = (lds % 2 == 0) && (ldd % 2 == 0) && ((uintptr_t)src % 16 == 0) &&
                   ((uintptr_t)dst % 16 == 0);
  if (vec)
    hipLaunchKernelGGL(k_copy_cols<true>, dim3((unsigned)bx), dim3(256), 0, s, m, n, src, lds, dst,
                       ldd);
  else
    hipLaunchKernelGGL(k_copy_cols<false>, dim3((unsigned)bx), dim3(256), 0, s, m, n, src, lds, dst,
                       ldd);
  return hipGetLastError();
}

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
