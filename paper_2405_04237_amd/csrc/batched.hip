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
// A wave's MFMA accumulators cover at most kTnFlushRows of its rows before
// they are added into the LDS result (the four waves in a fixed order), so
// no running sum sees more than ~128 sequential additions at either level.
constexpr int kTnFlushRows = 512;

// LDS layout (doubles)
constexpr int kYSize = kBatchMaxPanel * kBatchMaxN + 64;  // projections (+ read slack)
constexpr int kBB = kBatchMaxPanel * kBatchMaxPanel;
struct Lds {
  double *y, *w, *ua, *ub, *ui, *s, *d;
  int *flag;
  double *trash;  // a word that absorbs masked-off writes
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
  L.flag = reinterpret_cast<int *>(L.d + kBatchMaxPanel);  // flag[0]: slot, flag[1]: team wait
  L.trash = reinterpret_cast<double *>(L.flag + 8);           // inside the 64-byte flag area
  return L;
}

// The matrices' addresses are read from device arrays, so the compiler cannot
// prove they point to global memory and would emit flat instructions, which
// count against the LDS wait counter as well: every LDS read would then wait
// for the whole load ring. Every matrix access goes through these
// global-typed helpers instead.
// Pairs of doubles use a plain vector type (HIP's double2 is a class whose
// copy goes through a generic pointer) aligned to 8 bytes only: a column
// with an odd leading dimension still moves two rows per 16-byte access
// (global memory accesses need only 4-byte alignment).
typedef double dpair __attribute__((ext_vector_type(2)));
typedef dpair dpair8 __attribute__((aligned(8)));
typedef __attribute__((address_space(1))) double gdouble;
typedef __attribute__((address_space(1))) dpair8 gdpair;
__device__ __forceinline__ double gld(const double *p) { return *(const gdouble *)p; }
__device__ __forceinline__ double2 gld2(const double *p) {
  const dpair v = *(const gdpair *)p;
  return double2{v.x, v.y};
}
__device__ __forceinline__ void gst(double *p, double v) { *(gdouble *)p = v; }
__device__ __forceinline__ void gst2(double *p, double2 v) {
  dpair w;
  w.x = v.x;
  w.y = v.y;
  *(gdpair *)p = w;
}

// Global-memory writes made by one wave before the barrier are visible to
// every wave of the workgroup after it. All waves of a workgroup run on one
// compute unit and share its vector L1, so workgroup-scope release and
// acquire (the barrier's own fences) suffice: agent scope would write back
// and invalidate the L2 at every phase. Exchanges between the workgroups of
// a team use agent-scope fences of their own (team_reduce).
__device__ inline void wg_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __syncthreads();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// ---------------------------------------------------------------------------
// TN product reduced over the rows: out (LDS) = A^T B over rows [0, m), A is
// m x na and B m x nb (column-major; na <= 16 NA, nb <= 16 NB columns). The
// four waves split the rows (wave w takes the w-th SR-row block of every
// 4 SR-row round) and each accumulates every 16 x 16 output block, so each
// column line is loaded once per wave; loads run through a three-deep
// register ring. trans = false: out[i * ldo + j]; true: out[j * ldo + i].
// Lane maps as in the single-matrix k_tn: lane (cl, g) feeds rows 4g..4g+3
// of column 16 a + cl; D element e of block (a, b) is (16a + g + 4e, 16b + cl).
// ---------------------------------------------------------------------------
template <int NA, int NB, bool SAME>
__device__ __forceinline__ void tn_run(int64_t m, int na, int nb, const double *A, int64_t lda,
                                       const double *B, int64_t ldb, double *out, int ldo,
                                       bool trans, double *trash) {
  // SAME: B is A (a Gram matrix), so only A's columns are loaded and each
  // loaded value feeds both operands
  constexpr int NL = SAME ? NA : NA + NB;  // column blocks loaded per stage
  // 16-row steps per ring stage: a stage holds at most 16 doubles per lane
  constexpr int U = (NL <= 1) ? 4 : (NL <= 3 ? 2 : 1);
  constexpr int SR = 16 * U;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, g = lane >> 4, cl = lane & 15;
  for (int e = tid; e < na * nb; e += kThreads) {
    const int i = e / nb, j = e % nb;
    out[trans ? j * ldo + i : i * ldo + j] = 0.0;
  }
  __syncthreads();

  // columns past na / nb read column 0: they reach only outputs never stored
  const double *pa[NA];
  const double *pb[NB];
#pragma unroll
  for (int a = 0; a < NA; ++a) {
    const int c = 16 * a + cl;
    pa[a] = A + (int64_t)(c < na ? c : 0) * lda + 4 * g + wave * SR;
  }
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    const int c = 16 * b + cl;
    pb[b] = B + (int64_t)(c < nb ? c : 0) * ldb + 4 * g + wave * SR;
  }
  d4 acc[NA][NB];
#pragma unroll
  for (int a = 0; a < NA; ++a)
#pragma unroll
    for (int b = 0; b < NB; ++b) acc[a][b] = d4{0.0, 0.0, 0.0, 0.0};

  auto flush = [&]() {  // out += acc, wave 0 first; acc = 0
    // the lane coordinates pass through an empty asm statement so that the
    // destination addresses are formed here, not hoisted out of the row
    // loop where they would stay live in registers
    int fg = g, fcl = cl;
    asm volatile("" : "+v"(fg), "+v"(fcl));
#pragma unroll
    for (int w = 0; w < 4; ++w) {
      if (wave == w) {
#pragma unroll
        for (int a = 0; a < NA; ++a)
#pragma unroll
          for (int b = 0; b < NB; ++b)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
              // entries outside na x nb go to the trash word (an address
              // select rather than a lane mask per entry: those masks would
              // stay live in scalar registers through the whole row loop)
              const int I = 16 * a + fg + 4 * e, J = 16 * b + fcl;
              double *dst = (I < na && J < nb) ? out + (trans ? J * ldo + I : I * ldo + J) : trash;
              *dst += acc[a][b][e];
            }
      }
      __syncthreads();
    }
#pragma unroll
    for (int a = 0; a < NA; ++a)
#pragma unroll
      for (int b = 0; b < NB; ++b) acc[a][b] = d4{0.0, 0.0, 0.0, 0.0};
  };
  typedef double Stage[NL][U][4];
  auto load = [&](Stage &v, int64_t off) {  // off: row offset of the round
#pragma unroll
    for (int c = 0; c < NL; ++c) {
      const double *p = (c < NA ? pa[c] : pb[c - NA]) + off;
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const double2 x0 = gld2(p + 16 * u);
        const double2 x1 = gld2(p + 16 * u + 2);
        v[c][u][0] = x0.x;
        v[c][u][1] = x0.y;
        v[c][u][2] = x1.x;
        v[c][u][3] = x1.y;
      }
    }
  };
  auto compute = [&](const Stage &v) {
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int a = 0; a < NA; ++a)
#pragma unroll
          for (int b = 0; b < NB; ++b)
            acc[a][b] = mfma16x16x4(v[a][u][s], v[SAME ? b : NA + b][u][s], acc[a][b]);
  };

  // 32-bit round and tile counters (a matrix has at most 2^33 rows)
  constexpr int round_rows = 4 * SR;
  constexpr int per_flush = kTnFlushRows / SR;  // rounds between flushes
  const int nfull = (int)(m / round_rows);      // rounds with every row present
  if (nfull > 0) {
    auto at = [&](int r) -> int64_t { return (int64_t)round_rows * (r < nfull ? r : nfull - 1); };
    int since = 0;  // rounds since the last flush
    auto step = [&](const Stage &v, int) {
      compute(v);
      if (++since == per_flush) {
        flush();
        since = 0;
      }
    };
    if constexpr (NL >= 5) {  // wide products: two stages (at least 40 MFMAs of cover each)
      Stage v0, v1;
      load(v0, 0);
      int r = 0;
      for (; r + 2 <= nfull; r += 2) {
        load(v1, at(r + 1));
        __builtin_amdgcn_sched_barrier(0);
        step(v0, r);
        __builtin_amdgcn_sched_barrier(0);
        load(v0, at(r + 2));
        __builtin_amdgcn_sched_barrier(0);
        step(v1, r + 1);
        __builtin_amdgcn_sched_barrier(0);
      }
      if (r < nfull) step(v0, r);
    } else {
      Stage v0, v1, v2;
      load(v0, 0);
      load(v1, at(1));
      int r = 0;
      for (; r + 3 <= nfull; r += 3) {
        load(v2, at(r + 2));
        __builtin_amdgcn_sched_barrier(0);
        step(v0, r);
        __builtin_amdgcn_sched_barrier(0);
        load(v0, at(r + 3));
        __builtin_amdgcn_sched_barrier(0);
        step(v1, r + 1);
        __builtin_amdgcn_sched_barrier(0);
        load(v1, at(r + 4));
        __builtin_amdgcn_sched_barrier(0);
        step(v2, r + 2);
        __builtin_amdgcn_sched_barrier(0);
      }
      if (r < nfull) step(v0, r);
      if (r + 1 < nfull) step(v1, r + 1);
    }
  }
  // the last, partial round: rows past m contribute zeros
  const int64_t rt = (int64_t)nfull * round_rows;
  if (rt < m) {
    Stage v;
#pragma unroll
    for (int c = 0; c < NL; ++c) {
      const double *p = (c < NA ? pa[c] : pb[c - NA]) + rt;
#pragma unroll
      for (int u = 0; u < U; ++u)
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          const int64_t row = rt + wave * SR + 16 * u + 4 * g + s;
          double x = 0.0;
          if (row < m) x = gld(p + 16 * u + s);
          v[c][u][s] = x;
        }
    }
    compute(v);
  }
  flush();
  wg_sync();
}

// One call site for every TN product of the factorisation: dispatch on the
// block counts (A side <= 2 blocks: the panel; B side up to 8 blocks, 128
// columns, taken in passes of at most 4 blocks; a Gram matrix in one pass
// with one operand stream).
__device__ __forceinline__ void wg_tn(int64_t m, int na, int nb, const double *A, int64_t lda,
                                   const double *B, int64_t ldb, double *out, int ldo, bool trans,
                                   double *trash) {
  const int ka = (na + 15) / 16;
  if (A == B && na == nb) {
    if (ka == 1) tn_run<1, 1, true>(m, na, nb, A, lda, B, ldb, out, ldo, trans, trash);
    if (ka == 2) tn_run<2, 2, true>(m, na, nb, A, lda, B, ldb, out, ldo, trans, trash);
    return;
  }
  for (int j0 = 0; j0 < nb; j0 += 64) {
    const int nbp = (nb - j0 < 64) ? nb - j0 : 64;
    const int kb = (nbp + 15) / 16;
    const double *Bp = B + (int64_t)j0 * ldb;
    double *op = out + (trans ? (int64_t)j0 * ldo : j0);
#define CQR_TN_CASE(X, Y) \
    if (ka == X && kb == Y) tn_run<X, Y, false>(m, na, nbp, A, lda, Bp, ldb, op, ldo, trans, trash);
    CQR_TN_CASE(1, 1) CQR_TN_CASE(1, 2) CQR_TN_CASE(1, 3) CQR_TN_CASE(1, 4)
    CQR_TN_CASE(2, 1) CQR_TN_CASE(2, 2) CQR_TN_CASE(2, 3) CQR_TN_CASE(2, 4)
#undef CQR_TN_CASE
  }
}

// ---------------------------------------------------------------------------
// Row-streaming NN product C = L Y (+ Cin when sub) over rows [0, m): L m x p
// column-major, Y p x q row-major in LDS (ld ldy; reads up to 64 columns past
// a tile's start stay inside the LDS region), Cin / C m x q column-major.
// 32 x 16 NX tiles (NX = 1, 2 or 4: the narrowest that covers q, or 4) are
// dealt to the waves round-robin (tile t: row tile t / nct, column tile
// t % nct). The k steps of a wave's consecutive full tiles form
// one stream through a three-deep register ring; a tile's first stage also
// carries its Cin. C may alias L when q <= 64 (a wave reads its tile's rows
// fully before writing them, and no other wave touches those rows); Cin may
// equal C. Lane maps as in k_nn with two rows per lane: lane (cl, g) holds
// rows r0 + 2 cl + {0, 1} and columns c0 + NX (g + 4 e) + x of the tile.
// ---------------------------------------------------------------------------
// NS: the 4-wide k groups of each 16-wide k step that are streamed (2 when
// p <= 8: the other two hold only k >= p, whose terms are exact zeros).
template <int NX, bool SUB, int NS = 4>
__device__ __forceinline__ void nn_run(int64_t m, int p, int q, const double *L, int64_t ldl,
                                       const double *Y, int ldy, const double *Cin, int64_t ldci,
                                       double *C, int64_t ldc) {
  constexpr int TW = 16 * NX;  // tile width
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, g = lane >> 4, cl = lane & 15;
  const int nct = (q + TW - 1) / TW;
  const int nk = (p + 15) / 16;
  // 32-bit tile and step counters (a matrix has at most 2^33 rows)
  const int nrt_full = (int)(m / 32);
  const int nt_full = nrt_full * nct;
  const int mine = (nt_full > wave) ? (nt_full - wave + 3) / 4 : 0;  // full tiles of this wave
  const int T = mine * nk;                                            // steps

  struct Stage {
    double l[4][2];  // L[rl + y][k], k = 16 ks + 4 s + g
  };
  d4 acc[NX][2];
  double cn[4][NX][2];  // Cin[rl + y][c0 + NX (g + 4 e) + x] of the next tile to start

  auto tile_of = [&](int i, int64_t &r0, int &c0) {  // i-th tile of this wave
    const int t = wave + 4 * i;
    r0 = (int64_t)(t / nct) * 32;
    c0 = (int)(t % nct) * TW;
  };
  auto load_l = [&](double (&l)[4][2], int64_t rl, int ks, int64_t rows_left) {
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      const int k = 16 * ks + 4 * s + g;
      const double *pl = L + (int64_t)(k < p ? k : p - 1) * ldl + rl;
      double x0, x1;
      if (rows_left >= 2) {
        const double2 t = gld2(pl);
        x0 = t.x;
        x1 = t.y;
      } else {
        x0 = x1 = 0.0;
        if (rows_left > 0) x0 = gld(pl);
        if (rows_left > 1) x1 = gld(pl + 1);
      }
      l[s][0] = (k < p) ? x0 : 0.0;
      l[s][1] = (k < p) ? x1 : 0.0;
    }
  };
  auto load_c = [&](double (&cv)[4][NX][2], int64_t rl, int c0, int64_t rows_left) {
#pragma unroll
    for (int e = 0; e < 4; ++e)
#pragma unroll
      for (int x = 0; x < NX; ++x) {
        const int col = c0 + NX * (g + 4 * e) + x;
        double x0 = 0.0, x1 = 0.0;
        if constexpr (SUB) {
          // columns past q read column q - 1: they reach only outputs never stored
          const double *pc = Cin + (int64_t)(col < q ? col : q - 1) * ldci + rl;
          if (rows_left >= 2) {
            const double2 t = gld2(pc);
            x0 = t.x;
            x1 = t.y;
          } else {
            if (rows_left > 0) x0 = gld(pc);
            if (rows_left > 1) x1 = gld(pc + 1);
          }
        }
        cv[e][x][0] = x0;
        cv[e][x][1] = x1;
      }
  };
  auto mma = [&](const double (&l)[4][2], int ks, int c0) {
    const double *yl = Y + c0 + NX * cl;
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      const int k = 16 * ks + 4 * s + g;
      double ya[NX];
#pragma unroll
      for (int x = 0; x < NX; ++x) {
        const double yv = yl[(k < p ? k : 0) * ldy + x];
        ya[x] = (k < p) ? yv : 0.0;
      }
#pragma unroll
      for (int x = 0; x < NX; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y) acc[x][y] = mfma16x16x4(ya[x], l[s][y], acc[x][y]);
    }
  };
  auto store_one = [&](int64_t rl, int col, int x, int e, int64_t rows_left) {
    double *pc = C + (int64_t)col * ldc + rl;
    if (rows_left >= 2) {
      gst2(pc, double2{acc[x][0][e], acc[x][1][e]});
    } else {
      if (rows_left > 0) gst(pc, acc[x][0][e]);
      if (rows_left > 1) gst(pc + 1, acc[x][1][e]);
    }
  };
  auto store = [&](int64_t rl, int c0, int64_t rows_left) {
    if (c0 + TW <= q) {  // every column of the tile is stored (uniform)
#pragma unroll
      for (int e = 0; e < 4; ++e)
#pragma unroll
        for (int x = 0; x < NX; ++x) store_one(rl, c0 + NX * (g + 4 * e) + x, x, e, rows_left);
    } else {
#pragma unroll
      for (int e = 0; e < 4; ++e)
#pragma unroll
        for (int x = 0; x < NX; ++x) {
          const int col = c0 + NX * (g + 4 * e) + x;
          if (col < q) store_one(rl, col, x, e, rows_left);
        }
    }
  };
  auto init_acc = [&](const double (&cv)[4][NX][2]) {
#pragma unroll
    for (int e = 0; e < 4; ++e)
#pragma unroll
      for (int x = 0; x < NX; ++x) {
        acc[x][0][e] = cv[e][x][0];
        acc[x][1][e] = cv[e][x][1];
      }
  };

  if (T > 0) {
    // load cursor (L only: a tile's Cin is loaded when the tile before it
    // starts, into cn, so the ring stages stay small)
    int li = 0, lc0, lks = 0, lt = 0;
    int64_t lr0;
    tile_of(0, lr0, lc0);
    auto load = [&](Stage &st) {
      const int64_t rl = lr0 + 2 * cl;
      load_l(st.l, rl, lks, 2);
      if (lt + 1 < T) {  // advance (past the end the last step is loaded again)
        ++lt;
        if (++lks == nk) {
          lks = 0;
          tile_of(++li, lr0, lc0);
        }
      }
    };
    // compute cursor
    int ci = 0, cc0, cks = 0;
    int64_t cr0;
    tile_of(0, cr0, cc0);
    load_c(cn, cr0 + 2 * cl, cc0, 2);
    auto step = [&](const Stage &st) {
      if (cks == 0) {
        init_acc(cn);
        // the next tile's Cin (the last tile loads its own again: an
        // unconditional load keeps the registers in place)
        int64_t nr0;
        int nc0;
        tile_of(ci + 1 < mine ? ci + 1 : ci, nr0, nc0);
        load_c(cn, nr0 + 2 * cl, nc0, 2);
      }
      mma(st.l, cks, cc0);
      if (++cks == nk) {
        store(cr0 + 2 * cl, cc0, 2);
        cks = 0;
        tile_of(++ci, cr0, cc0);
      }
    };
    Stage s0, s1, s2;
    load(s0);
    load(s1);
    int t = 0;
    for (; t + 3 <= T; t += 3) {
      load(s2);
      __builtin_amdgcn_sched_barrier(0);
      step(s0);
      __builtin_amdgcn_sched_barrier(0);
      load(s0);
      __builtin_amdgcn_sched_barrier(0);
      step(s1);
      __builtin_amdgcn_sched_barrier(0);
      load(s1);
      __builtin_amdgcn_sched_barrier(0);
      step(s2);
      __builtin_amdgcn_sched_barrier(0);
    }
    if (t < T) step(s0);
    if (t + 1 < T) step(s1);
  }
  // the last, partial row tile (fewer than 32 rows), masked
  if ((int64_t)nrt_full * 32 < m) {
    for (int ct = 0; ct < nct; ++ct) {
      if ((nt_full + ct) % 4 != wave) continue;
      const int64_t r0 = (int64_t)nrt_full * 32;
      const int c0 = ct * TW;
      const int64_t rl = r0 + 2 * cl;
      const int64_t left = m - rl;
      Stage st;
      load_c(cn, rl, c0, left);
      init_acc(cn);
      for (int ks = 0; ks < nk; ++ks) {
        load_l(st.l, rl, ks, left);
        mma(st.l, ks, c0);
      }
      store(rl, c0, left);
    }
  }
  wg_sync();
}

// Dispatch on the tile width (the narrowest of 16, 32, 64 columns that
// covers q, else 64) and on SUB (C = Cin + L Y, Y then holding the negated
// factor, or C = L Y).
template <int NX>
__device__ __forceinline__ void nn_sub(int64_t m, int p, int q, const double *L, int64_t ldl,
                                       const double *Y, int ldy, const double *Cin, int64_t ldci,
                                       double *C, int64_t ldc, bool sub) {
  if (NX == 1 && p <= 8) {  // an 8-column panel: half of each k step
    if (sub)
      nn_run<NX, true, 2>(m, p, q, L, ldl, Y, ldy, Cin, ldci, C, ldc);
    else
      nn_run<NX, false, 2>(m, p, q, L, ldl, Y, ldy, Cin, ldci, C, ldc);
    return;
  }
  if (sub)
    nn_run<NX, true>(m, p, q, L, ldl, Y, ldy, Cin, ldci, C, ldc);
  else
    nn_run<NX, false>(m, p, q, L, ldl, Y, ldy, Cin, ldci, C, ldc);
}

__device__ __forceinline__ void wg_nn(int64_t m, int p, int q, const double *L, int64_t ldl,
                                   const double *Y, int ldy, const double *Cin, int64_t ldci,
                                   double *C, int64_t ldc, bool sub) {
  if (q <= 16)
    nn_sub<1>(m, p, q, L, ldl, Y, ldy, Cin, ldci, C, ldc, sub);
  else if (q <= 32)
    nn_sub<2>(m, p, q, L, ldl, Y, ldy, Cin, ldci, C, ldc, sub);
  else
    nn_sub<4>(m, p, q, L, ldl, Y, ldy, Cin, ldci, C, ldc, sub);
}

// Spin limit of a team barrier (s_sleep 2 per try, about 3 s in all): a
// partner that never arrives ends the wait with an error, not a hang.
constexpr int64_t kTeamSpins = int64_t(1) << 25;

// A workgroup's share of one matrix: rows [r0, r0 + mloc) of the member-th of
// `team` workgroups; part / cnt: the team's exchange buffer and counter.
struct Team {
  int64_t r0, mloc;
  int member, team;
  double *part;
  int *cnt;
  int barriers;  // team barriers passed so far
};

// out (LDS, count doubles: this member's partial sum over its rows) := the
// sum of all members' partials, in member order, identical in every member.
// Returns false if a partner did not arrive within the spin limit.
__device__ __forceinline__ bool team_reduce(const Lds &S, Team &T, double *out, int count) {
  const int tid = threadIdx.x;
  double *buf = T.part + (int64_t)(T.barriers & 1) * T.team * kTeamSlot;
  double *mine = buf + (int64_t)T.member * kTeamSlot;
  for (int e = tid; e < count; e += kThreads) gst(mine + e, out[e]);
  __threadfence();  // release this member's partial (all L2s)
  __syncthreads();
  if (tid == 0) {
    const int target = T.team * (T.barriers + 1);
    atomicAdd(T.cnt, 1);
    int ok = 0;
    for (int64_t i = 0; i < kTeamSpins; ++i) {
      if (__hip_atomic_load(T.cnt, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) >= target) {
        ok = 1;
        break;
      }
      __builtin_amdgcn_s_sleep(2);
    }
    S.flag[1] = ok;
  }
  __syncthreads();
  const bool ok = S.flag[1] != 0;
  __threadfence();  // acquire the partners' partials
  if (ok) {
    for (int e = tid; e < count; e += kThreads) {
      double x = 0.0;
      for (int k = 0; k < T.team; ++k) x += gld(buf + (int64_t)k * kTeamSlot + e);
      out[e] = x;
    }
  }
  __syncthreads();
  ++T.barriers;
  return ok;
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
    gst(R + (r0 + i) + (int64_t)(r0 + c) * n, (i <= c) ? acc : 0.0);
  }
}

// mCQR2GS of one matrix by one workgroup, as a sequence of phases with one
// call site per streaming primitive. Returns 0 or the breakdown column.
__device__ __forceinline__ int wg_mcqr2gs(const Lds &S, int n, int b, const double *A0,
                                          int64_t lda, double *Q0, double *R, Team &T) {
  const int tid = threadIdx.x;
  const bool lead = T.member == 0;  // the member that writes R
  const int64_t m = T.mloc;         // this workgroup's rows: [T.r0, T.r0 + m)
  const double *A = A0 + T.r0;
  double *Q = Q0 + T.r0;
  if (lead)
    for (int e = tid; e < n * n; e += kThreads) gst(R + e, 0.0);
  const int w0 = n < b ? n : b;
  int s = 0;  // first column of the current panel
  int w = w0;
  int ph = 0;
  for (;;) {
    // one of: TN product, NN product, or a small step done in place
    int op = 0;  // 1 = TN, 2 = NN
    int64_t tm = m;
    int ta = 0, tb = 0, tldo = 0, np = 0, nq = 0, nldy = 0;
    // LDS operands start at an LDS address (not null), so that the compiler
    // still sees every value they may take as LDS and emits LDS instructions
    const double *tA = nullptr, *tB = nullptr, *nL = nullptr, *nY = S.y, *nCin = nullptr;
    double *tout = S.w, *nC = nullptr;
    bool ttrans = false, nsub = false;
    const int ps = s - b, nr = n - s;
    double *Xj = Q + (int64_t)s * lda;
    const int ldw = (int)padded_ld(w);
    bool next = false;
    switch (ph) {
      // first panel: CholeskyQR2, reading A and writing Q
      case 0: op = 1; ta = tb = w; tA = tB = A; tout = S.w; tldo = w; break;
      case 1: { const int f = wg_chol_inv(S, w, S.ua, ldw); if (f) return f; break; }
      case 2: op = 2; np = nq = w; nL = A; nY = S.ui; nldy = ldw; nC = Q; break;
      case 3: op = 1; ta = tb = w; tA = tB = Q; tout = S.w; tldo = w; break;
      case 4: { const int f = wg_chol_inv(S, w, S.ub, ldw); if (f) return f; break; }
      case 5: op = 2; np = nq = w; nL = Q; nY = S.ui; nldy = ldw; nC = Q; break;
      case 6:
        if (lead) wg_r_upper_product(R, n, 0, w, S.ub, S.ua);
        next = true;
        break;
      // panel s >= b: project the finished panel (columns ps..s-1 of Q) out
      // of every column to its right; the projection is that block row of R
      case 7:
        op = 1; ta = b; tb = nr; tA = Q + (int64_t)ps * lda; tB = (ps == 0) ? A + (int64_t)s * lda : Xj;
        tout = S.y; tldo = (int)padded_ld(nr);
        break;
      case 8: {
        const int ldy = (int)padded_ld(nr);
        for (int e = tid; e < b * nr; e += kThreads) {
          const int i = e / nr, j = e % nr;
          if (lead) gst(R + (ps + i) + (int64_t)(s + j) * n, S.y[i * ldy + j]);
          S.y[i * ldy + j] = -S.y[i * ldy + j];
        }
        __syncthreads();
        break;
      }
      case 9:
        op = 2; np = b; nq = nr; nL = Q + (int64_t)ps * lda; nY = S.y; nldy = (int)padded_ld(nr);
        nCin = (ps == 0) ? A + (int64_t)s * lda : Xj; nC = Xj; nsub = true;
        break;
      // first CholeskyQR of the new panel (factor Ua)
      case 10: op = 1; ta = tb = w; tA = tB = Xj; tout = S.w; tldo = w; break;
      case 11: { const int f = wg_chol_inv(S, w, S.ua, ldw); if (f) return s + f; break; }
      case 12: op = 2; np = nq = w; nL = Xj; nY = S.ui; nldy = ldw; nC = Xj; break;
      // one Gram-Schmidt pass of the new panel against all finished columns
      // (the coefficients as Qt^T Q_{1:j-1}, stored transposed)
      case 13: op = 1; ta = w; tb = s; tA = Xj; tB = Q; tout = S.y; tldo = ldw; ttrans = true; break;
      case 14: {
        // the coefficients times Ua add into R's block above the panel; the
        // update then subtracts Q_{1:j-1} times the coefficients
        for (int e = tid; lead && e < s * w; e += kThreads) {
          const int i = e % s, c = e / s;
          double acc = 0.0;
          for (int k = 0; k <= c; ++k) acc += S.y[i * ldw + k] * S.ua[k * w + c];
          double *pr = R + i + (int64_t)(s + c) * n;
          gst(pr, gld(pr) + acc);
        }
        __syncthreads();
        for (int e = tid; e < s * ldw; e += kThreads) S.y[e] = -S.y[e];
        __syncthreads();
        break;
      }
      case 15: op = 2; np = s; nq = w; nL = Q; nY = S.y; nldy = ldw; nCin = Xj; nC = Xj; nsub = true; break;
      // second CholeskyQR of the panel (factor Ub); its R block is Ub Ua
      case 16: op = 1; ta = tb = w; tA = tB = Xj; tout = S.w; tldo = w; break;
      case 17: { const int f = wg_chol_inv(S, w, S.ub, ldw); if (f) return s + f; break; }
      case 18: op = 2; np = nq = w; nL = Xj; nY = S.ui; nldy = ldw; nC = Xj; break;
      case 19:
        if (lead) wg_r_upper_product(R, n, s, w, S.ub, S.ua);
        __syncthreads();
        next = true;
        break;
    }
    if (op == 1) {
      wg_tn(tm, ta, tb, tA, lda, tB, lda, tout, tldo, ttrans, S.trash);
      if (T.team > 1 && !team_reduce(S, T, tout, (ttrans ? tb : ta) * tldo)) return -1;
    } else if (op == 2) {
      wg_nn(tm, np, nq, nL, lda, nY, nldy, nCin ? nCin : nC, lda, nC, lda, nsub);
    }
    if (next) {
      if (s == 0) s = b; else s += b;
      if (s >= n) return 0;
      w = (n - s < b) ? n - s : b;
      ph = 7;
    } else {
      ++ph;
    }
  }
}

// queue word and team counters to zero (a kernel, so that graphs replay it)
__global__ void k_reset_batched(int *queue, int *cnt, int ncnt) {
  if (blockIdx.x == 0 && threadIdx.x == 0) *queue = 0;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < ncnt; i += gridDim.x * blockDim.x) cnt[i] = 0;
}

__global__ __launch_bounds__(kThreads) void k_batched_mod(
    const BatchSlot *__restrict__ slots, int nslots, const int64_t *__restrict__ ms,
    const int *__restrict__ ns, const int *__restrict__ bs, const double *const *__restrict__ dA,
    const int64_t *__restrict__ dlda, double *const *__restrict__ dQ, double *const *__restrict__ dR,
    int *__restrict__ dinfo, int *queue, double *team_part, int *team_cnt) {
  extern __shared__ double lds[];
  const Lds S = lds_layout(lds);
  const int tid = threadIdx.x;
  for (;;) {
    if (tid == 0) S.flag[0] = atomicAdd(queue, 1);
    __syncthreads();
    const int slot = S.flag[0];
    __syncthreads();
    if (slot >= nslots) break;  // uniform: every wave leaves together
    const BatchSlot sl = slots[slot];
    const int i = sl.matrix;
    const int64_t m = ms[i];
    Team T;
    T.member = sl.member;
    T.team = sl.team;
    // members take equal 64-row-aligned shares; the last takes the rest
    const int64_t share = (m / sl.team) / 64 * 64;
    T.r0 = share * sl.member;
    T.mloc = (sl.member == sl.team - 1) ? m - T.r0 : share;
    T.part = team_part + sl.part;
    T.cnt = team_cnt + sl.cnt;
    T.barriers = 0;
    const int fail = wg_mcqr2gs(S, ns[i], bs[i], dA[i], dlda[i], dQ[i], dR[i], T);
    if (tid == 0 && sl.member == 0) dinfo[i] = fail;
    wg_sync();
  }
}

}  // namespace

size_t batched_lds_bytes() {
  return (size_t)(kYSize + 4 * kBB + 64 + kBB + kBatchMaxPanel) * sizeof(double) + 64;
}

// The kernel's dynamic LDS limit, raised once per process (a function-local
// static is initialised once and thread-safely) before it is launched or its
// occupancy is queried.
static hipError_t batched_lds_attr() {
  static const hipError_t attr =
      hipFuncSetAttribute((const void *)k_batched_mod, hipFuncAttributeMaxDynamicSharedMemorySize,
                          (int)batched_lds_bytes());
  return attr;
}

hipError_t launch_batched_mod(int grid, const BatchSlot *slots, int nslots, const int64_t *ms,
                              const int *ns, const int *bs, const double *const *dA,
                              const int64_t *dlda, double *const *dQ, double *const *dR,
                              int *dinfo, int *queue, double *team_part, int *team_cnt, int nteams,
                              hipStream_t s) {
  const size_t lds = batched_lds_bytes();
  const hipError_t attr = batched_lds_attr();
  if (attr != hipSuccess) return attr;
  hipLaunchKernelGGL(k_reset_batched, dim3(1), dim3(256), 0, s, queue, team_cnt, nteams);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_batched_mod, dim3((unsigned)grid), dim3(kThreads), lds, s, slots, nslots, ms,
                     ns, bs, dA, dlda, dQ, dR, dinfo, queue, team_part, team_cnt);
  return hipGetLastError();
}

int batched_blocks_per_cu() {
  if (batched_lds_attr() != hipSuccess) return 1;
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, (const void *)k_batched_mod, kThreads,
                                                   batched_lds_bytes()) != hipSuccess)
    return 1;
  return nb > 0 ? nb : 1;
}

}  // namespace cqr
