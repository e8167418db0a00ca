// libcqr host library: the C ABI of include/cqr.h.
//
// Argument checks, workspace layout, the split-m plan, and the two panel
// schedules of arXiv 2405.04237 as stream-ordered kernel chains:
//   CQR2GS  (Algorithm 7 = Algorithm 6/8 twice, then R = R2 R1)
//   mCQR2GS (Algorithm 9)
//   sCQR3   (Algorithm 5: shifted CholeskyQR, Algorithm 4, then CholeskyQR2)
// Nothing here synchronises with the device except cqr_get_info and
// cqr_profile_query.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <numeric>
#include <map>
#include <mutex>
#include <vector>

#include "batched.h"
#include "cqr.h"
#include "kernels.h"

namespace {

using cqr::kMaxPanel;

constexpr int64_t kAlign = 256;
constexpr int64_t kPartChunks = 256;   // split-m partial capacity, in units of n*b doubles
constexpr int64_t kPartGramChunks = 2048;  // ... and at least this many b x b Gram partials
constexpr int64_t kTargetWaves = 2048; // split-m grid size aimed for (8 waves per CU)
constexpr int64_t kMaxChunkRows = 16384;

// Waves of the split-m product kernel resident at once on MI355X (256 CUs x 4
// SIMDs, one wave each). Grids are sized to whole multiples of it so that no
// round of waves runs nearly empty; a constant, so the plan (and with it the
// rounding of every sum) does not depend on the device queried.
constexpr int64_t kWaveSlots = 1024;

// Number of row chunks for `units` output tiles (x batch): at least
// kTargetWaves waves and chunks of at most kMaxChunkRows rows, rounded down
// to fill whole rounds of kWaveSlots waves.
int64_t split_m_chunks(int64_t m, int64_t units) {
  const int64_t min_chunks = (m + kMaxChunkRows - 1) / kMaxChunkRows;
  const int64_t waves = std::max(kTargetWaves, units * min_chunks);
  const int64_t rounds = (waves + kWaveSlots - 1) / kWaveSlots;
  return std::max<int64_t>(1, rounds * kWaveSlots / units);
}

int64_t round_up(int64_t x, int64_t a) { return (x + a - 1) / a * a; }

// Column strides that are multiples of 8 KiB put the 128 column lines one
// wave of the split-m product reads at one row into a handful of cache sets;
// on MI355X that costs the projection kernels about a third of their rate.
// Such inputs are factored in a staging copy whose stride is shifted by one
// 128-byte line, then copied out to Q.
bool aliasing_ld(int64_t ld) { return ld % 1024 == 0; }
int64_t staging_ld(int64_t m) {
  const int64_t l = round_up(m, 16);
  return aliasing_ld(l) ? l + 16 : l;
}

// ---------------------------------------------------------------- workspace
struct Layout {
  int64_t w, uinv, ua, ub, g, y, yz, part, r1, r2, stage, flags, total;  // byte offsets / size
  int64_t part_elems, ldw;                                 // ldw: staging leading dim
};

Layout make_layout(int64_t m, int64_t n, int64_t b, int schedule, bool stage) {
  Layout L{};
  int64_t off = 0;
  auto take = [&](int64_t elems) {
    const int64_t o = off;
    off = round_up(off + elems * 8, kAlign);
    return o;
  };
  L.flags = take(32);  // adaptive repetition decisions (ints)
  L.w = take(b * b);
  L.uinv = take(b * cqr::padded_ld(b));
  L.ua = take(b * b);
  L.ub = take(b * b);
  // panels wider than the LDS Cholesky holds are factored in device scratch
  L.g = cqr::chol_scratch_doubles((int)b) > 0 ? take(cqr::chol_scratch_doubles((int)b)) : -1;
  L.y = take(n * cqr::padded_ld(std::max(n, b)));
  // MOD with look-ahead: the re-orthogonalisation coefficients Z (at most
  // n x b) get their own buffer, since the trailing Y is still being read
  L.yz = (schedule == CQR_SCHED_MOD) ? take(n * cqr::padded_ld(b)) : -1;
  // Room for the split-m plan of every product: kPartChunks slices of the
  // widest projection, and enough b x b slices that a Gram of few panels
  // (sCQR3, or n a small multiple of b) still fills the GPU; never more
  // slices than the 16-row chunks m has (rounded up so that the size does
  // not change with every m).
  const int64_t slices = round_up((m + 15) / 16, 1024);
  L.part_elems = std::max(kPartChunks * std::max(n * b, b * b), kPartGramChunks * b * b);
  L.part_elems = std::min(L.part_elems, slices * std::max(n * b, b * b));
  L.part = take(L.part_elems);
  if (schedule == CQR_SCHED_ORIG || schedule == CQR_SCHED_SCQR3) {
    L.r1 = take(n * n);
    L.r2 = take(n * n);
  } else {
    L.r1 = L.r2 = -1;
  }
  if (stage) {
    L.ldw = staging_ld(m);
    L.stage = take(L.ldw * n);
  } else {
    L.ldw = 0;
    L.stage = -1;
  }
  L.total = off;
  return L;
}

bool valid_schedule(int schedule) {
  return schedule == CQR_SCHED_MOD || schedule == CQR_SCHED_ORIG || schedule == CQR_SCHED_SCQR3;
}

int64_t effective_panel(int64_t m, int64_t n, int64_t b, int schedule) {
  if (schedule == CQR_SCHED_SCQR3) return n;  // whole-matrix algorithm
  if (b == 0) b = cqr_default_panel(m, n, schedule);
  return std::min(b, n);
}

// ---------------------------------------------------------------- per device
struct LibBuf {
  void *p = nullptr;
  size_t bytes = 0;
};

struct DevState {
  LibBuf ws;            // factorisation workspace
  LibBuf bwd;           // backward workspace
  int *info = nullptr;  // internal info word (read by cqr_get_info)
  // recorded on the caller's stream after every call that used ws or bwd
  hipEvent_t last_use = nullptr;
  // side stream (default priority) for independent small work, forked from
  // and joined back into the caller's stream with events
  hipStream_t aux = nullptr;
  hipEvent_t fork = nullptr, join = nullptr;
  std::mutex side;  // one fork/join sequence at a time on this device
};
std::mutex g_mu;
std::map<int, DevState> g_dev;

// The current device's side stream and its fork/join events (created on
// first use). Callers hold DevState::side while they enqueue a fork/join
// sequence.
hipError_t side_stream(DevState **out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  std::lock_guard<std::mutex> lk(g_mu);
  DevState &d = g_dev[dev];
  if (!d.aux) {
    e = hipStreamCreateWithFlags(&d.aux, hipStreamNonBlocking);
    if (e != hipSuccess) return e;
    e = hipEventCreateWithFlags(&d.fork, hipEventDisableTiming);
    if (e != hipSuccess) return e;
    e = hipEventCreateWithFlags(&d.join, hipEventDisableTiming);
    if (e != hipSuccess) return e;
  }
  *out = &d;
  return hipSuccess;
}

#define CQR_TRY(expr)                    \
  do {                                   \
    const hipError_t e_ = (expr);        \
    if (e_ != hipSuccess) return e_;     \
  } while (0)

// True when `s` is being captured into a graph.
bool capturing(hipStream_t s) {
  hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(s, &st) != hipSuccess) return false;
  return st != hipStreamCaptureStatusNone;
}

// A library-owned buffer of at least `bytes`, grown in stream order on `s`:
// `s` first waits for the last call that used the old buffer (d.last_use,
// recorded on that call's stream), the old buffer is released with
// hipFreeAsync and the new one taken with hipMallocAsync, both on `s`. The
// host never waits for the device. Caller holds g_mu.
hipError_t ensure_buffer(DevState &d, LibBuf &b, size_t bytes, hipStream_t s) {
  if (b.bytes >= bytes) return hipSuccess;
  if (b.p) {
    if (d.last_use) CQR_TRY(hipStreamWaitEvent(s, d.last_use, 0));
    CQR_TRY(hipFreeAsync(b.p, s));
    b.p = nullptr;
    b.bytes = 0;
  }
  CQR_TRY(hipMallocAsync(&b.p, bytes, s));
  b.bytes = bytes;
  return hipSuccess;
}

// Mark the end of a call that used a library-owned buffer on `s`.
hipError_t mark_use(DevState &d, hipStream_t s) {
  if (!d.last_use) CQR_TRY(hipEventCreateWithFlags(&d.last_use, hipEventDisableTiming));
  return hipEventRecord(d.last_use, s);
}

// ---------------------------------------------------------------- profiling
struct Rec {
  hipEvent_t a, b;
  int kind;
  double flops, bytes;
};
struct Acc {
  int64_t n = 0;
  double ms = 0, flops = 0, bytes = 0;
};
bool g_prof = false;
// Set while cqr_factor_noalloc runs on this thread: its launches are never
// bracketed by timing events (creating an event may allocate).
thread_local bool t_no_events = false;
unsigned g_prof_mask = ~0u;  // kernel classes bracketed while profiling is on
std::vector<Rec> g_recs;
std::vector<hipEvent_t> g_pool;
Acc g_acc[CQR_K_COUNT];

hipEvent_t pool_get() {
  if (!g_pool.empty()) {
    hipEvent_t e = g_pool.back();
    g_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

template <class F>
hipError_t timed(hipStream_t s, int kind, double flops, double bytes, F &&f) {
  if (!g_prof || t_no_events || !(g_prof_mask & (1u << kind))) return f();
  std::lock_guard<std::mutex> lk(g_mu);
  hipEvent_t a = pool_get(), b = pool_get();
  if (!a || !b) return hipErrorOutOfMemory;
  hipError_t e = hipEventRecord(a, s);
  if (e != hipSuccess) return e;
  e = f();
  if (e != hipSuccess) return e;
  e = hipEventRecord(b, s);
  if (e != hipSuccess) return e;
  g_recs.push_back({a, b, kind, flops, bytes});
  return hipSuccess;
}

// ---------------------------------------------------------------- one factorisation
struct Run {
  hipStream_t s;
  hipStream_t aux;               // look-ahead side stream (null: none)
  hipEvent_t fork, join;         // main -> aux and aux -> main
  double *Yz;                    // Z buffer of the look-ahead chain
  double adaptive;               // > 0: tolerance of the run-time repetition choice
  int *zskip, *cskip;            // its decisions (device words)
  int *info;
  int64_t m, n;
  double *W, *Uinv, *Ua, *Ub, *G, *Y, *part, *R1, *R2;
  int64_t part_elems;
  double *Qout;  // staged runs: the caller's Q, written by each panel's final step
  int64_t ldq;
  int upd_tile, proj_tile;  // kernel variants of the updates and projections
};

void plan_chunks(const Run &r, int64_t tiles, int64_t pq, int64_t *rc, int64_t *nch) {
  const int64_t cap = std::max<int64_t>(1, r.part_elems / std::max<int64_t>(1, pq));
  int64_t want = split_m_chunks(r.m, tiles);
  want = std::min({want, cap, (r.m + 15) / 16, int64_t(4096)});
  want = std::max<int64_t>(want, 1);
  int64_t rows = round_up((r.m + want - 1) / want, 16);
  *rc = rows;
  *nch = (r.m + rows - 1) / rows;
}

// W = X^T X for the w columns at X (split-m partials + fixed-order reduce)
hipError_t step_gram(Run &r, const double *X, int64_t ldx, int w) {
  int64_t rc, nch;
  const int64_t tiles = cqr::tn_tiles(true, w, w, true);
  plan_chunks(r, tiles, (int64_t)w * w, &rc, &nch);
  CQR_TRY(timed(r.s, CQR_K_GRAM, double(r.m) * w * w, 8.0 * r.m * w, [&] {
    return cqr::launch_tn(true, r.m, w, w, X, ldx, X, ldx, r.part, rc, nch, r.info, r.s);
  }));
  return timed(r.s, CQR_K_REDUCE, double(nch) * w * w, 8.0 * (nch + 1) * w * w, [&] {
    return cqr::launch_reduce(true, r.part, nch, w, w, r.W, w, nullptr, 0, false, r.info, r.s);
  });
}

// U = chol(W), Uinv = U^{-1}; U optionally to uout (row-major) and/or the R block.
// skip: a repeated CholeskyQR under the run-time choice (U = I when W is
// within r.adaptive of I; the decision goes to *skip).
hipError_t step_chol(Run &r, int w, double *uout, double *rblk, int64_t ldr, int col0,
                     int *skip = nullptr) {
  const double wf = w;
  return timed(r.s, CQR_K_CHOL, 2.0 * wf * wf * wf / 3.0, 8.0 * 4 * wf * wf, [&] {
    return cqr::launch_chol_inv(r.W, w, uout, rblk, ldr, r.Uinv, r.info, col0, r.s, r.adaptive,
                                skip, r.G);
  });
}

// Q = X U^{-1} (the Q_j := A_j U^{-1} step); Q may be X (in place). col >= 0
// marks the panel's final Q, which a staged run also writes to the caller's
// Q at that column.
// skip: U^{-1} may be I by the run-time choice; an in-place product without a
// second destination is then left out.
hipError_t step_trsm(Run &r, const double *X, double *Qo, int64_t ld, int w, int64_t col = -1,
                     const int *skip = nullptr) {
  double *q2 = (col >= 0 && r.Qout) ? r.Qout + col * r.ldq : nullptr;
  const int *sk = (X == Qo && !q2) ? skip : nullptr;
  return timed(r.s, CQR_K_TRSM, double(r.m) * w * w, (q2 ? 24.0 : 16.0) * r.m * w, [&] {
    return cqr::launch_nn(false, true, r.m, w, w, X, ld, r.Uinv, cqr::padded_ld(w), nullptr, ld, Qo,
                          ld, r.info, r.s, nullptr, 0, 0, 1, 0, 0, 0, 0, 0, q2, r.ldq, sk);
  });
}

// Y = Qp^T Z: -Y row-major in r.Y (the update's operand), +Y into the R block if given
hipError_t step_proj(Run &r, const double *Qp, int64_t ld, int p, const double *Z, int q,
                     double *rblk, int64_t ldr) {
  int64_t rc, nch;
  // the split-m plan (and with it the order of every sum) is that of the
  // default tiles whatever variant runs, so the variants agree bit for bit
  const int64_t tiles = cqr::tn_tiles(false, p, q);
  plan_chunks(r, tiles, (int64_t)p * q, &rc, &nch);
  CQR_TRY(timed(r.s, CQR_K_PROJ, 2.0 * r.m * p * q, 8.0 * r.m * (p + q), [&] {
    return cqr::launch_tn(false, r.m, p, q, Qp, ld, Z, ld, r.part, rc, nch, r.info, r.s, 1, 0, 0,
                          0, r.proj_tile);
  }));
  return timed(r.s, CQR_K_REDUCE, double(nch) * p * q, 8.0 * (nch + 1) * p * q, [&] {
    return cqr::launch_reduce(false, r.part, nch, p, q, r.Y, cqr::padded_ld(q), rblk, ldr, true,
                              r.info, r.s);
  });
}

// Zo = Zi - Qp Y with Ym = -Y (row-major, leading dim ldy); Zo may be Zi
// skip (in place only): Y may have been set to 0 by the run-time choice,
// and the update is then left out.
hipError_t step_update_y(Run &r, const double *Qp, int64_t ld, int p, const double *Zi, double *Zo,
                         int q, const double *Ym, int64_t ldy, const int *skip = nullptr) {
  const int kind = cqr::nn_short_k(p, Qp, ld, Zi, ld, Zo, ld) ? CQR_K_UPDATE : CQR_K_UPDATE_LONG;
  const int *sk = (Zi == Zo) ? skip : nullptr;
  return timed(r.s, kind, 2.0 * r.m * p * q, 8.0 * r.m * (p + 2.0 * q), [&] {
    return cqr::launch_nn(true, false, r.m, p, q, Qp, ld, Ym, ldy, Zi, ld, Zo, ld, r.info, r.s,
                          nullptr, 0, 0, 1, 0, 0, 0, 0, 0, nullptr, 0, sk, r.upd_tile);
  });
}

// Zo = Zi - Qp Y  (r.Y holds -Y for these q columns); Zo may be Zi (in place)
hipError_t step_update(Run &r, const double *Qp, int64_t ld, int p, const double *Zi, double *Zo,
                       int q, const int *skip = nullptr) {
  return step_update_y(r, Qp, ld, p, Zi, Zo, q, r.Y, cqr::padded_ld(q), skip);
}

// One CQRGS pass (Algorithm 6; Algorithm 8 with the Allreduces replaced by
// split-m reductions), writing Q into X and its R into Rd (n x n, ld n).
// Columns not yet produced are read from src (A on the first pass, so that
// A is never copied or written); src may equal X.
hipError_t pass_cqrgs(Run &r, const double *src, double *X, int64_t ld, int64_t b, double *Rd,
                      bool final) {
  const int64_t n = r.n;
  for (int64_t s = 0; s < n; s += b) {
    const int64_t e = std::min(n, s + b);
    const int w = (int)(e - s);
    double *Xj = X + s * ld;
    const double *Aj = (s == 0) ? src : Xj;                          // panel j before its CQR
    const double *Ar = (s == 0) ? src + e * ld : X + e * ld;         // trailing panels
    // CholeskyQR of the panel; its factor is the diagonal block of R
    CQR_TRY(step_gram(r, Aj, ld, w));
    CQR_TRY(step_chol(r, w, nullptr, Rd + s + s * n, n, (int)s));
    CQR_TRY(step_trsm(r, Aj, Xj, ld, w, final ? s : -1));
    if (e < n) {
      // remove the new Q panel from the columns to its right; the
      // coefficients are the panel's block row of R
      CQR_TRY(step_proj(r, Xj, ld, w, Ar, (int)(n - e), Rd + s + e * n, n));
      CQR_TRY(step_update(r, Xj, ld, w, Ar, X + e * ld, (int)(n - e)));
    }
  }
  return hipSuccess;
}

hipError_t run_orig(Run &r, const double *A, double *Q, int64_t ld, int64_t b, double *R) {
  const int64_t n = r.n;
  CQR_TRY(timed(r.s, CQR_K_SMALL, 0, 16.0 * n * n, [&] { return cqr::launch_zero(r.R1, n * n, r.s); }));
  CQR_TRY(timed(r.s, CQR_K_SMALL, 0, 16.0 * n * n, [&] { return cqr::launch_zero(r.R2, n * n, r.s); }));
  CQR_TRY(pass_cqrgs(r, A, Q, ld, b, r.R1, false));  // [Q1, R1] = CQRGS(A)
  CQR_TRY(pass_cqrgs(r, Q, Q, ld, b, r.R2, true));   // [Q, R2]  = CQRGS(Q1)
  const double nf = n;
  return timed(r.s, CQR_K_SMALL, nf * nf * nf / 3.0, 24.0 * nf * nf, [&] {
    return cqr::launch_trmm_upper((int)n, r.R2, r.R1, R, r.info, r.s);  // R = R2 R1
  });
}

// Shifted CholeskyQR3 (Algorithm 5) on the whole matrix (n <= kMaxPanel):
// [Q1, R1] = sCQR(A) (Algorithm 4), [Q, R2] = CQR2(Q1) (Algorithm 3) with
// R2 = Rc Rb, R = R2 R1.
hipError_t run_scqr3(Run &r, const double *A, double *Q, int64_t ld, double *R) {
  const int w = (int)r.n;
  // s = sqrt(m) u ||A||_F^2, u = 2^-53; ||A||_F^2 = trace(A^T A)
  const double sqrt_m_u = std::sqrt((double)r.m) * std::ldexp(1.0, -53);
  CQR_TRY(step_gram(r, A, ld, w));                                   // G = A^T A
  CQR_TRY(timed(r.s, CQR_K_SMALL, 2.0 * w, 16.0 * w, [&] {
    return cqr::launch_shift_diag(r.W, w, sqrt_m_u, r.info, r.s);    // W = G + s I
  }));
  CQR_TRY(step_chol(r, w, nullptr, r.R1, w, 0));                     // W = R1^T R1
  CQR_TRY(step_trsm(r, A, Q, ld, w));                                // Q1 = A R1^{-1}
  CQR_TRY(step_gram(r, Q, ld, w));                                   // CholeskyQR2 of Q1
  CQR_TRY(step_chol(r, w, r.Ua, nullptr, 0, 0));
  CQR_TRY(step_trsm(r, Q, Q, ld, w));
  CQR_TRY(step_gram(r, Q, ld, w));
  CQR_TRY(step_chol(r, w, r.Ub, nullptr, 0, 0));
  CQR_TRY(step_trsm(r, Q, Q, ld, w, 0));
  const double wf = w;
  CQR_TRY(timed(r.s, CQR_K_SMALL, wf * wf * wf / 3.0, 24.0 * wf * wf, [&] {
    return cqr::launch_r_upper_product(w, r.Ub, r.Ua, r.R2, w, r.info, r.s);  // R2 = Rc Rb
  }));
  return timed(r.s, CQR_K_SMALL, wf * wf * wf / 3.0, 24.0 * wf * wf, [&] {
    return cqr::launch_trmm_upper(w, r.R2, r.R1, R, r.info, r.s);             // R = R2 R1
  });
}

hipError_t run_mod(Run &r, const double *A, double *Q, int64_t ld, int64_t b, double *R);

hipError_t run_schedule(Run &r, int schedule, const double *A, double *Q, int64_t ld, int64_t b,
                        double *R) {
  if (schedule == CQR_SCHED_ORIG) return run_orig(r, A, Q, ld, b, R);
  if (schedule == CQR_SCHED_SCQR3) return run_scqr3(r, A, Q, ld, R);
  return run_mod(r, A, Q, ld, b, R);
}

hipError_t run_mod(Run &r, const double *A, double *Q, int64_t ld, int64_t b, double *R) {
  const int64_t n = r.n;
  CQR_TRY(timed(r.s, CQR_K_SMALL, 0, 8.0 * n * n, [&] { return cqr::launch_zero(R, n * n, r.s); }));
  // first panel: CholeskyQR2, reading A_1 and writing Q_1
  {
    const int w = (int)std::min(n, b);
    CQR_TRY(step_gram(r, A, ld, w));
    CQR_TRY(step_chol(r, w, r.Ua, nullptr, 0, 0));
    CQR_TRY(step_trsm(r, A, Q, ld, w));
    int *cs = r.adaptive > 0 ? r.cskip : nullptr;
    CQR_TRY(step_gram(r, Q, ld, w));
    CQR_TRY(step_chol(r, w, r.Ub, nullptr, 0, 0, cs));
    CQR_TRY(step_trsm(r, Q, Q, ld, w, 0, cs));
    CQR_TRY(timed(r.s, CQR_K_SMALL, 0, 0, [&] {
      return cqr::launch_r_upper_product(w, r.Ub, r.Ua, R, n, r.info, r.s);  // R_11 = R2 R1
    }));
  }
  for (int64_t s = b; s < n; s += b) {
    const int64_t ps = s - b, e = std::min(n, s + b);
    const int w = (int)(e - s), pw = (int)b;
    double *Qprev = Q + ps * ld, *Xj = Q + s * ld;
    // the trailing columns are still A's until the first update writes them to Q
    const double *Ar = (ps == 0) ? A + s * ld : Xj;
    // project the finished previous panel out of every column to its right;
    // the coefficients fill the previous panel's block row of R
    CQR_TRY(step_proj(r, Qprev, ld, pw, Ar, (int)(n - s), R + ps + s * n, n));
    // Look-ahead: update panel j's own columns first; panel j's chain then
    // runs on the side stream while this stream updates panels j+1..k. The
    // chain touches only columns <= e and its own workspace (W, U^{-1}, Ua,
    // Ub, partials, Z); the rest of the update only columns > e and Y.
    const bool ahead = r.aux && e < n;
    Run c = r;
    if (ahead) {
      const int64_t ldy = cqr::padded_ld((int)(n - s));
      CQR_TRY(step_update_y(r, Qprev, ld, pw, Ar, Xj, w, r.Y, ldy));
      CQR_TRY(hipEventRecord(r.fork, r.s));
      CQR_TRY(hipStreamWaitEvent(r.aux, r.fork, 0));
      c.s = r.aux;
      c.Y = r.Yz;
    } else {
      CQR_TRY(step_update(r, Qprev, ld, pw, Ar, Xj, (int)(n - s)));
    }
    // first CholeskyQR of the panel (factor Ua)
    CQR_TRY(step_gram(c, Xj, ld, w));
    CQR_TRY(step_chol(c, w, c.Ua, nullptr, 0, (int)s));
    CQR_TRY(step_trsm(c, Xj, Xj, ld, w));
    // one classical Gram-Schmidt pass against all finished panels
    // (coefficients Z); R above the panel gains Z Ua (c.Y holds -Z, so the
    // R update subtracts (-Z) Ua)
    CQR_TRY(step_proj(c, Q, ld, (int)s, Xj, w, nullptr, 0));
    int *zs = nullptr, *cs = nullptr;
    if (c.adaptive > 0) {  // run-time choice: Z := 0 when ||Z||_F is within the tolerance
      zs = c.zskip;
      cs = c.cskip;
      CQR_TRY(timed(c.s, CQR_K_SMALL, 2.0 * s * w, 8.0 * s * w, [&] {
        return cqr::launch_zskip(c.Y, (int)s, w, cqr::padded_ld(w), c.adaptive, zs, c.info, c.s);
      }));
    }
    CQR_TRY(step_update(c, Q, ld, (int)s, Xj, Xj, w, zs));
    CQR_TRY(timed(c.s, CQR_K_SMALL, 2.0 * s * w * w / 2, 0, [&] {
      return cqr::launch_r_add_zu((int)s, w, c.Y, cqr::padded_ld(w), c.Ua, R + s * n, n, c.info, c.s);
    }));
    // CholeskyQR again (factor Ub); the diagonal block of R is Ub Ua
    CQR_TRY(step_gram(c, Xj, ld, w));
    CQR_TRY(step_chol(c, w, c.Ub, nullptr, 0, (int)s, cs));
    CQR_TRY(step_trsm(c, Xj, Xj, ld, w, s, cs));
    CQR_TRY(timed(c.s, CQR_K_SMALL, 0, 0, [&] {
      return cqr::launch_r_upper_product(w, c.Ub, c.Ua, R + s + s * n, n, c.info, c.s);
    }));
    if (ahead) {
      const int64_t ldy = cqr::padded_ld((int)(n - s));
      CQR_TRY(step_update_y(r, Qprev, ld, pw, Ar + (int64_t)w * ld, Xj + (int64_t)w * ld,
                            (int)(n - e), r.Y + w, ldy));
      CQR_TRY(hipEventRecord(r.join, r.aux));
      CQR_TRY(hipStreamWaitEvent(r.s, r.join, 0));
    }
  }
  return hipSuccess;
}

bool misaligned(const void *p, uintptr_t a) { return ((uintptr_t)p % a) != 0; }

int check_args(int64_t m, int64_t n, int64_t b, const double *A, int64_t lda, const double *Q,
               const double *R, int schedule) {
  if (n < 1 || m < n || lda < std::max<int64_t>(1, m) || b < 0) return CQR_ERR_ARG;
  if (n > (int64_t(1) << 20) || m > (int64_t(1) << 40)) return CQR_ERR_ARG;
  if (!A || !Q || !R) return CQR_ERR_ARG;
  if (misaligned(A, 8) || misaligned(Q, 8) || misaligned(R, 8)) return CQR_ERR_ARG;
  if (!valid_schedule(schedule)) return CQR_ERR_ARG;
  if (effective_panel(m, n, b, schedule) > kMaxPanel) return CQR_ERR_UNSUPPORTED;
  return CQR_OK;
}

// ---------------------------------------------------------------- backward
struct BwdLayout {
  int64_t info, part, t, rinv, rinvt, c, g, y, total;
  int64_t nch, rc, ldy;
};

BwdLayout make_bwd_layout(int64_t m, int64_t n, int64_t batch) {
  BwdLayout L{};
  // pass 1 (upper 64 x 64 tiles): about one round of resident waves
  // (kWaveSlots), so that every wave streams a long run of rows; the
  // factorisation's plan (two rounds or more) cut 262144 rows into 400-row
  // chunks whose partials and start-up cost as much as their products
  const int64_t tiles = cqr::tn_tiles(true, (int)n, (int)n);
  int64_t want = std::max<int64_t>(1, kWaveSlots / (tiles * batch));
  want = std::max(want, (m + kMaxChunkRows - 1) / kMaxChunkRows);
  want = std::min({want, (m + 15) / 16, int64_t(1024)});
  want = std::max<int64_t>(want, 1);
  L.rc = round_up((m + want - 1) / want, 16);
  L.nch = (m + L.rc - 1) / L.rc;
  L.ldy = cqr::padded_ld(n);
  int64_t off = 0;
  auto take = [&](int64_t bytes) {
    const int64_t o = off;
    off = round_up(off + bytes, kAlign);
    return o;
  };
  L.info = take(kAlign);
  L.part = take(8 * batch * L.nch * n * n);
  L.t = take(8 * batch * n * n);
  L.rinv = take(8 * batch * n * n);
  L.rinvt = take(8 * batch * n * n);
  L.c = take(8 * batch * n * n);
  L.g = take(8 * batch * n * n);
  L.y = take(8 * batch * 2 * n * L.ldy);
  L.total = off;
  return L;
}

int check_bwd(int64_t batch, int64_t m, int64_t n, const double *Q, const double *A, int64_t lda,
              int64_t stride, const double *R, const double *dQ, const double *dR, const double *dA) {
  if (batch < 1 || batch > 65535 || n < 1 || m < n || lda < std::max<int64_t>(1, m)) return CQR_ERR_ARG;
  if (batch > 1 && stride < lda * n) return CQR_ERR_ARG;
  if (!R || !dA || (!Q && !A)) return CQR_ERR_ARG;
  const void *ptrs[] = {Q, A, R, dQ, dR, dA};
  for (const void *p : ptrs)
    if (p && misaligned(p, 8)) return CQR_ERR_ARG;
  if (n > kMaxPanel) return CQR_ERR_UNSUPPORTED;
  return CQR_OK;
}

}  // namespace

extern "C" {

int64_t cqr_default_panel(int64_t m, int64_t n, int schedule) {
  (void)m;
  if (n <= 0) return 0;
  if (schedule == CQR_SCHED_SCQR3) return n;
  // mCQR2GS keeps O(u) orthogonality at kappa = 1e15 with a handful of
  // panels (the paper uses three); CQR2GS needs narrower panels there.
  const int64_t parts = (schedule == CQR_SCHED_ORIG) ? 16 : 4;
  int64_t b = round_up((n + parts - 1) / parts, 16);
  b = std::max<int64_t>(16, std::min<int64_t>(b, schedule == CQR_SCHED_ORIG ? 64 : cqr::kLdsPanel));
  return std::min(b, n);
}

size_t cqr_workspace_bytes_ld(int64_t m, int64_t n, int64_t b, int64_t lda, int schedule) {
  if (n < 1 || m < n || b < 0 || lda < m) return 0;
  if (!valid_schedule(schedule)) return 0;
  const int64_t be = effective_panel(m, n, b, schedule);
  return (size_t)make_layout(m, n, be, schedule, aliasing_ld(lda)).total;
}

size_t cqr_workspace_bytes(int64_t m, int64_t n, int64_t b, int schedule) {
  return cqr_workspace_bytes_ld(m, n, b, m, schedule);
}

int cqr_factor_ex(int64_t m, int64_t n, int64_t b, const double *A, int64_t lda, double *Q,
                  double *R, void *stream, const cqr_options *opt) {
  const int schedule = opt ? opt->schedule : CQR_SCHED_MOD;
  const int st = check_args(m, n, b, A, lda, Q, R, schedule);
  if (st != CQR_OK) return st;
  if (opt && (opt->update_tile < CQR_TILE_AUTO || opt->update_tile > CQR_TILE_RESIDENT ||
              opt->proj_tile < CQR_TILE_AUTO || opt->proj_tile > CQR_TILE_NARROW))
    return CQR_ERR_ARG;
  const int64_t be = effective_panel(m, n, b, schedule);
  // staged when lda aliases and the workspace has room (else factored in place)
  Layout lay = make_layout(m, n, be, schedule, aliasing_ld(lda));
  const Layout plain = make_layout(m, n, be, schedule, false);
  hipStream_t s = (hipStream_t)stream;

  char *ws = nullptr;
  int *info = opt ? opt->d_info : nullptr;
  if (opt && opt->workspace) {
    if (opt->workspace_bytes < (size_t)plain.total) return CQR_ERR_WORKSPACE;
    if (misaligned(opt->workspace, kAlign)) return CQR_ERR_ARG;
    if (opt->workspace_bytes < (size_t)lay.total) lay = plain;
    ws = (char *)opt->workspace;
  }
  DevState *lib_state = nullptr;  // set when the library's workspace is used
  if (!ws || !info) {
    const bool cap = capturing(s);
    if (cap && !ws) return CQR_ERR_ARG;  // captured calls bring their own workspace
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return CQR_ERR_HIP;
    std::lock_guard<std::mutex> lk(g_mu);
    DevState &d = g_dev[dev];
    if (!d.info) {
      if (cap) return CQR_ERR_ARG;  // the first call on a device allocates
      if (hipMalloc(&d.info, kAlign) != hipSuccess) return CQR_ERR_NOMEM;
    }
    if (!ws) {
      if (ensure_buffer(d, d.ws, (size_t)lay.total, s) != hipSuccess) {
        (void)hipGetLastError();  // no room for the staging copy: factor in place
        lay = plain;
        if (ensure_buffer(d, d.ws, (size_t)lay.total, s) != hipSuccess) return CQR_ERR_NOMEM;
      }
      ws = (char *)d.ws.p;
      lib_state = &d;
    }
    if (!info) info = d.info;
  }

  Run r{};
  r.s = s;
  r.info = info;
  r.m = m;
  r.n = n;
  r.W = (double *)(ws + lay.w);
  r.Uinv = (double *)(ws + lay.uinv);
  r.Ua = (double *)(ws + lay.ua);
  r.Ub = (double *)(ws + lay.ub);
  r.G = lay.g >= 0 ? (double *)(ws + lay.g) : nullptr;
  r.Y = (double *)(ws + lay.y);
  r.part = (double *)(ws + lay.part);
  r.part_elems = lay.part_elems;
  r.R1 = lay.r1 >= 0 ? (double *)(ws + lay.r1) : nullptr;
  r.R2 = lay.r2 >= 0 ? (double *)(ws + lay.r2) : nullptr;
  r.Yz = lay.yz >= 0 ? (double *)(ws + lay.yz) : nullptr;
  r.zskip = (int *)(ws + lay.flags);
  r.cskip = r.zskip + 1;
  r.adaptive = (opt && opt->adaptive && schedule == CQR_SCHED_MOD) ? CQR_ADAPTIVE_TOL : 0.0;
  r.upd_tile = opt ? opt->update_tile : CQR_TILE_AUTO;
  r.proj_tile = opt ? opt->proj_tile : CQR_TILE_AUTO;
  std::unique_lock<std::mutex> side_lock;
  if (opt && opt->lookahead && schedule == CQR_SCHED_MOD && r.Yz && be < n) {
    DevState *ds = nullptr;
    if (side_stream(&ds) != hipSuccess) return CQR_ERR_HIP;
    side_lock = std::unique_lock<std::mutex>(ds->side);
    r.aux = ds->aux;
    r.fork = ds->fork;
    r.join = ds->join;
  }

  if (timed(s, CQR_K_SMALL, 0, 0, [&] { return cqr::launch_set_int(info, 0, s); }) != hipSuccess)
    return CQR_ERR_HIP;
  hipError_t e;
  if (lay.stage >= 0) {
    // factor in the staging copy; each panel's final Q_j goes to both copies
    double *S = (double *)(ws + lay.stage);
    const int64_t ldw = lay.ldw;
    r.Qout = Q;
    r.ldq = lda;
    e = timed(s, CQR_K_COPY, 0, 16.0 * m * n,
              [&] { return cqr::launch_copy_cols(m, n, A, lda, S, ldw, s); });
    if (e == hipSuccess) e = run_schedule(r, schedule, S, S, ldw, be, R);
  } else {
    e = run_schedule(r, schedule, A, Q, lda, be, R);
  }
  if (e == hipSuccess && lib_state) {
    std::lock_guard<std::mutex> lk(g_mu);
    e = mark_use(*lib_state, s);
  }
  return e == hipSuccess ? CQR_OK : CQR_ERR_HIP;
}

int cqr_factor(int64_t m, int64_t n, int64_t b, const double *A, int64_t lda, double *Q,
               double *R, void *stream) {
  return cqr_factor_ex(m, n, b, A, lda, Q, R, stream, nullptr);
}

}  // extern "C"

// ---------------------------------------------------------------- no-allocation scratch
// The workspace of cqr_factor_noalloc: a fixed array in the library's device
// code, one copy per device, created when the code is loaded on that device
// and held until the process ends. In host code `scratch` names a host-side
// stand-in, not device memory: host code uses only the device address
// hipGetSymbolAddress returns for the current device (g_scratch).
static __device__ __align__(256) char scratch[CQR_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
void *g_scratch[kMaxDevices];  // device address of `scratch` per device (null until set up)
std::mutex g_scratch_mu;

// The current device's address of `scratch`, looked up on its first use.
hipError_t scratch_address(void **out) {
  int dev = 0;
  CQR_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch[dev]) {
    void *p = nullptr;
    CQR_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return hipErrorInvalidSymbol;
    g_scratch[dev] = p;
  }
  *out = g_scratch[dev];
  return hipSuccess;
}
}  // namespace

extern "C" {

int cqr_factor_noalloc(int64_t m, int64_t n, int64_t b, const double *A, int64_t lda, double *Q,
                       double *R, int schedule, int *d_info, void *stream) {
  const int st = check_args(m, n, b, A, lda, Q, R, schedule);
  if (st != CQR_OK) return st;
  if (!d_info || misaligned(d_info, 4)) return CQR_ERR_ARG;
  // the in-place layout only: a staging copy of an aliasing lda would need
  // lda * n more doubles
  const Layout plain = make_layout(m, n, effective_panel(m, n, b, schedule), schedule, false);
  if ((size_t)plain.total > (size_t)CQR_NOALLOC_SCRATCH_BYTES) return CQR_ERR_WORKSPACE;
  void *ws = nullptr;
  if (scratch_address(&ws) != hipSuccess) return CQR_ERR_HIP;
  cqr_options opt{};
  opt.schedule = schedule;
  opt.d_info = d_info;
  opt.workspace = ws;
  opt.workspace_bytes = (size_t)plain.total;
  t_no_events = true;
  const int rc = cqr_factor_ex(m, n, b, A, lda, Q, R, stream, &opt);
  t_no_events = false;
  return rc;
}

int cqr_get_info(void *stream, int *info) {
  if (!info) return CQR_ERR_ARG;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return CQR_ERR_HIP;
  int *d = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_dev.find(dev);
    if (it == g_dev.end() || !it->second.info) {
      *info = 0;
      return CQR_OK;
    }
    d = it->second.info;
  }
  if (hipStreamSynchronize((hipStream_t)stream) != hipSuccess) return CQR_ERR_HIP;
  if (hipMemcpy(info, d, sizeof(int), hipMemcpyDeviceToHost) != hipSuccess) return CQR_ERR_HIP;
  return CQR_OK;
}

const char *cqr_status_string(int status) {
  switch (status) {
    case CQR_OK: return "success";
    case CQR_ERR_ARG: return "invalid argument";
    case CQR_ERR_HIP: return "HIP runtime or launch failure";
    case CQR_ERR_NOMEM: return "device allocation failed";
    case CQR_ERR_WORKSPACE: return "workspace too small";
    case CQR_ERR_UNSUPPORTED: return "size not supported by this build";
    default: return "unknown status";
  }
}

int cqr_profile_enable(int on) {
  std::lock_guard<std::mutex> lk(g_mu);
  g_prof = on != 0;
  return CQR_OK;
}

int cqr_profile_select(unsigned kind_mask) {
  std::lock_guard<std::mutex> lk(g_mu);
  g_prof_mask = kind_mask;
  return CQR_OK;
}

int cqr_profile_reset(void) {
  std::lock_guard<std::mutex> lk(g_mu);
  int st = CQR_OK;
  for (auto &rec : g_recs) {
    if (hipEventSynchronize(rec.b) != hipSuccess) st = CQR_ERR_HIP;
    g_pool.push_back(rec.a);
    g_pool.push_back(rec.b);
  }
  g_recs.clear();
  for (auto &a : g_acc) a = Acc{};
  return st;
}

int cqr_profile_query(int kind, int64_t *launches, double *ms, double *flops, double *bytes) {
  if (kind < 0 || kind >= CQR_K_COUNT) return CQR_ERR_ARG;
  std::lock_guard<std::mutex> lk(g_mu);
  for (auto &rec : g_recs) {
    if (hipEventSynchronize(rec.b) != hipSuccess) return CQR_ERR_HIP;
    float t = 0.f;
    if (hipEventElapsedTime(&t, rec.a, rec.b) != hipSuccess) return CQR_ERR_HIP;
    Acc &a = g_acc[rec.kind];
    a.n += 1;
    a.ms += t;
    a.flops += rec.flops;
    a.bytes += rec.bytes;
    g_pool.push_back(rec.a);
    g_pool.push_back(rec.b);
  }
  g_recs.clear();
  const Acc &a = g_acc[kind];
  if (launches) *launches = a.n;
  if (ms) *ms = a.ms;
  if (flops) *flops = a.flops;
  if (bytes) *bytes = a.bytes;
  return CQR_OK;
}

size_t cqr_backward_workspace_bytes(int64_t m, int64_t n, int64_t batch) {
  if (batch < 1 || n < 1 || m < n) return 0;
  return (size_t)make_bwd_layout(m, n, batch).total;
}

int cqr_backward_batched(int64_t batch, int64_t m, int64_t n, const double *Q, const double *A,
                         int64_t lda, int64_t stride, const double *R, const double *dQ,
                         const double *dR, double *dA, void *stream, void *workspace,
                         size_t workspace_bytes) {
  const int st = check_bwd(batch, m, n, Q, A, lda, stride, R, dQ, dR, dA);
  if (st != CQR_OK) return st;
  if (batch == 1) stride = lda * n;
  const BwdLayout lay = make_bwd_layout(m, n, batch);
  hipStream_t s = (hipStream_t)stream;
  char *ws = (char *)workspace;
  DevState *lib_state = nullptr;  // set when the library's workspace is used
  if (ws) {
    if (workspace_bytes < (size_t)lay.total) return CQR_ERR_WORKSPACE;
    if (misaligned(ws, kAlign)) return CQR_ERR_ARG;
  } else {
    if (capturing(s)) return CQR_ERR_ARG;  // captured calls bring their own workspace
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return CQR_ERR_HIP;
    std::lock_guard<std::mutex> lk(g_mu);
    DevState &d = g_dev[dev];
    if (ensure_buffer(d, d.bwd, (size_t)lay.total, s) != hipSuccess) return CQR_ERR_NOMEM;
    ws = (char *)d.bwd.p;
    lib_state = &d;
  }
  int *info = (int *)(ws + lay.info);
  double *part = (double *)(ws + lay.part), *T = (double *)(ws + lay.t);
  double *Rinv = (double *)(ws + lay.rinv), *RinvT = (double *)(ws + lay.rinvt);
  double *C = (double *)(ws + lay.c), *G = (double *)(ws + lay.g);
  double *Y = (double *)(ws + lay.y);
  const int ni = (int)n, b = (int)batch;
  const int64_t nn = n * n, sy = 2 * n * lay.ldy;
  const bool recompute = (Q == nullptr);
  const double *S = recompute ? A : Q;
  const double mf = (double)m, nf = (double)n, bf = (double)batch;
  auto fail = [&](hipError_t e) {
    if (e == hipSuccess && lib_state) {
      std::lock_guard<std::mutex> lk(g_mu);
      e = mark_use(*lib_state, s);
    }
    return e == hipSuccess ? CQR_OK : CQR_ERR_HIP;
  };

  if (!dQ && !dR)
    return fail(timed(s, CQR_K_SMALL, 0, 8.0 * bf * mf * nf,
                      [&] { return cqr::launch_zero2d(dA, m, n, lda, stride, b, s); }));
  hipError_t e = cqr::launch_set_int(info, 0, s);
  if (e != hipSuccess) return CQR_ERR_HIP;
  // R^{-1} and R^{-T} need only R: they run on the side stream while pass 1
  // streams over the rows, and are joined back before the n x n step (the
  // inverse's waves use few registers, so they share SIMDs with pass 1's)
  DevState *dev_state = nullptr;
  if (side_stream(&dev_state) != hipSuccess) return CQR_ERR_HIP;
  std::lock_guard<std::mutex> side_lock(dev_state->side);
  hipStream_t aux = dev_state->aux;
  if (hipEventRecord(dev_state->fork, s) != hipSuccess ||
      hipStreamWaitEvent(aux, dev_state->fork, 0) != hipSuccess)
    return CQR_ERR_HIP;
  e = timed(aux, CQR_K_CHOL, bf * nf * nf * nf / 3.0, 16.0 * bf * nn,
            [&] { return cqr::launch_tri_inv(R, ni, nn, Rinv, nn, b, aux, RinvT); });
  if (e != hipSuccess) return CQR_ERR_HIP;
  if (hipEventRecord(dev_state->join, aux) != hipSuccess) return CQR_ERR_HIP;
  // pass 1: T = S^T dQ (upper 64x64 tiles), split over m, fixed-order reduce
  if (dQ) {
    const bool upper = true;
    e = timed(s, CQR_K_PROJ, bf * mf * nf * nf, 16.0 * bf * mf * nf, [&] {
      return cqr::launch_tn(upper, m, ni, ni, S, lda, dQ, lda, part, lay.rc, lay.nch, info, s, b,
                            stride, stride, lay.nch * nn);
    });
    if (e != hipSuccess) return CQR_ERR_HIP;
    e = timed(s, CQR_K_REDUCE, bf * lay.nch * nn, 8.0 * bf * (lay.nch + 1) * nn, [&] {
      return cqr::launch_reduce(upper, part, lay.nch, ni, ni, T, n, nullptr, 0, false, info, s, b,
                                lay.nch * nn, nn, 0);
    });
    if (e != hipSuccess) return CQR_ERR_HIP;
  }
  // n x n part: C = copyltu(M), the stacked right operand (after R^{-1})
  if (hipStreamWaitEvent(s, dev_state->join, 0) != hipSuccess) return CQR_ERR_HIP;
  e = timed(s, CQR_K_SMALL, bf * 2.0 * nf * nf * nf, 8.0 * bf * 6 * nn, [&] {
    return cqr::launch_adj_small(ni, T, nn, R, dR, nn, Rinv, RinvT, nn, dQ ? 1 : 0, recompute ? 1 : 0, C, G,
                                 nn, Y, lay.ldy, sy, dQ ? 1 : 0, b, s);
  });
  if (e != hipSuccess) return CQR_ERR_HIP;
  // pass 2: dA = [dQ | S] [R^{-T}; G]   (or S G when dQ is absent)
  if (dQ) {
    e = timed(s, CQR_K_UPDATE, bf * 4.0 * mf * nf * nf, 24.0 * bf * mf * nf, [&] {
      // Y's upper block is R^{-T}: lower triangular
      return cqr::launch_nn(false, false, m, 2 * ni, ni, dQ, lda, Y, lay.ldy, nullptr, 0, dA, lda,
                            info, s, S, lda, ni, b, stride, stride, sy, 0, stride, nullptr, 0,
                            nullptr, cqr::kTileAuto, true);
    });
  } else {
    e = timed(s, CQR_K_UPDATE, bf * 2.0 * mf * nf * nf, 16.0 * bf * mf * nf, [&] {
      return cqr::launch_nn(false, false, m, ni, ni, S, lda, Y, lay.ldy, nullptr, 0, dA, lda, info,
                            s, nullptr, 0, 0, b, stride, 0, sy, 0, stride);
    });
  }
  return fail(e);
}

int cqr_backward(int64_t m, int64_t n, const double *Q, const double *A, int64_t lda,
                 const double *R, const double *dQ, const double *dR, double *dA, void *stream,
                 void *workspace, size_t workspace_bytes) {
  return cqr_backward_batched(1, m, n, Q, A, lda, lda * n, R, dQ, dR, dA, stream, workspace,
                              workspace_bytes);
}

// ---------------------------------------------------------------- batched
}  // extern "C"

struct cqr_batch_plan {
  int64_t count = 0;
  int device = 0;
  int grid = 0;
  int nslots = 0, nteams = 0;
  void *mem = nullptr;  // slots | m | n | b | queue | team counters | team partials
  cqr::BatchSlot *slots = nullptr;
  int64_t *m = nullptr;
  int *n = nullptr;
  int *b = nullptr;
  int *queue = nullptr;
  int *team_cnt = nullptr;
  double *team_part = nullptr;
  double flops = 0, bytes = 0;
};

extern "C" {

int cqr_plan_batched(int64_t batch, const int64_t *h_m, const int64_t *h_n, const int64_t *h_b,
                     int schedule, cqr_batch_plan **plan) {
  if (!plan) return CQR_ERR_ARG;
  *plan = nullptr;
  if (batch < 1 || batch > (int64_t(1) << 30) || !h_m || !h_n) return CQR_ERR_ARG;
  if (!valid_schedule(schedule)) return CQR_ERR_ARG;
  if (schedule != CQR_SCHED_MOD) return CQR_ERR_UNSUPPORTED;
  std::vector<int64_t> m(h_m, h_m + batch);
  std::vector<int> n(batch), b(batch);
  double flops = 0, bytes = 0;
  for (int64_t i = 0; i < batch; ++i) {
    if (h_n[i] < 1 || m[i] < h_n[i]) return CQR_ERR_ARG;
    if (m[i] > (int64_t(1) << 33)) return CQR_ERR_UNSUPPORTED;  // the kernel counts rows in 32 bits
    const int64_t bi = h_b ? h_b[i] : 0;
    if (bi < 0) return CQR_ERR_ARG;
    // default: two or more panels, at most kBatchMaxPanel wide (a single panel
    // is plain CholeskyQR2, which breaks down for kappa beyond about 1e8)
    const int64_t bdef = std::min<int64_t>((h_n[i] + 1) / 2, cqr::kBatchMaxPanel);
    const int64_t be = std::min<int64_t>(bi == 0 ? bdef : bi, h_n[i]);
    if (h_n[i] > cqr::kBatchMaxN || be > cqr::kBatchMaxPanel) return CQR_ERR_UNSUPPORTED;
    n[i] = (int)h_n[i];
    b[i] = (int)be;
    const double mf = (double)m[i], nf = n[i];
    flops += 2.0 * mf * nf * nf - 2.0 * nf * nf * nf / 3.0;  // Householder-equivalent
    bytes += 24.0 * mf * nf + 24.0 * mf * nf * nf / be;
  }
  int cus = 0, dev = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return CQR_ERR_HIP;
  const int64_t resident = std::max<int64_t>(1, (int64_t)cus * cqr::batched_blocks_per_cu());
  // Teams: a matrix whose work exceeds a resident workgroup's fair share is
  // split by rows over up to kBatchMaxTeam workgroups (at least 2048 rows
  // each), so that no single matrix sets the makespan. The kernel streams
  // its matrices from memory, so work is priced by the bytes it moves (~ m n
  // (1 + n / b)) plus a per-panel fixed cost (the n / b small Cholesky steps
  // and workgroup barriers, about 2048 n rows' worth each), not by flops.
  std::vector<double> work(batch);
  double total = 0;
  for (int64_t i = 0; i < batch; ++i)
    total += (work[i] = (double)m[i] * n[i] * (1.0 + (double)n[i] / b[i]) +
                        2048.0 * n[i] * n[i] / b[i]);
  // (the share is taken over every resident workgroup, so a batch of fewer
  // matrices than workgroups still splits its largest matrices)
  const double share = total / (double)resident;
  // A batch of at most one matrix per eight resident workgroups is a latency
  // problem rather than a throughput one: every matrix is split over as many
  // row shares of at least kTeamMinRows rows as the idle workgroups allow
  // (up to kBatchMaxTeamSmall), trading team barriers for parallel streams
  // (one 4096 x 64 matrix: 1.25 -> 0.47 ms; 16 of 32768 x 128: 20 -> 5 ms).
  std::vector<int> team(batch, 1);
  const bool small_batch = batch * 8 <= resident;
  for (int64_t i = 0; i < batch; ++i) {
    int64_t t;
    if (small_batch) {
      t = std::min<int64_t>({resident / batch, std::max<int64_t>(1, m[i] / cqr::kTeamMinRows),
                             (int64_t)cqr::kBatchMaxTeamSmall});
    } else {
      t = (int64_t)std::ceil(work[i] / share - 1e-9);
      t = std::min<int64_t>({std::max<int64_t>(t, 1), (int64_t)cqr::kBatchMaxTeam, resident,
                             std::max<int64_t>(1, m[i] / 2048)});
    }
    team[i] = (int)t;
  }
  // longest processing time first: per-member work, ties by index
  std::vector<int> order(batch);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(),
                   [&](int x, int y) { return work[x] / team[x] > work[y] / team[y]; });
  std::vector<cqr::BatchSlot> slots;
  int64_t nteams = 0, part_doubles = 0;
  for (int i : order) {
    const int t = team[i];
    const int ci = (t > 1) ? (int)nteams++ : 0;
    const int64_t po = (t > 1) ? part_doubles : 0;
    if (t > 1) part_doubles += 2LL * t * cqr::kTeamSlot;
    for (int k = 0; k < t; ++k) slots.push_back({i, k, t, ci, po});
  }
  const int64_t nslots = (int64_t)slots.size();
  cqr_batch_plan *pl = new cqr_batch_plan();
  pl->count = batch;
  pl->device = dev;
  pl->nslots = (int)nslots;
  pl->nteams = (int)nteams;
  const size_t ss = round_up(sizeof(cqr::BatchSlot) * nslots, kAlign), sm = round_up(8 * batch, kAlign);
  const size_t sn = round_up(4 * batch, kAlign), sb = round_up(4 * batch, kAlign);
  const size_t sq = kAlign, sc = round_up(4 * std::max<int64_t>(nteams, 1), kAlign);
  const size_t sp = round_up(8 * std::max<int64_t>(part_doubles, 1), kAlign);
  if (hipMalloc(&pl->mem, ss + sm + sn + sb + sq + sc + sp) != hipSuccess) {
    delete pl;
    return CQR_ERR_NOMEM;
  }
  char *base = (char *)pl->mem;
  pl->slots = (cqr::BatchSlot *)base;
  pl->m = (int64_t *)(base + ss);
  pl->n = (int *)(base + ss + sm);
  pl->b = (int *)(base + ss + sm + sn);
  pl->queue = (int *)(base + ss + sm + sn + sb);
  pl->team_cnt = (int *)(base + ss + sm + sn + sb + sq);
  pl->team_part = (double *)(base + ss + sm + sn + sb + sq + sc);
  const bool ok =
      hipMemcpy(pl->slots, slots.data(), sizeof(cqr::BatchSlot) * nslots, hipMemcpyHostToDevice) ==
          hipSuccess &&
      hipMemcpy(pl->m, m.data(), 8 * batch, hipMemcpyHostToDevice) == hipSuccess &&
      hipMemcpy(pl->n, n.data(), 4 * batch, hipMemcpyHostToDevice) == hipSuccess &&
      hipMemcpy(pl->b, b.data(), 4 * batch, hipMemcpyHostToDevice) == hipSuccess &&
      hipMemset(pl->queue, 0, sizeof(int)) == hipSuccess;
  if (!ok) {
    (void)hipFree(pl->mem);
    delete pl;
    return CQR_ERR_HIP;
  }
  // every workgroup of the grid is resident at once, so team members that
  // wait for each other always find their partners running
  pl->grid = (int)std::min<int64_t>(nslots, resident);
  pl->flops = flops;
  pl->bytes = bytes;
  *plan = pl;
  return CQR_OK;
}

int cqr_factor_batched(const cqr_batch_plan *plan, const double *const *d_A, const int64_t *d_lda,
                       double *const *d_Q, double *const *d_R, int *d_info, void *stream) {
  if (!plan || !d_A || !d_lda || !d_Q || !d_R || !d_info) return CQR_ERR_ARG;
  hipStream_t s = (hipStream_t)stream;
  const hipError_t e = timed(s, CQR_K_BATCHED, plan->flops, plan->bytes, [&] {
    return cqr::launch_batched_mod(plan->grid, plan->slots, plan->nslots, plan->m, plan->n,
                                   plan->b, d_A, d_lda, d_Q, d_R, d_info, plan->queue,
                                   plan->team_part, plan->team_cnt, plan->nteams, s);
  });
  return e == hipSuccess ? CQR_OK : CQR_ERR_HIP;
}

void cqr_plan_destroy(cqr_batch_plan *plan) {
  if (!plan) return;
  if (plan->mem) (void)hipFree(plan->mem);
  delete plan;
}

}  // extern "C"
