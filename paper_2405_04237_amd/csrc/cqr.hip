// libcqr host library: the C ABI of include/cqr.h.
//
// Argument checks, workspace layout, the split-m plan, and the two panel
// schedules of arXiv 2405.04237 as stream-ordered kernel chains:
//   CQR2GS  (Algorithm 7 = Algorithm 6/8 twice, then R = R2 R1)
//   mCQR2GS (Algorithm 9)
// Nothing here synchronises with the device except cqr_get_info and
// cqr_profile_query.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <vector>

#include "cqr.h"
#include "kernels.h"

namespace {

using cqr::kMaxPanel;

constexpr int64_t kAlign = 256;
constexpr int64_t kPartChunks = 256;   // split-m partial capacity, in units of n*b doubles
constexpr int64_t kTargetWaves = 2048; // split-m grid size aimed for (8 waves per CU)
constexpr int64_t kMaxChunkRows = 16384;

int64_t round_up(int64_t x, int64_t a) { return (x + a - 1) / a * a; }

// ---------------------------------------------------------------- workspace
struct Layout {
  int64_t w, uinv, ua, ub, y, part, r1, r2, total;  // byte offsets / size
  int64_t part_elems;
};

Layout make_layout(int64_t n, int64_t b, int schedule) {
  Layout L{};
  int64_t off = 0;
  auto take = [&](int64_t elems) {
    const int64_t o = off;
    off = round_up(off + elems * 8, kAlign);
    return o;
  };
  L.w = take(b * b);
  L.uinv = take(b * cqr::padded_ld(b));
  L.ua = take(b * b);
  L.ub = take(b * b);
  L.y = take(n * cqr::padded_ld(std::max(n, b)));
  L.part_elems = kPartChunks * std::max(n * b, b * b);
  L.part = take(L.part_elems);
  if (schedule == CQR_SCHED_ORIG) {
    L.r1 = take(n * n);
    L.r2 = take(n * n);
  } else {
    L.r1 = L.r2 = -1;
  }
  L.total = off;
  return L;
}

int64_t effective_panel(int64_t m, int64_t n, int64_t b, int schedule) {
  if (b == 0) b = cqr_default_panel(m, n, schedule);
  return std::min(b, n);
}

// ---------------------------------------------------------------- per device
struct DevState {
  void *ws = nullptr;
  size_t ws_bytes = 0;
  int *info = nullptr;
};
std::mutex g_mu;
std::map<int, DevState> g_dev;

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
  if (!g_prof) return f();
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
  int *info;
  int64_t m, n;
  double *W, *Uinv, *Ua, *Ub, *Y, *part, *R1, *R2;
  int64_t part_elems;
};

void plan_chunks(const Run &r, int64_t tiles, int64_t pq, int64_t *rc, int64_t *nch) {
  const int64_t cap = std::max<int64_t>(1, r.part_elems / std::max<int64_t>(1, pq));
  int64_t want = (kTargetWaves + tiles - 1) / tiles;
  want = std::max(want, (r.m + kMaxChunkRows - 1) / kMaxChunkRows);
  want = std::min({want, cap, (r.m + 15) / 16, int64_t(4096)});
  want = std::max<int64_t>(want, 1);
  int64_t rows = round_up((r.m + want - 1) / want, 16);
  *rc = rows;
  *nch = (r.m + rows - 1) / rows;
}

#define CQR_TRY(expr)                    \
  do {                                   \
    const hipError_t e_ = (expr);        \
    if (e_ != hipSuccess) return e_;     \
  } while (0)

// W = X^T X for the w columns at X (split-m partials + fixed-order reduce)
hipError_t step_gram(Run &r, const double *X, int64_t ldx, int w) {
  int64_t rc, nch;
  const int64_t tiles = cqr::tn_tiles(true, w, w);
  plan_chunks(r, tiles, (int64_t)w * w, &rc, &nch);
  CQR_TRY(timed(r.s, CQR_K_GRAM, double(r.m) * w * w, 8.0 * r.m * w, [&] {
    return cqr::launch_tn(true, r.m, w, w, X, ldx, X, ldx, r.part, rc, nch, r.info, r.s);
  }));
  return timed(r.s, CQR_K_REDUCE, double(nch) * w * w, 8.0 * (nch + 1) * w * w, [&] {
    return cqr::launch_reduce(true, r.part, nch, w, w, r.W, w, nullptr, 0, false, r.info, r.s);
  });
}

// U = chol(W), Uinv = U^{-1}; U optionally to uout (row-major) and/or the R block
hipError_t step_chol(Run &r, int w, double *uout, double *rblk, int64_t ldr, int col0) {
  const double wf = w;
  return timed(r.s, CQR_K_CHOL, 2.0 * wf * wf * wf / 3.0, 8.0 * 4 * wf * wf, [&] {
    return cqr::launch_chol_inv(r.W, w, uout, rblk, ldr, r.Uinv, r.info, col0, r.s);
  });
}

// X = X U^{-1} in place (the Q_j := A_j U^{-1} step)
hipError_t step_trsm(Run &r, double *X, int64_t ldx, int w) {
  return timed(r.s, CQR_K_TRSM, double(r.m) * w * w, 16.0 * r.m * w, [&] {
    return cqr::launch_nn(false, true, r.m, w, w, X, ldx, r.Uinv, cqr::padded_ld(w), X, ldx, r.info,
                          r.s);
  });
}

// Y = Qp^T Z: -Y row-major in r.Y (the update's operand), +Y into the R block if given
hipError_t step_proj(Run &r, const double *Qp, int64_t ld, int p, const double *Z, int q,
                     double *rblk, int64_t ldr) {
  int64_t rc, nch;
  const int64_t tiles = cqr::tn_tiles(false, p, q);
  plan_chunks(r, tiles, (int64_t)p * q, &rc, &nch);
  CQR_TRY(timed(r.s, CQR_K_PROJ, 2.0 * r.m * p * q, 8.0 * r.m * (p + q), [&] {
    return cqr::launch_tn(false, r.m, p, q, Qp, ld, Z, ld, r.part, rc, nch, r.info, r.s);
  }));
  return timed(r.s, CQR_K_REDUCE, double(nch) * p * q, 8.0 * (nch + 1) * p * q, [&] {
    return cqr::launch_reduce(false, r.part, nch, p, q, r.Y, cqr::padded_ld(q), rblk, ldr, true,
                              r.info, r.s);
  });
}

// Z -= Qp Y  (r.Y holds -Y)
hipError_t step_update(Run &r, const double *Qp, int64_t ld, int p, double *Z, int q) {
  return timed(r.s, CQR_K_UPDATE, 2.0 * r.m * p * q, 8.0 * r.m * (p + 2.0 * q), [&] {
    return cqr::launch_nn(true, false, r.m, p, q, Qp, ld, r.Y, cqr::padded_ld(q), Z, ld, r.info, r.s);
  });
}

// One CQRGS pass (Algorithm 6; Algorithm 8 with the Allreduces replaced by
// split-m reductions) in place on X, writing its R into Rd (n x n, ld n).
hipError_t pass_cqrgs(Run &r, double *X, int64_t ld, int64_t b, double *Rd) {
  const int64_t n = r.n;
  for (int64_t s = 0; s < n; s += b) {
    const int64_t e = std::min(n, s + b);
    const int w = (int)(e - s);
    double *Xj = X + s * ld;
    CQR_TRY(step_gram(r, Xj, ld, w));                          // W_j := A_j^T A_j
    CQR_TRY(step_chol(r, w, nullptr, Rd + s + s * n, n, (int)s));  // W_j = U^T U; R_jj := U
    CQR_TRY(step_trsm(r, Xj, ld, w));                          // Q_j := A_j U^{-1}
    if (e < n) {
      CQR_TRY(step_proj(r, Xj, ld, w, X + e * ld, (int)(n - e), Rd + s + e * n, n));  // Y; R_{j,j+1:k}
      CQR_TRY(step_update(r, Xj, ld, w, X + e * ld, (int)(n - e)));                   // A_{j+1:k} -= Q_j Y
    }
  }
  return hipSuccess;
}

hipError_t run_orig(Run &r, double *Q, int64_t ld, int64_t b, double *R) {
  const int64_t n = r.n;
  CQR_TRY(timed(r.s, CQR_K_SMALL, 0, 16.0 * n * n, [&] { return cqr::launch_zero(r.R1, n * n, r.s); }));
  CQR_TRY(timed(r.s, CQR_K_SMALL, 0, 16.0 * n * n, [&] { return cqr::launch_zero(r.R2, n * n, r.s); }));
  CQR_TRY(pass_cqrgs(r, Q, ld, b, r.R1));  // [Q1, R1] = CQRGS(A)
  CQR_TRY(pass_cqrgs(r, Q, ld, b, r.R2));  // [Q, R2]  = CQRGS(Q1)
  const double nf = n;
  return timed(r.s, CQR_K_SMALL, nf * nf * nf / 3.0, 24.0 * nf * nf, [&] {
    return cqr::launch_trmm_upper((int)n, r.R2, r.R1, R, r.info, r.s);  // R = R2 R1
  });
}

hipError_t run_mod(Run &r, double *Q, int64_t ld, int64_t b, double *R) {
  const int64_t n = r.n;
  CQR_TRY(timed(r.s, CQR_K_SMALL, 0, 8.0 * n * n, [&] { return cqr::launch_zero(R, n * n, r.s); }));
  // first panel: CholeskyQR2
  {
    const int w = (int)std::min(n, b);
    CQR_TRY(step_gram(r, Q, ld, w));
    CQR_TRY(step_chol(r, w, r.Ua, nullptr, 0, 0));
    CQR_TRY(step_trsm(r, Q, ld, w));
    CQR_TRY(step_gram(r, Q, ld, w));
    CQR_TRY(step_chol(r, w, r.Ub, nullptr, 0, 0));
    CQR_TRY(step_trsm(r, Q, ld, w));
    CQR_TRY(timed(r.s, CQR_K_SMALL, 0, 0, [&] {
      return cqr::launch_r_upper_product(w, r.Ub, r.Ua, R, n, r.info, r.s);  // R_11 = R2 R1
    }));
  }
  for (int64_t s = b; s < n; s += b) {
    const int64_t ps = s - b, e = std::min(n, s + b);
    const int w = (int)(e - s), pw = (int)b;
    double *Qprev = Q + ps * ld, *Xj = Q + s * ld;
    // Y := Q_{j-1}^T A_{:,j:k}; R_{j-1,j:k} := Y; A_{:,j:k} -= Q_{j-1} Y
    CQR_TRY(step_proj(r, Qprev, ld, pw, Xj, (int)(n - s), R + ps + s * n, n));
    CQR_TRY(step_update(r, Qprev, ld, pw, Xj, (int)(n - s)));
    // CQR(A_j): A_j = Qt Ua
    CQR_TRY(step_gram(r, Xj, ld, w));
    CQR_TRY(step_chol(r, w, r.Ua, nullptr, 0, (int)s));
    CQR_TRY(step_trsm(r, Xj, ld, w));
    // re-orthogonalise: Z := Q_{1:j-1}^T Qt; Qt -= Q_{1:j-1} Z; R_{1:j-1,j} += Z Ua
    // (r.Y holds -Z, so the R update subtracts (-Z) Ua)
    CQR_TRY(step_proj(r, Q, ld, (int)s, Xj, w, nullptr, 0));
    CQR_TRY(step_update(r, Q, ld, (int)s, Xj, w));
    CQR_TRY(timed(r.s, CQR_K_SMALL, 2.0 * s * w * w / 2, 0, [&] {
      return cqr::launch_r_add_zu((int)s, w, r.Y, cqr::padded_ld(w), r.Ua, R + s * n, n, r.info, r.s);
    }));
    // CQR again: Qt = Q_j Ub; R_jj = Ub Ua
    CQR_TRY(step_gram(r, Xj, ld, w));
    CQR_TRY(step_chol(r, w, r.Ub, nullptr, 0, (int)s));
    CQR_TRY(step_trsm(r, Xj, ld, w));
    CQR_TRY(timed(r.s, CQR_K_SMALL, 0, 0, [&] {
      return cqr::launch_r_upper_product(w, r.Ub, r.Ua, R + s + s * n, n, r.info, r.s);
    }));
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
  if (schedule != CQR_SCHED_MOD && schedule != CQR_SCHED_ORIG) return CQR_ERR_ARG;
  if (effective_panel(m, n, b, schedule) > kMaxPanel) return CQR_ERR_UNSUPPORTED;
  return CQR_OK;
}

}  // namespace

extern "C" {

int64_t cqr_default_panel(int64_t m, int64_t n, int schedule) {
  (void)m;
  if (n <= 0) return 0;
  // mCQR2GS keeps O(u) orthogonality at kappa = 1e15 with a handful of
  // panels (the paper uses three); CQR2GS needs narrower panels there.
  const int64_t parts = (schedule == CQR_SCHED_ORIG) ? 16 : 4;
  int64_t b = round_up((n + parts - 1) / parts, 16);
  b = std::max<int64_t>(16, std::min<int64_t>(b, schedule == CQR_SCHED_ORIG ? 64 : kMaxPanel));
  return std::min(b, n);
}

size_t cqr_workspace_bytes(int64_t m, int64_t n, int64_t b, int schedule) {
  if (n < 1 || m < n || b < 0) return 0;
  if (schedule != CQR_SCHED_MOD && schedule != CQR_SCHED_ORIG) return 0;
  const int64_t be = effective_panel(m, n, b, schedule);
  return (size_t)make_layout(n, be, schedule).total;
}

int cqr_factor_ex(int64_t m, int64_t n, int64_t b, const double *A, int64_t lda, double *Q,
                  double *R, void *stream, const cqr_options *opt) {
  const int schedule = opt ? opt->schedule : CQR_SCHED_MOD;
  const int st = check_args(m, n, b, A, lda, Q, R, schedule);
  if (st != CQR_OK) return st;
  const int64_t be = effective_panel(m, n, b, schedule);
  const Layout lay = make_layout(n, be, schedule);
  hipStream_t s = (hipStream_t)stream;

  char *ws = nullptr;
  int *info = opt ? opt->d_info : nullptr;
  if (opt && opt->workspace) {
    if (opt->workspace_bytes < (size_t)lay.total) return CQR_ERR_WORKSPACE;
    if (misaligned(opt->workspace, kAlign)) return CQR_ERR_ARG;
    ws = (char *)opt->workspace;
  }
  if (!ws || !info) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return CQR_ERR_HIP;
    std::lock_guard<std::mutex> lk(g_mu);
    DevState &d = g_dev[dev];
    if (!d.info) {
      if (hipMalloc(&d.info, kAlign) != hipSuccess) return CQR_ERR_NOMEM;
      if (hipMemset(d.info, 0, kAlign) != hipSuccess) return CQR_ERR_HIP;
    }
    if (!ws && d.ws_bytes < (size_t)lay.total) {
      // the stream may still use the old buffer: wait for the device first
      if (d.ws) {
        if (hipDeviceSynchronize() != hipSuccess) return CQR_ERR_HIP;
        if (hipFree(d.ws) != hipSuccess) return CQR_ERR_HIP;
        d.ws = nullptr;
        d.ws_bytes = 0;
      }
      if (hipMalloc(&d.ws, (size_t)lay.total) != hipSuccess) return CQR_ERR_NOMEM;
      d.ws_bytes = (size_t)lay.total;
    }
    if (!ws) ws = (char *)d.ws;
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
  r.Y = (double *)(ws + lay.y);
  r.part = (double *)(ws + lay.part);
  r.part_elems = lay.part_elems;
  r.R1 = lay.r1 >= 0 ? (double *)(ws + lay.r1) : nullptr;
  r.R2 = lay.r2 >= 0 ? (double *)(ws + lay.r2) : nullptr;

  if (timed(s, CQR_K_SMALL, 0, 0, [&] { return cqr::launch_set_int(info, 0, s); }) != hipSuccess)
    return CQR_ERR_HIP;
  if (Q != A) {
    const hipError_t e = timed(s, CQR_K_COPY, 0, 16.0 * m * n, [&] {
      return hipMemcpy2DAsync(Q, lda * 8, A, lda * 8, m * 8, n, hipMemcpyDeviceToDevice, s);
    });
    if (e != hipSuccess) return CQR_ERR_HIP;
  }
  const hipError_t e = (schedule == CQR_SCHED_ORIG) ? run_orig(r, Q, lda, be, R)
                                                    : run_mod(r, Q, lda, be, R);
  return e == hipSuccess ? CQR_OK : CQR_ERR_HIP;
}

int cqr_factor(int64_t m, int64_t n, int64_t b, const double *A, int64_t lda, double *Q,
               double *R, void *stream) {
  return cqr_factor_ex(m, n, b, A, lda, Q, R, stream, nullptr);
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

}  // extern "C"
