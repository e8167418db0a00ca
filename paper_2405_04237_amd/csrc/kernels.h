// Internal launch interface of the libcqr device kernels (not part of the
// C ABI). Every launcher enqueues on `s`, returns hipSuccess or the launch
// error, and takes the device info word: kernels return early once a
// Cholesky breakdown has been recorded there.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cqr {

constexpr int kTile = 64;        // output tile edge of the MFMA GEMM kernels
constexpr int kNnWaves = 4;      // waves per workgroup of the row-streaming GEMM
constexpr int kLdsPanel = 128;   // largest panel width the LDS Cholesky holds
constexpr int kMaxPanel = 256;   // widest panel (above kLdsPanel: through device memory)

// Kernel variants of the streaming products (the tile fields of
// cqr_options, same values): kTileAuto = the library's default for the
// shape; kTileSlab = update with a 64-column slab of Y staged in LDS (inner
// dimension <= 128); kTileWide = 64 x 128 output tiles per wave (update:
// k_nn_wide, projection: k_tn_wide); kTileNarrow = 32 x 64 update tiles
// (k_nn) or 64 x 64 projection tiles (k_tn); kTileResident = update with each
// wave's rows of L held in registers across every slab of C (inner
// dimension <= 128, a multiple of 16). A variant that does not apply to a
// shape or alignment falls back to the default.
enum TileVariant { kTileAuto = 0, kTileSlab = 1, kTileWide = 2, kTileNarrow = 3, kTileResident = 4 };

// Doubles of device scratch the Cholesky / inverse of a w x w matrix needs
// (0 for w <= kLdsPanel; the identity-padded order-256 matrix otherwise).
inline int64_t chol_scratch_doubles(int w) { return w > kLdsPanel ? int64_t(kMaxPanel) * kMaxPanel : 0; }

// Split-m product partials. For chunk c (rows [c*rc, min(m,(c+1)*rc))):
//   part[c][i*q + j] = sum_rows L[row, i] * Rt[row, j],  i < p, j < q.
// gram = true: p == q and only 64x64 tiles on or above the diagonal are
// produced (entries below the diagonal of `part` are left unwritten); L and
// Rt may differ (a Gram matrix passes the same matrix twice).
// batch > 1: `batch` independent problems of the same shape, operand i at
// base + i * stride (strides in doubles).
// tile (single-matrix projections): kTileNarrow keeps the 64 x 64 tiles
// where the 64 x 128 ones would be used (same bits either way).
hipError_t launch_tn(bool gram, int64_t m, int p, int q, const double *L, int64_t ldl,
                     const double *Rt, int64_t ldr, double *part, int64_t rc, int64_t nch,
                     const int *info, hipStream_t s, int batch = 1, int64_t sL = 0,
                     int64_t sRt = 0, int64_t sPart = 0, int tile = kTileAuto);

// Number of waves one row chunk of launch_tn occupies (its output tiles).
// An upper product with p = q = 128 (batch 1) runs the two-wave balanced
// kernel (one operand loaded once when both are the same matrix); `same` is
// kept for callers and does not change the count. tile = kTileNarrow: the
// count of the plain 64 x 64 tiles.
int64_t tn_tiles(bool gram, int p, int q, bool same = false, int tile = kTileAuto);

// Row-streaming product over all m rows, Y row-major p x q (leading dim ldy):
//   subtract = false: C = L * Y   (Cin unused; C may alias L when q <= 256:
//                                   each workgroup reads its rows of L fully
//                                   before it writes them)
//   subtract = true:  C = Cin + L * Y, where the caller passes Y = -(the
//                     projection), so this is the update C = Cin - L * Yproj.
//                     Cin may equal C (in place); neither may overlap L.
// upper_y: Y is upper triangular (only k <= column terms are summed).
// L2/ldl2/psplit: optional second left operand; rows k >= psplit of Y
// multiply columns k - psplit of L2, i.e. the left operand is
// [L(:, 0:psplit) | L2]. L2 = nullptr means L alone.
// C2/ldc2 (subtract = false, batch = 1 only): a second destination that
// receives the same values as C.
// skip (optional): the kernels do nothing when *skip != 0 at run time (the
// caller has made the product an identity: Y = 0 for an update, Y = I for
// an in-place product).
// tile: the kernel variant of a single-matrix update (subtract = true,
// batch = 1, no L2, no C2); every variant gives the same bits.
// lower_first: rows k < psplit of Y are lower triangular (Y[k][c] = 0 for
// c > k, exact zeros), so the wide product of an input-free [L | L2] Y may
// skip their zero blocks (the adjoint's [dQ | Q] [R^{-T}; G]).
hipError_t launch_nn(bool subtract, bool upper_y, int64_t m, int p, int q, const double *L,
                     int64_t ldl, const double *Y, int64_t ldy, const double *Cin, int64_t ldci,
                     double *C, int64_t ldc, const int *info, hipStream_t s,
                     const double *L2 = nullptr, int64_t ldl2 = 0, int psplit = 0, int batch = 1,
                     int64_t sL = 0, int64_t sL2 = 0, int64_t sY = 0, int64_t sCin = 0,
                     int64_t sC = 0, double *C2 = nullptr, int64_t ldc2 = 0,
                     const int *skip = nullptr, int tile = kTileAuto, bool lower_first = false);

// True when launch_nn runs a single-matrix subtract = true product through
// the short-inner-dimension kernel (Y staged in LDS); false: the general one.
bool nn_short_k(int p, const double *L, int64_t ldl, const double *Cin, int64_t ldci,
                const double *C, int64_t ldc);

// Leading dimension used for row-major p x q operands written by the
// library (a multiple of 4 doubles, so rows stay 32-byte aligned).
__host__ __device__ inline int64_t padded_ld(int64_t q) { return (q + 3) / 4 * 4; }

// Fixed-order (pairwise) sum over nch partials of p x q. The partial buffer
// is used as scratch (overwritten) when nch is large.
// gram = true: out[i*p + j] = sum for i <= j, 0 below the diagonal.
// gram = false: out[i*ldo + j] = neg ? -sum : sum; if rblk != nullptr also
//               rblk[i + j*ldr] = sum (an R block, column-major).
hipError_t launch_reduce(bool gram, double *part, int64_t nch, int p, int q, double *out,
                         int64_t ldo, double *rblk, int64_t ldr, bool neg, const int *info,
                         hipStream_t s, int batch = 1, int64_t sPart = 0, int64_t sOut = 0,
                         int64_t sR = 0);

// One workgroup: W (row-major w x w, upper triangle read) = U^T U, then
// U^{-1}. Writes U row-major (ld w) to uout (if non-null), U column-major into
// the R block rblk (if non-null, strict lower part set to 0), U^{-1}
// row-major with leading dimension padded_ld(w) to uinv (strict lower part 0). A pivot that is not > 0 sets *info = col0 + i
// + 1 (first failure wins) and leaves the outputs undefined.
// skip (optional): first ||W - I||_F is summed in a fixed order; if it is
// <= skip_tol the outputs are U = U^{-1} = I and *skip = 1 (no Cholesky),
// else *skip = 0.
// w <= kMaxPanel; for w > kLdsPanel, gwork is device scratch of
// chol_scratch_doubles(w) doubles (the matrix is factored there).
hipError_t launch_chol_inv(const double *W, int w, double *uout, double *rblk, int64_t ldr,
                           double *uinv, int *info, int col0, hipStream_t s,
                           double skip_tol = 0.0, int *skip = nullptr, double *gwork = nullptr);

// ||Z||_F of the rows x cols row-major Z (leading dim ldz), fixed order; if
// <= tol, Z := 0 and *skip = 1, else *skip = 0. One workgroup.
hipError_t launch_zskip(double *Z, int rows, int cols, int64_t ldz, double tol, int *skip,
                        const int *info, hipStream_t s);

// Rinv = R^{-1} for `batch` upper triangular n x n matrices (R column-major
// ld n at R + i*sR; Rinv row-major ld n at Rinv + i*sRi); n <= kMaxPanel.
// RinvT (optional, same strides): R^{-T} row-major as well.
hipError_t launch_tri_inv(const double *R, int n, int64_t sR, double *Rinv, int64_t sRi, int batch,
                          hipStream_t s, double *RinvT = nullptr);

// The n x n part of the QR adjoint, per matrix i of the batch (Rinv and
// RinvT = R^{-1} and R^{-T}, both row-major, from launch_tri_inv):
//   C = copyltu(R dR^T - P) with P = dQ^T Q taken from T = S^T dQ (upper
//   triangle of a row-major n x n; S = Q, or A when recompute != 0, in which
//   case Q = A R^{-1} is applied through Rinv); has_p = 0 drops P, dR =
//   nullptr drops R dR^T;
//   G = C R^{-T};
//   Y (row-major, ld ldy) = [R^{-T}; G] (with_rt) or [G], where G becomes
//   R^{-1} G under recompute.
// C and G are n x n row-major scratch at C + i*sCG, G + i*sCG.
hipError_t launch_adj_small(int n, const double *T, int64_t sT, const double *R, const double *dR,
                            int64_t sRn, const double *Rinv, const double *RinvT, int64_t sRi,
                            int has_p, int recompute, double *C, double *G, int64_t sCG, double *Y,
                            int64_t ldy, int64_t sY, int with_rt, int batch, hipStream_t s);

// R[0:s, 0:w] -= Zn * Ua  (R block column-major ldr; Zn = -Z row-major s x w
//                          with leading dim ldz, as stored by the reduction
//                          for the update; Ua row-major w x w upper triangular)
hipError_t launch_r_add_zu(int s_rows, int w, const double *Z, int64_t ldz, const double *Ua,
                           double *rblk, int64_t ldr, const int *info, hipStream_t s);

// R[0:w, 0:w] = Ub * Ua (both row-major w x w upper triangular); the strict
// lower part of the block is set to 0.
hipError_t launch_r_upper_product(int w, const double *Ub, const double *Ua, double *rblk,
                                  int64_t ldr, const int *info, hipStream_t s);

// Shifted Gram (Algorithm 4): W += s I with s = sqrt_m_u * trace(W), for the
// w x w Gram matrix W as the reduction stores it (leading dim w). trace(W) = ||X||_F^2 when W = X^T X;
// it is summed by one thread in column order. No-op when *info != 0.
hipError_t launch_shift_diag(double *W, int w, double sqrt_m_u, const int *info, hipStream_t s);

// R = R2 * R1 for n x n upper triangular column-major matrices (leading
// dimension n); strict lower part of R set to 0.
hipError_t launch_trmm_upper(int n, const double *R2, const double *R1, double *R, const int *info,
                             hipStream_t s);

// p[0:count] = 0
hipError_t launch_zero(double *p, int64_t count, hipStream_t s);

// zero `batch` column-major rows x cols blocks (leading dim ld, block i at
// p + i*sb)
hipError_t launch_zero2d(double *p, int64_t rows, int64_t cols, int64_t ld, int64_t sb, int batch,
                         hipStream_t s);

// dst[0:m, c] = src[0:m, c] for c < n (column-major, leading dims lds / ldd)
hipError_t launch_copy_cols(int64_t m, int64_t n, const double *src, int64_t lds, double *dst,
                            int64_t ldd, hipStream_t s);

// *p = v (a kernel, not a memset, so that it is safe inside captured graphs)
hipError_t launch_set_int(int *p, int v, hipStream_t s);

}  // namespace cqr
