// Kernels of block GMRES: every right-hand side of the deflated Schur system
// (Algorithm 3 step 4) in one block Krylov space.  The Gram-Schmidt sums and updates
// of a block against the shared basis are tall-skinny products on FP64 matrix cores
// (the update of at most 8 columns against an FP32 basis on FP64 vector FMAs); the
// block's own orthonormalization is Cholesky QR applied twice with rank
// deflation; the block Hessenberg least-squares problem is updated by Householder
// reflections in one workgroup.  Vectors are column-blocked: vector i of a set
// starts at i * len.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace smpm {

constexpr int kBgMaxCols = 32;  // widest block (columns per block)

// doubles of partial sums launch_bg_dot may use (its part argument)
int64_t bg_dot_part_size();

// out[b * ldo + a] = beta * out[b * ldo + a] + sum_x A[a * len + x] B[b * len + x]
// for a < na, b < nb (nb <= kBgMaxCols); beta = 0 does not read out; outT, if given,
// receives the same values at outT[a * kBgMaxCols + b].  Deterministic: fixed x chunks
// summed in a fixed order.
// A is FP64, or FP32 (a basis stored in FP32; the products are FP64).
template <typename AT>
void launch_bg_dot(const AT* A, int na, const double* B, int nb, int64_t len, double* part, double* out, int ldo,
                   double beta, hipStream_t s, double* outT = nullptr);

// out[b * len + x] = beta * win[b * len + x] + alpha * sum_a A[a * len + x] H[a * sa + b * sb]
// for b < nb (nb <= kBgMaxCols), x < len.  out may equal win, never A; beta = 0 does
// not read win.  Instantiated for (A, out) = (FP64, FP64), (FP32, FP64) and (FP64,
// FP32): FP64 arithmetic, an FP32 basis read or written.
template <typename AT, typename OT>
void launch_bg_update(const AT* A, int na, const double* H, int64_t sa, int64_t sb, double alpha, const OT* win,
                      double beta, OT* out, int nb, int64_t len, hipStream_t s);

// b = (double) a, n entries
void launch_bg_widen(const float* a, double* b, int64_t n, hipStream_t s);

// One pass of Cholesky QR of a block of m columns (Gram matrix G, m x m, ld m):
// columns taken in order, a column whose part orthogonal to the kept ones is <= drop
// times its own norm (drop = 0: only a non-positive pivot) adds no vector.  Writes
// the kept count to *cnt, T (m x m, ld m; column c = coefficients of kept vector c on
// the block's columns, columns >= *cnt zero) and R (ld kBgMaxCols; R[c + 32 i] =
// coefficient of kept vector c in column i).  With cnt_in non-null only its first
// *cnt_in columns are considered (the rest are zero vectors of an earlier pass), and
// with rprev non-null R is returned multiplied by rprev (R rprev, rprev of the same
// layout and *cnt_in rows).
void launch_bg_chol(const double* G, int m, double drop, const int* cnt_in, const double* rprev, int* cnt,
                    double* T, double* R, hipStream_t s);

// State of the block Hessenberg least-squares problem min |E_1 R_0 - Hbar Y| per
// column, reduced by Householder reflections as block columns arrive.
struct BgLsq {
  double* H;     // (ldH rows) x cap columns: rotated Hbar (upper triangle: its R factor)
  int ldH;       // cap + kBgMaxCols
  double* refl;  // cap x (2 kBgMaxCols): the reflection vector of each column
  double* rbeta; // cap: 2 / |v|^2 of each reflection (0: identity)
  double* G;     // ldH x s: rotated right-hand side block
  int s;         // right-hand-side columns
  double* res;   // s: least-squares residual of each column after the last update
};

// Block step: columns n0 .. n0+r-1 of Hbar arrive (h: nv x r, ld ldh, the basis
// coefficients; R: cnts[1] x r, ld kBgMaxCols, the new block's coefficients, its rows
// nv .. nv + cnts[1] - 1; cnts: the kept counts of the two Cholesky QR passes).
// Applies the earlier reflections, reduces the new columns, rotates G, sets res and
// publishes res (s doubles) and both counts (2 ints) to host memory (pinned).
void launch_bg_lsq(const BgLsq& L, int n0, int r, int nv, const double* h, int ldh, const double* R,
                   const int* cnts, double* host_res, int* host_cnt, hipStream_t s);

// Y (ncol x s, ld ldy) = triangle(H)^{-1} G[0 .. ncol)
void launch_bg_backsolve(const BgLsq& L, int ncol, double* Y, int ldy, hipStream_t s);

// G = 0 (rows 0 .. ldH of every column), then G[0 .. m) = R0 (m x s, ld kBgMaxCols)
void launch_bg_lsq_start(const BgLsq& L, const double* R0, const int* m, hipStream_t s);

}  // namespace smpm
