// Device-resident GMRES state and launchers (see smpm_gmres.hip).
#pragma once
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "smpm_kernels.h"

namespace smpm {

constexpr int kMaxIt = 1000;     // largest Krylov dimension per solve
constexpr int kRowsMax = 2048;   // rows of a k-vector handled by one block

struct GmState {
  double* V;        // basis: V + i*vvs + col*k
  int64_t vvs;      // stride between basis vectors (= k * nrhs)
  double* w;        // working vector, col*k
  double* z;        // M^{-1} v_j
  double* t;        // S z
  double* c;        // Z^T t
  double* sides;    // per-side sums of t (nsides per column), for Z^T t
  double* c2;       // G c
  double* part1;    // partial dots, col*ldv*nch + i*nch + chunk
  double* part2;
  double* part3;    // partial squared norms, col*nch + chunk
  double* h1;       // first-pass coefficients, col*ldv
  double* h2;       // second-pass coefficients
  double* H;        // rotated Hessenberg R, col*ldv*maxit_alloc + j*ldv + i
  double* cs;       // Givens cosines, col*ldv
  double* sn;       // Givens sines
  double* g;        // rotated right-hand side
  double* y;        // least-squares solution
  double* beta_cur; // norm of the vector being normalized
  double* beta0;    // initial residual norm
  double* tolb;     // tol * beta0
  double* res;      // residual estimate |g_{j+1}|
  int* active;      // 1 while the column iterates
  int* iters;       // completed Arnoldi steps
  int* counter;     // last-block tickets, col*4
  int ldv;          // leading dimension (allocated maxit + 1)
  int maxit;        // iteration limit of this solve
  int nch;          // row chunks of a k-vector
  int rows;         // rows per chunk
  double* tolv;     // relative stopping tolerance (device scalar, set by gm_start)
  int* jdev;        // index j of the next Arnoldi step (device counter, two slots)
  int prereduce;    // 1: h1, h2 and beta are reduced once per column by small kernels
                    // (large grids x many columns); 0: every consumer block reduces
                    // the partials itself (fewer launches).  Same summation order.
  const double* bref2;  // squared reference norm per column (|b|^2): stop when |g| <= tol |b|
};

// initial residual norms, all columns active, j = 0 and the tolerance on the device
void gm_start(const DevPlan& P, const GmState& S, int nrhs, double tol, hipStream_t s);
// One Arnoldi step with j read from slot `par` of the device counter (its last kernel
// writes j + 1 into slot par ^ 1; the q-th step after gm_start uses par = q % 2), so
// a captured sequence of steps replays for any j.  Steps past maxit do nothing:
// every column retires at j = maxit.
// kind: 1 = S, 2 = S M^{-1}, 3 = P S M^{-1}; tr selects the transposed operators
// sprec / mprec: OpPrec of the Schur and block-Jacobi operators
void gm_step(const DevPlan& P, const GmState& S, int nrhs, int par, int kind, bool tr, hipStream_t s,
             int sprec = PREC_F64, int mprec = PREC_F64);
// Givens step for the last column of the steps enqueued so far (par = steps % 2)
void gm_close(const DevPlan& P, const GmState& S, int nrhs, int par, int kind, bool tr, hipStream_t s);
void gm_finish(const DevPlan& P, const GmState& S, int nrhs, double* x, hipStream_t s);
int gm_rows_per_chunk(int64_t k);

}  // namespace smpm
