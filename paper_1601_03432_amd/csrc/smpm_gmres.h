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
  double* V;        // basis: V + i*vvs + col*k (V_j holds the candidate u_j until it is final);
                    // with basis32 the same buffer holds FP32 entries at the same indices
  int64_t vvs;      // stride between basis vectors (= k * nrhs)
  double* w;        // operator output of the current step, col*k
  double* z;        // M^{-1} u_j
  double* t;        // S z
  double* c;        // Z^T t
  double* sides;    // per-side sums of t (nsides per column), for Z^T t
  double* c2;       // G c
  double* part1;    // partial dots with w, col*ldv*nch + chunk*ldv + i (chunk-major)
  double* part2;    // partial dots with u_j
  double* h1;       // h' = Q^T A q of the last finished vector, col*ldv
  double* h2;       // pre-reduced dots with u_j
  double* dw;       // pre-reduced dots with w
  double* H;        // rotated Hessenberg R, col*ldv*maxit_alloc + j*ldv + i
  double* Hu;       // unrotated Hessenberg, same layout
  double* cs;       // Givens cosines, col*ldv
  double* sn;       // Givens sines
  double* g;        // rotated right-hand side
  double* y;        // least-squares solution
  double* tolb;     // tol * |b|
  double* res;      // residual estimate |g_{j+1}|
  int* active;      // 1 while the column iterates
  int* iters;       // completed Arnoldi steps
  int ldv;          // leading dimension (allocated maxit + 1)
  int maxit;        // iteration limit of this solve
  int nch;          // row chunks of a k-vector
  int rows;         // rows per chunk
  double* tolv;     // relative stopping tolerance (device scalar, set by gm_start)
  int* jdev;        // index j of the next Arnoldi step (device counter, two slots)
  int prereduce;    // 1: the dot sums are reduced once per column by a small kernel
                    // (large grids x many columns); 0: every consumer block reduces
                    // the partials itself (fewer launches).  Same summation order.
  const double* bref2;  // squared reference norm per column (|b|^2): stop when |g| <= tol |b|
  int stream;       // basis loads: -1 non-temporal once a pass reads more than the
                    // last-level cache keeps, 0 always ordinary, 1 always non-temporal
  // progress for the host (pinned, coherent memory): the step that completes every
  // pub_every-th step (0: none) writes each column's activity flag and residual
  // estimate / threshold into slot (chunk % 2) of hflag / hratio (pub_stride entries
  // a slot), then, after a system-scope fence, the number of such chunks into *hseq
  int* hflag;
  double* hratio;
  int* hseq;
  int pub_stride;
  int pub_every;
  int basis32;      // 1: the basis is stored in FP32 (a float view of V; low-precision inner solves)
};

// u_0 = w into V_0, all columns active, j = 0 and the tolerance on the device
void gm_start(const DevPlan& P, const GmState& S, int nrhs, double tol, hipStream_t s);
// the same from b with u_0 = w = b - (Z c2 + {S, S^T} Z c2) (c2 = G Z^T b already formed)
void gm_start_deflated(const DevPlan& P, const GmState& S, int nrhs, const double* b, const double* c2, bool tr,
                       double tol, hipStream_t s);
// One Arnoldi step with j read from slot `par` of the device counter (its last kernel
// writes j + 1 into slot par ^ 1; the q-th step after gm_start uses par = q % 2), so
// a captured sequence of steps replays for any j.  Step j finishes Hessenberg column
// j - 2; every column retires by step maxit + 1, and later steps do nothing.
// kind: 1 = S, 2 = S M^{-1}, 3 = P S M^{-1}; tr selects the transposed operators
// sprec / mprec: OpPrec of the Schur and block-Jacobi operators
void gm_step(const DevPlan& P, const GmState& S, int nrhs, int par, int kind, bool tr, hipStream_t s,
             int sprec = PREC_F64, int mprec = PREC_F64);
// y = R^{-1} g over each column's iterations, then x = V y
void gm_finish(const DevPlan& P, const GmState& S, int nrhs, double* x, hipStream_t s);
int gm_rows_per_chunk(int64_t k);

}  // namespace smpm
