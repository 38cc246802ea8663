// Device-resident GMRES iteration for the deflated Schur complement system.
//
// One Arnoldi step j of right-preconditioned GMRES on P S M^{-1} (Algorithm 3,
// step 4) is five kernels that read j from a device counter and keep every scalar
// on the device, so the host never waits inside the loop and a captured chunk of
// steps (hipGraph) replays for any j.  The counter is double-buffered: step q of a
// chunk reads slot q % 2 and its last kernel writes j + 1 into the other slot, so
// no kernel reads a value another block of it may be changing:
//   gm_precond  h2 and beta_j from the previous step's partials; block 0 applies
//               the Givens rotations to Hessenberg column j-1 and retires the
//               column once its residual estimate reaches tol * |b|;
//               v_j = (w - V h2) / beta_j (into V), z = M^{-1} v_j
//   Schur       t = S z, with the per-side sums of t for Z^T t
//   coarse      c2 = G Z^T t
//   gm_orth1    w = t - Z c2 - S Z c2 (deflation), partial dots V^T w
//   gm_orth2    h1 = sum of partials; w -= V h1; partial dots V^T w and |w|^2;
//               next j
// Classical Gram-Schmidt is applied twice, the second pass delayed into the next
// step's gm_precond: h2 = V^T w from gm_orth2's partials, beta^2 = |w|^2 - |h2|^2
// (Pythagoras), v = (w - V h2) / beta per slot.  One reduction fewer per step, as
// in the low-synchronization CGS2 variants of Swirydowicz, Bielich, Langou,
// Thomas et al.
// Each block handles a chunk of rows.  Every block that needs a reduced value
// sums the previous kernel's per-chunk partials itself, in one fixed order, so
// results are deterministic and no inter-block fence is needed.
#include <hip/hip_runtime.h>

#include "smpm_gmres.h"

namespace smpm {

namespace {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;
constexpr int kDotUnroll = 8;

__device__ __forceinline__ double wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

__device__ __forceinline__ double block_sum(double v, double* red) {
  v = wave_sum(v);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  return (red[0] + red[1]) + (red[2] + red[3]);
}

// out[i] = sum_c part[i*nch + c], i < nvec, into LDS.  Wave q owns groups of
// eight vectors; lanes take chunks lane, lane+64, ... and a fixed shuffle tree
// combines them, so every block obtains bit-identical sums.
__device__ void reduce_partials(const double* __restrict__ part, int nvec, int nch, double* out) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  for (int i0 = wave * 8; i0 < nvec; i0 += kWaves * 8) {
    double acc[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    for (int c = lane; c < nch; c += 64) {
#pragma unroll
      for (int u = 0; u < 8; ++u)
        if (i0 + u < nvec) acc[u] += part[(int64_t)(i0 + u) * nch + c];
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const double v = wave_sum(acc[u]);
      if (lane == 0 && i0 + u < nvec) out[i0 + u] = v;
    }
  }
}

// Partial dots of the chunk held in LDS (wv, `rows` rows) with V_0..V_{nvec-1}:
// wave q handles groups of kDotUnroll vectors whose loads are all issued before
// the shuffle reductions; lanes run over rows.
__device__ void chunk_dots(const double* __restrict__ V, int64_t vvs, int64_t x0, int rows, const double* wv,
                           int nvec, double* part, int nch, int chunk) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  for (int i0 = wave * kDotUnroll; i0 < nvec; i0 += kWaves * kDotUnroll) {
    double acc[kDotUnroll];
#pragma unroll
    for (int u = 0; u < kDotUnroll; ++u) acc[u] = 0.0;
    for (int x = lane; x < rows; x += 64) {
      const double wx = wv[x];
#pragma unroll
      for (int u = 0; u < kDotUnroll; ++u)
        if (i0 + u < nvec) acc[u] = fma(V[(int64_t)(i0 + u) * vvs + x0 + x], wx, acc[u]);
    }
#pragma unroll
    for (int u = 0; u < kDotUnroll; ++u) {
      const double v = wave_sum(acc[u]);
      if (lane == 0 && i0 + u < nvec) part[(int64_t)(i0 + u) * nch + chunk] = v;
    }
  }
}

// Givens step for Hessenberg column jc = j-1 of one right-hand side, run by
// block 0 of gm_precond: H(:, jc) = h1 + h2 with beta below the diagonal,
// rotated by the previous rotations; a new rotation zeroes beta.
__device__ void givens_column(const GmState& S, int col, int j, double beta, const double* h2) {
  __shared__ double hc[kMaxIt + 2];
  __shared__ double csl[kMaxIt + 1], snl[kMaxIt + 1];
  const int tid = threadIdx.x;
  const int jc = j - 1;
  const double* h1 = S.h1 + (int64_t)col * S.ldv;
  double* csg = S.cs + (int64_t)col * S.ldv;
  double* sng = S.sn + (int64_t)col * S.ldv;
  for (int i = tid; i <= jc; i += kThreads) hc[i] = h1[i] + h2[i];
  for (int i = tid; i < jc; i += kThreads) {
    csl[i] = csg[i];
    snl[i] = sng[i];
  }
  __syncthreads();
  if (tid == 0) {
    hc[jc + 1] = beta;
    for (int i = 0; i < jc; ++i) {
      const double a = hc[i], b = hc[i + 1];
      hc[i] = csl[i] * a + snl[i] * b;
      hc[i + 1] = -snl[i] * a + csl[i] * b;
    }
    const double a = hc[jc], b = hc[jc + 1];
    const double rr = hypot(a, b);
    const double c = rr > 0.0 ? a / rr : 1.0;
    const double s = rr > 0.0 ? b / rr : 0.0;
    hc[jc] = rr;
    csg[jc] = c;
    sng[jc] = s;
    double* gc = S.g + (int64_t)col * S.ldv;
    const double gj = gc[jc];
    gc[jc + 1] = -s * gj;
    gc[jc] = c * gj;
    const double res = fabs(gc[jc + 1]);
    S.res[col] = res;
    if (!(res > S.tolb[col]) || j >= S.maxit || !(beta > 0.0)) {
      S.active[col] = 0;
      S.iters[col] = j;
    }
  }
  __syncthreads();
  double* Hcol = S.H + (int64_t)col * S.ldv * S.maxit + (int64_t)jc * S.ldv;
  for (int i = tid; i <= jc; i += kThreads) Hcol[i] = hc[i];
}

}  // namespace

// ------------------------------------------------------------------ kernels

// beta_j, Givens for column j-1 (block 0), v_j = w / beta_j into V_j and
// z = M^{-1} v_j (or z = v_j).  givens_only: stop after the Givens step.
template <typename OpT>
__global__ __launch_bounds__(256) void k_gm_precond(DevPlan P, GmState S, int par, int use_precond, int transpose,
                                                    int givens_only) {
  using Acc = typename AccOf<OpT>::type;
  __shared__ Acc xs[8 * kMaxN];
  __shared__ double red[kWaves];
  __shared__ double h2s[kMaxIt + 1];
  const int col = blockIdx.y, tid = threadIdx.x;
  if (!S.active[col]) return;
  const int j = S.jdev[par];
  if (j > S.maxit) return;
  // second Gram-Schmidt pass of the previous step: h2 and beta (see the file header)
  const int nh = j;  // h2 has j entries (none before the first step)
  double beta;
  if (S.prereduce && nh > 0) {
    for (int i = tid; i < nh; i += kThreads) h2s[i] = S.h2[(int64_t)col * S.ldv + i];
    __syncthreads();
    beta = S.beta_cur[col];
  } else {
    if (nh > 0) reduce_partials(S.part2 + (int64_t)col * S.ldv * S.nch, nh, S.nch, h2s);
    __syncthreads();
    if (tid < 64) {
      double acc = 0.0, hh = 0.0;
      for (int c = tid; c < S.nch; c += 64) acc += S.part3[(int64_t)col * S.nch + c];
      for (int i = tid; i < nh; i += 64) hh = fma(h2s[i], h2s[i], hh);
      acc = wave_sum(acc);
      hh = wave_sum(hh);
      if (tid == 0) red[0] = sqrt(fmax(acc - hh, 0.0));
    }
    __syncthreads();
    beta = red[0];
  }
  if (blockIdx.x == 0) {
    if (j == 0) {
      if (tid == 0) {
        S.tolb[col] = S.tolv[0] * (S.bref2 ? sqrt(S.bref2[col]) : beta);
        S.g[(int64_t)col * S.ldv] = beta;
        S.res[col] = beta;
        if (!(beta > 0.0)) {
          S.active[col] = 0;
          S.iters[col] = 0;
        }
      }
    } else {
      givens_column(S, col, j, beta, h2s);
    }
  }
  if (givens_only) return;
  const double inv = beta > 0.0 ? 1.0 / beta : 0.0;
  const int64_t k = P.k;
  const double* wc = S.w + (int64_t)col * k;
  const double* Vc = S.V + (int64_t)col * k;
  double* vj = S.V + (int64_t)j * S.vvs + (int64_t)col * k;
  double* zc = S.z + (int64_t)col * k;
  // v_j = (w - V h2) / beta at one slot
  auto vnew = [&](int64_t x) {
    double acc = wc[x];
#pragma unroll 8
    for (int i = 0; i < nh; ++i) acc = fma(-h2s[i], Vc[(int64_t)i * S.vvs + x], acc);
    return acc * inv;
  };
  if (!use_precond) {
    for (int64_t x = (int64_t)blockIdx.x * kThreads + tid; x < k; x += (int64_t)gridDim.x * kThreads) {
      const double v = vnew(x);
      vj[x] = v;
      zc[x] = v;
    }
    return;
  }
  for (int b = blockIdx.x; b < P.nblk; b += gridDim.x) {
    const int o = P.blk_off[b], sb = P.blk_off[b + 1] - o;
    const int bc = P.blk_cls[b];
    __syncthreads();
    for (int i = tid; i < sb; i += kThreads) {
      const int slot = P.blk_slots[o + i];
      const double v = vnew(slot);
      xs[i] = (Acc)v;
      vj[slot] = v;
    }
    __syncthreads();
    const OpT* Mp = minv_op<OpT>(P, transpose != 0) + P.bcls_off[bc];
    for (int r = tid; r < sb; r += kThreads) {
      Acc acc = 0;
#pragma unroll 8
      for (int c = 0; c < sb; ++c) acc = fma(to_acc(Mp[c * sb + r]), xs[c], acc);
      zc[P.blk_slots[o + r]] = (double)acc;
    }
  }
}

// w = t - (Z c2 + {S Z c2 | S^T Z c2}) on this block's rows (or w = t), then
// partial dots with V_0..V_j.
__global__ __launch_bounds__(256) void k_gm_orth1(DevPlan P, GmState S, int par, int defl, int transpose) {
  __shared__ double wv[kRowsMax];
  const int col = blockIdx.y, chunk = blockIdx.x, tid = threadIdx.x;
  if (!S.active[col]) return;
  const int j = S.jdev[par];
  const int64_t k = P.k, x0 = (int64_t)chunk * S.rows;
  const int rows = (int)min((int64_t)S.rows, k - x0);
  const double* tc = S.t + (int64_t)col * k;
  double* wc = S.w + (int64_t)col * k;
  const double* cc = S.c2 + (int64_t)col * P.d;
  const int n = P.n;
  for (int q = tid; q < rows; q += kThreads) {
    const int64_t slot = x0 + q;
    double v = tc[slot];
    if (defl) {
      const int si = (int)(slot / n), tt = (int)(slot - (int64_t)si * n);
      const int e = P.side_elem[si], s = P.side_dir[si];
      double acc = cc[P.iface[e * 4 + s]];
      if (!transpose) {
        const int J = P.nbr[e * 4 + s], cJ = P.cls[J], so = s ^ 1;
        const double* wz = P.WZ + (((int64_t)cJ * 4 + so) * n + tt) * 4;
        for (int s2 = 0; s2 < 4; ++s2) {
          const int j2 = P.iface[J * 4 + s2];
          if (j2 >= 0) acc = fma(wz[s2], cc[j2], acc);
        }
      } else {
        const int ce = P.cls[e];
        const int cidx = (int)(slot - P.slot_off[e]);
        for (int s2 = 0; s2 < 4; ++s2) {
          const int j2 = P.iface[e * 4 + s2];
          if (j2 >= 0) acc = fma(P.WZc[((int64_t)ce * 4 + s2) * 4 * n + cidx], cc[j2], acc);
        }
      }
      v -= acc;
    }
    wc[slot] = v;
    wv[q] = v;
  }
  __syncthreads();
  chunk_dots(S.V + (int64_t)col * k, S.vvs, x0, rows, wv, j + 1, S.part1 + (int64_t)col * S.ldv * S.nch, S.nch,
             chunk);
}

// h1 = sum of part1 (block 0 stores it for the Givens step); w -= V h1; partial dots
// V^T w into part2 and partial |w|^2 into part3; the next step's index.
__global__ __launch_bounds__(256) void k_gm_orth2(DevPlan P, GmState S, int par) {
  __shared__ double wv[kRowsMax];
  __shared__ double hs[kMaxIt + 1];
  __shared__ double red[kWaves];
  const int col = blockIdx.y, chunk = blockIdx.x, tid = threadIdx.x;
  const int j = S.jdev[par];
  // the step's last kernel sets the next step's index in the other slot (whatever the
  // columns' activity, so steps keep counting)
  if (blockIdx.x == 0 && blockIdx.y == 0 && tid == 0) S.jdev[par ^ 1] = j + 1;
  if (!S.active[col]) return;
  const int64_t k = P.k, x0 = (int64_t)chunk * S.rows;
  const int rows = (int)min((int64_t)S.rows, k - x0);
  const int nvec = j + 1;
  if (S.prereduce) {
    for (int i = tid; i < nvec; i += kThreads) hs[i] = S.h1[(int64_t)col * S.ldv + i];
    __syncthreads();
  } else {
    reduce_partials(S.part1 + (int64_t)col * S.ldv * S.nch, nvec, S.nch, hs);
    __syncthreads();
    if (chunk == 0) {
      double* hdst = S.h1 + (int64_t)col * S.ldv;
      for (int i = tid; i < nvec; i += kThreads) hdst[i] = hs[i];
    }
  }
  double* wc = S.w + (int64_t)col * k;
  const double* Vc = S.V + (int64_t)col * k;
  double nrm = 0.0;
  for (int q = tid; q < rows; q += kThreads) {
    const int64_t x = x0 + q;
    double acc = 0.0;
#pragma unroll 16
    for (int i = 0; i < nvec; ++i) acc = fma(hs[i], Vc[(int64_t)i * S.vvs + x], acc);
    const double v = wc[x] - acc;
    wc[x] = v;
    wv[q] = v;
    nrm = fma(v, v, nrm);
  }
  __syncthreads();
  chunk_dots(Vc, S.vvs, x0, rows, wv, nvec, S.part2 + (int64_t)col * S.ldv * S.nch, S.nch, chunk);
  const double bs = block_sum(nrm, red);
  if (tid == 0) S.part3[(int64_t)col * S.nch + chunk] = bs;
}

// Pre-reduction (one block per column): h1 from gm_orth1's partials.
__global__ __launch_bounds__(256) void k_gm_reduce_h1(GmState S, int par) {
  __shared__ double hs[kMaxIt + 1];
  const int col = blockIdx.y;
  if (!S.active[col]) return;
  const int nvec = S.jdev[par] + 1;
  reduce_partials(S.part1 + (int64_t)col * S.ldv * S.nch, nvec, S.nch, hs);
  __syncthreads();
  for (int i = threadIdx.x; i < nvec; i += kThreads) S.h1[(int64_t)col * S.ldv + i] = hs[i];
}

// Pre-reduction after gm_orth2: h2 and beta for the next step, summed exactly as
// gm_precond sums them itself.
__global__ __launch_bounds__(256) void k_gm_reduce_beta(GmState S, int par) {
  __shared__ double hs[kMaxIt + 1];
  const int col = blockIdx.y, tid = threadIdx.x;
  if (!S.active[col]) return;
  const int nh = S.jdev[par] + 1;
  reduce_partials(S.part2 + (int64_t)col * S.ldv * S.nch, nh, S.nch, hs);
  __syncthreads();
  for (int i = tid; i < nh; i += kThreads) S.h2[(int64_t)col * S.ldv + i] = hs[i];
  if (tid < 64) {
    double acc = 0.0, hh = 0.0;
    for (int c = tid; c < S.nch; c += 64) acc += S.part3[(int64_t)col * S.nch + c];
    for (int i = tid; i < nh; i += 64) hh = fma(hs[i], hs[i], hh);
    acc = wave_sum(acc);
    hh = wave_sum(hh);
    if (tid == 0) S.beta_cur[col] = sqrt(fmax(acc - hh, 0.0));
  }
}

// Start of a solve: partial |w|^2 of the initial residual; all columns active;
// j = 0 and the tolerance.
__global__ __launch_bounds__(256) void k_gm_start(DevPlan P, GmState S, double tol) {
  __shared__ double red[kWaves];
  const int col = blockIdx.y, chunk = blockIdx.x, tid = threadIdx.x;
  const int64_t k = P.k, x0 = (int64_t)chunk * S.rows;
  const int rows = (int)min((int64_t)S.rows, k - x0);
  const double* wc = S.w + (int64_t)col * k;
  double nrm = 0.0;
  for (int q = tid; q < rows; q += kThreads) nrm = fma(wc[x0 + q], wc[x0 + q], nrm);
  const double bs = block_sum(nrm, red);
  if (tid == 0) S.part3[(int64_t)col * S.nch + chunk] = bs;
  if (chunk == 0 && tid == 0) {
    S.active[col] = 1;
    S.iters[col] = 0;
    if (col == 0) {
      S.jdev[0] = 0;
      S.tolv[0] = tol;
    }
  }
}

// y = R^{-1} g for the first iters[col] columns (R = rotated Hessenberg), one
// block per column, column-oriented back substitution.
__global__ __launch_bounds__(256) void k_gm_lsq(GmState S) {
  __shared__ double gs[kMaxIt + 1];
  const int col = blockIdx.x, tid = threadIdx.x;
  const int J = S.iters[col];
  const double* gc = S.g + (int64_t)col * S.ldv;
  const double* Hc = S.H + (int64_t)col * S.ldv * S.maxit;
  double* yc = S.y + (int64_t)col * S.ldv;
  for (int i = tid; i < J; i += kThreads) gs[i] = gc[i];
  for (int i = J + tid; i < S.ldv; i += kThreads) yc[i] = 0.0;
  __syncthreads();
  for (int i = J - 1; i >= 0; --i) {
    const double yi = gs[i] / Hc[(int64_t)i * S.ldv + i];
    __syncthreads();
    for (int m = tid; m < i; m += kThreads) gs[m] -= Hc[(int64_t)i * S.ldv + m] * yi;
    if (tid == 0) yc[i] = yi;
    __syncthreads();
  }
}

// x = sum_{i < iters[col]} y_i V_i
__global__ __launch_bounds__(256) void k_gm_combine(DevPlan P, GmState S, double* __restrict__ x) {
  const int col = blockIdx.y;
  const int64_t k = P.k;
  const int J = S.iters[col];
  const double* yc = S.y + (int64_t)col * S.ldv;
  const double* Vc = S.V + (int64_t)col * k;
  for (int64_t q = (int64_t)blockIdx.x * kThreads + threadIdx.x; q < k; q += (int64_t)gridDim.x * kThreads) {
    double acc = 0.0;
#pragma unroll 8
    for (int i = 0; i < J; ++i) acc = fma(yc[i], Vc[(int64_t)i * S.vvs + q], acc);
    x[(int64_t)col * k + q] = acc;
  }
}

// ------------------------------------------------------------------ launchers

void gm_start(const DevPlan& P, const GmState& S, int nrhs, double tol, hipStream_t s) {
  hipLaunchKernelGGL(k_gm_start, dim3(S.nch, nrhs), dim3(kThreads), 0, s, P, S, tol);
}

static int precond_grid(const DevPlan& P, const GmState& S, int kind) {
  return kind == 1 ? S.nch : std::max(1, std::min(P.nblk, 1024));
}

void gm_step(const DevPlan& P, const GmState& S, int nrhs, int par, int kind, bool tr, hipStream_t s, int sprec,
             int mprec) {
  const dim3 pg(precond_grid(P, S, kind), nrhs);
  const int up = kind == 1 ? 0 : 1, trn = tr ? 1 : 0;
  if (mprec == PREC_F32)
    hipLaunchKernelGGL(k_gm_precond<float>, pg, dim3(kThreads), 0, s, P, S, par, up, trn, 0);
  else if (mprec == PREC_BF16)
    hipLaunchKernelGGL(k_gm_precond<bf16s>, pg, dim3(kThreads), 0, s, P, S, par, up, trn, 0);
  else
    hipLaunchKernelGGL(k_gm_precond<double>, pg, dim3(kThreads), 0, s, P, S, par, up, trn, 0);
  const bool fused_sums = kind == 3 && !tr && schur_has_side_sums(P) && P.coarse_mode == 1;
  launch_schur_ex(P, S.z, S.t, nrhs, tr, S.active, fused_sums ? S.sides : nullptr, s, sprec);
  if (kind == 3) {
    if (fused_sums) {
      launch_coarse_sides(P, S.sides, S.c2, nrhs, tr, S.active, s);
    } else {
      launch_iface_sum(P, S.t, S.c, nrhs, S.active, s);
      launch_coarse(P, S.c, S.c2, nrhs, tr, S.active, s);
    }
  }
  hipLaunchKernelGGL(k_gm_orth1, dim3(S.nch, nrhs), dim3(kThreads), 0, s, P, S, par, kind == 3 ? 1 : 0,
                     tr ? 1 : 0);
  if (S.prereduce) hipLaunchKernelGGL(k_gm_reduce_h1, dim3(1, nrhs), dim3(kThreads), 0, s, S, par);
  hipLaunchKernelGGL(k_gm_orth2, dim3(S.nch, nrhs), dim3(kThreads), 0, s, P, S, par);
  if (S.prereduce) hipLaunchKernelGGL(k_gm_reduce_beta, dim3(1, nrhs), dim3(kThreads), 0, s, S, par);
}

void gm_close(const DevPlan& P, const GmState& S, int nrhs, int par, int kind, bool tr, hipStream_t s) {
  hipLaunchKernelGGL(k_gm_precond<double>, dim3(1, nrhs), dim3(kThreads), 0, s, P, S, par, kind == 1 ? 0 : 1,
                     tr ? 1 : 0, 1);
}

void gm_finish(const DevPlan& P, const GmState& S, int nrhs, double* x, hipStream_t s) {
  hipLaunchKernelGGL(k_gm_lsq, dim3(nrhs), dim3(kThreads), 0, s, S);
  const int64_t blocks = std::min<int64_t>((P.k + kThreads - 1) / kThreads, 2048);
  hipLaunchKernelGGL(k_gm_combine, dim3((unsigned)blocks, nrhs), dim3(kThreads), 0, s, P, S, x);
}

int gm_rows_per_chunk(int64_t k) {
  // chunks of 256..kRowsMax rows, at most ~256 chunks
  int64_t rows = 256;
  while (rows < kRowsMax && (k + rows - 1) / rows > 256) rows *= 2;
  return (int)rows;
}

}  // namespace smpm
