// Device-resident GMRES iteration for the deflated Schur complement system.
//
// One Arnoldi step j of right-preconditioned GMRES on P S M^{-1} (Algorithm 3,
// step 4) is six kernels, all reading j as a plain argument and per-column
// state from device memory, so the host never waits inside the loop:
//   gm_precond  v_j = w / beta (written into V), z = M^{-1} v_j
//   (Schur apply t = S z, coarse c2 = G Z^T t: operator kernels)
//   gm_orth1    w = t - Z c2 - S Z c2 (deflation), partial dots V^T w
//   gm_orth2    h1 = sum of partials; w -= V h1; partial dots V^T w
//   gm_orth3    h2 = ...; w -= V h2; partial |w|^2; the last block to finish
//               forms beta, the Hessenberg column h1 + h2, applies the Givens
//               rotations and retires the column when its residual estimate
//               reaches tol * beta_0.
// Partial sums are reduced by the last block of each kernel (atomic ticket per
// column) in a fixed order, so results are deterministic.  Each block handles
// a chunk of rows; its vectors' partial dots are reduced within a wavefront.
#include <hip/hip_runtime.h>

#include "smpm_gmres.h"

namespace smpm {

namespace {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;

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

// Partial sums written by other blocks are read after last_block()'s acquire
// fence, so ordinary loads see them.
__device__ __forceinline__ double load_agent(const double* p) { return *p; }

// Returns true in exactly one block per column: the last to arrive.  Partial
// results written before the call are visible to that block afterwards.
__device__ bool last_block(int* counter) {
  __shared__ int is_last;
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) {
    const int t = atomicAdd(counter, 1);
    is_last = (t == (int)gridDim.x - 1);
  }
  __syncthreads();
  if (is_last) __threadfence();
  return is_last != 0;
}

// Sum over chunks of part[i*nch + c] for i < nvec into out[i].  Wave q owns
// vector groups of eight; lanes take chunks lane, lane+64, ... and a fixed
// shuffle tree combines them, so the order of additions never changes.  Eight
// vectors are in flight per wave to hide the load latency.
__device__ void reduce_partials(const double* part, int nvec, int nch, double* out) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  for (int i0 = wave * 8; i0 < nvec; i0 += kWaves * 8) {
    double acc[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    for (int c = lane; c < nch; c += 64) {
#pragma unroll
      for (int u = 0; u < 8; ++u)
        if (i0 + u < nvec) acc[u] += load_agent(part + (int64_t)(i0 + u) * nch + c);
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const double v = wave_sum(acc[u]);
      if (lane == 0 && i0 + u < nvec) out[i0 + u] = v;
    }
  }
}

// Partial dots of the chunk held in LDS (wv, `rows` rows) with V_0..V_{nvec-1}:
// wave q handles vector groups q, q+4, ... of kDotUnroll vectors whose loads are
// all issued before the shuffle reductions; lanes run over rows.
constexpr int kDotUnroll = 8;
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

}  // namespace

// ------------------------------------------------------------------ kernels

// Finalizes v_j = w / beta into V_j and applies z = M^{-1} v_j (or z = v_j).
__global__ __launch_bounds__(256) void k_gm_precond(DevPlan P, GmState S, int j, int use_precond, int transpose) {
  __shared__ double xs[8 * kMaxN];
  const int col = blockIdx.y, tid = threadIdx.x;
  if (!S.active[col]) return;
  const double inv = 1.0 / S.beta_cur[col];
  const int64_t k = P.k;
  const double* wc = S.w + (int64_t)col * k;
  double* vj = S.V + (int64_t)j * S.vvs + (int64_t)col * k;
  double* zc = S.z + (int64_t)col * k;
  if (!use_precond) {
    for (int64_t x = (int64_t)blockIdx.x * kThreads + tid; x < k; x += (int64_t)gridDim.x * kThreads) {
      const double v = wc[x] * inv;
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
      const double v = wc[slot] * inv;
      xs[i] = v;
      vj[slot] = v;
    }
    __syncthreads();
    const double* Mp = (transpose ? P.MinvR : P.MinvC) + P.bcls_off[bc];
    for (int r = tid; r < sb; r += kThreads) {
      double acc = 0.0;
#pragma unroll 8
      for (int c = 0; c < sb; ++c) acc = fma(Mp[c * sb + r], xs[c], acc);
      zc[P.blk_slots[o + r]] = acc;
    }
  }
}

// w = t - (Z c2 + {S Z c2 | S^T Z c2}) on this block's rows (or w = t), then
// partial dots with V_0..V_j; the last block reduces them into h1.
__global__ __launch_bounds__(256) void k_gm_orth1(DevPlan P, GmState S, int j, int defl, int transpose) {
  __shared__ double wv[kRowsMax];
  const int col = blockIdx.y, chunk = blockIdx.x, tid = threadIdx.x;
  if (!S.active[col]) return;
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
  double* part = S.part1 + (int64_t)col * S.ldv * S.nch;
  chunk_dots(S.V + (int64_t)col * k, S.vvs, x0, rows, wv, j + 1, part, S.nch, chunk);
  if (last_block(S.counter + col * 4 + 0)) {
    reduce_partials(part, j + 1, S.nch, S.h1 + (int64_t)col * S.ldv);
    if (tid == 0) S.counter[col * 4 + 0] = 0;
  }
}

// w -= V h (h = h1 for pass 2, h2 for pass 3).  Pass 2 then forms partial dots
// (reduced into h2 by the last block); pass 3 forms |w|^2 and finishes the step.
template <int PASS>
__global__ __launch_bounds__(256) void k_gm_orth(DevPlan P, GmState S, int j) {
  __shared__ double wv[kRowsMax];
  __shared__ double hs[kMaxIt + 1];
  __shared__ double red[kWaves];
  const int col = blockIdx.y, chunk = blockIdx.x, tid = threadIdx.x;
  if (!S.active[col]) return;
  const int64_t k = P.k, x0 = (int64_t)chunk * S.rows;
  const int rows = (int)min((int64_t)S.rows, k - x0);
  const int nvec = j + 1;
  const double* hsrc = (PASS == 2 ? S.h1 : S.h2) + (int64_t)col * S.ldv;
  for (int i = tid; i < nvec; i += kThreads) hs[i] = hsrc[i];
  __syncthreads();
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
  if (PASS == 2) {
    double* part = S.part2 + (int64_t)col * S.ldv * S.nch;
    chunk_dots(Vc, S.vvs, x0, rows, wv, nvec, part, S.nch, chunk);
    if (last_block(S.counter + col * 4 + 1)) {
      reduce_partials(part, nvec, S.nch, S.h2 + (int64_t)col * S.ldv);
      if (tid == 0) S.counter[col * 4 + 1] = 0;
    }
    return;
  }
  const double bs = block_sum(nrm, red);
  double* part = S.part3 + (int64_t)col * S.nch;
  if (tid == 0) part[chunk] = bs;
  if (!last_block(S.counter + col * 4 + 2)) return;
  // ---- last block: beta, Hessenberg column, Givens rotations, convergence
  __shared__ double hc[kMaxIt + 2];
  __shared__ double csl[kMaxIt + 1], snl[kMaxIt + 1];
  __shared__ double beta_s;
  if (tid < 64) {
    double acc = 0.0;
    for (int c = tid; c < S.nch; c += 64) acc += load_agent(part + c);
    acc = wave_sum(acc);
    if (tid == 0) beta_s = sqrt(acc);
  }
  const double* h1 = S.h1 + (int64_t)col * S.ldv;
  double* csg = S.cs + (int64_t)col * S.ldv;
  double* sng = S.sn + (int64_t)col * S.ldv;
  for (int i = tid; i < nvec; i += kThreads) hc[i] = h1[i] + hs[i];
  for (int i = tid; i < j; i += kThreads) {
    csl[i] = csg[i];
    snl[i] = sng[i];
  }
  __syncthreads();
  if (tid == 0) {
    const double beta = beta_s;
    hc[j + 1] = beta;
    for (int i = 0; i < j; ++i) {
      const double a = hc[i], b = hc[i + 1];
      hc[i] = csl[i] * a + snl[i] * b;
      hc[i + 1] = -snl[i] * a + csl[i] * b;
    }
    const double a = hc[j], b = hc[j + 1];
    const double rr = hypot(a, b);
    const double c = rr > 0.0 ? a / rr : 1.0;
    const double s = rr > 0.0 ? b / rr : 0.0;
    hc[j] = rr;
    hc[j + 1] = 0.0;
    csg[j] = c;
    sng[j] = s;
    double* gc = S.g + (int64_t)col * S.ldv;
    const double gj = gc[j];
    gc[j + 1] = -s * gj;
    gc[j] = c * gj;
    const double res = fabs(gc[j + 1]);
    S.res[col] = res;
    S.iters[col] = j + 1;
    S.beta_cur[col] = beta;
    if (!(res > S.tolb[col]) || j + 1 >= S.maxit || !(beta > 0.0)) S.active[col] = 0;
    S.counter[col * 4 + 2] = 0;
  }
  __syncthreads();
  double* Hcol = S.H + (int64_t)col * S.ldv * S.maxit + (int64_t)j * S.ldv;
  for (int i = tid; i <= j; i += kThreads) Hcol[i] = hc[i];
}

// Start of a solve: beta_0 = |w|, g = beta_0 e_1, per-column activity.
__global__ __launch_bounds__(256) void k_gm_start(DevPlan P, GmState S, double tol) {
  __shared__ double red[kWaves];
  const int col = blockIdx.y, chunk = blockIdx.x, tid = threadIdx.x;
  const int64_t k = P.k, x0 = (int64_t)chunk * S.rows;
  const int rows = (int)min((int64_t)S.rows, k - x0);
  const double* wc = S.w + (int64_t)col * k;
  double nrm = 0.0;
  for (int q = tid; q < rows; q += kThreads) nrm = fma(wc[x0 + q], wc[x0 + q], nrm);
  const double bs = block_sum(nrm, red);
  double* part = S.part3 + (int64_t)col * S.nch;
  if (tid == 0) part[chunk] = bs;
  if (!last_block(S.counter + col * 4 + 3)) return;
  if (tid < 64) {
    double acc = 0.0;
    for (int c = tid; c < S.nch; c += 64) acc += load_agent(part + c);
    acc = wave_sum(acc);
    if (tid != 0) return;
    const double beta = sqrt(acc);
    S.beta_cur[col] = beta;
    S.beta0[col] = beta;
    S.tolb[col] = tol * beta;
    S.res[col] = beta;
    S.iters[col] = 0;
    S.active[col] = beta > 0.0 ? 1 : 0;
    S.g[(int64_t)col * S.ldv] = beta;
    S.counter[col * 4 + 3] = 0;
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

__global__ void k_fill_int(int* p, int v, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// ------------------------------------------------------------------ launchers

void gm_start(const DevPlan& P, const GmState& S, int nrhs, double tol, hipStream_t s) {
  hipLaunchKernelGGL(k_gm_start, dim3(S.nch, nrhs), dim3(kThreads), 0, s, P, S, tol);
}

void gm_step(const DevPlan& P, const GmState& S, int nrhs, int j, int kind, bool tr, hipStream_t s) {
  const int pre_grid = kind == 1 ? S.nch : std::max(1, std::min(P.nblk, 1024));
  hipLaunchKernelGGL(k_gm_precond, dim3(pre_grid, nrhs), dim3(kThreads), 0, s, P, S, j, kind == 1 ? 0 : 1,
                     tr ? 1 : 0);
  launch_schur(P, S.z, S.t, nrhs, tr, S.active, s);
  if (kind == 3) {
    launch_iface_sum(P, S.t, S.c, nrhs, S.active, s);
    launch_coarse(P, S.c, S.c2, nrhs, tr, S.active, s);
  }
  hipLaunchKernelGGL(k_gm_orth1, dim3(S.nch, nrhs), dim3(kThreads), 0, s, P, S, j, kind == 3 ? 1 : 0,
                     tr ? 1 : 0);
  hipLaunchKernelGGL(k_gm_orth<2>, dim3(S.nch, nrhs), dim3(kThreads), 0, s, P, S, j);
  hipLaunchKernelGGL(k_gm_orth<3>, dim3(S.nch, nrhs), dim3(kThreads), 0, s, P, S, j);
}

void gm_finish(const DevPlan& P, const GmState& S, int nrhs, double* x, hipStream_t s) {
  hipLaunchKernelGGL(k_gm_lsq, dim3(nrhs), dim3(kThreads), 0, s, S);
  const int64_t blocks = std::min<int64_t>((P.k + kThreads - 1) / kThreads, 2048);
  hipLaunchKernelGGL(k_gm_combine, dim3((unsigned)blocks, nrhs), dim3(kThreads), 0, s, P, S, x);
}

void gm_reset_counters(int* counter, int n, hipStream_t s) {
  hipLaunchKernelGGL(k_fill_int, dim3((n + 255) / 256), dim3(256), 0, s, counter, 0, n);
}

int gm_rows_per_chunk(int64_t k) {
  // chunks of 256..kRowsMax rows, at most ~256 chunks
  int64_t rows = 256;
  while (rows < kRowsMax && (k + rows - 1) / rows > 256) rows *= 2;
  return (int)rows;
}

}  // namespace smpm
