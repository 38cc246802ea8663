// Block GMRES kernels (see smpm_block.h).  The block Krylov method is not in the
// paper; it solves Algorithm 3's step 4 for all right-hand sides in one space.
#include "smpm_block.h"

#include <algorithm>
#include <atomic>
#include <type_traits>

namespace smpm {

namespace {

typedef double bg_v4d __attribute__((ext_vector_type(4)));

// 16x16x4 FP64 matrix-core step.  Lane l supplies A[l % 16][l / 16] and B[l / 16][l % 16]
// and holds C[(l / 16) + 4 v][l % 16] in register v.
__device__ __forceinline__ bg_v4d bg_mma(double a, double b, bg_v4d c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Lane move of a double by a DPP control (both 32-bit halves)
template <int CTRL>
__device__ __forceinline__ double dpp_move(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xf, 0xf, false);
  return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double read_lane(double v, int l) {
  return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), l),
                          __builtin_amdgcn_readlane(__double2loint(v), l));
}

// Sum over the 64 lanes, the same value on every lane.  Inside each row of 16 lanes a
// butterfly on DPP lane moves (partners lane ^ 1, lane ^ 2, then the half-row and row
// mirrors, 7 - i and 15 - i), then the four row sums are read as scalars.  Every lane
// of the wavefront must be active.
__device__ __forceinline__ double wave_sum(double v) {
  v += dpp_move<0xB1>(v);   // quad permutation 1 0 3 2
  v += dpp_move<0x4E>(v);   // quad permutation 2 3 0 1
  v += dpp_move<0x141>(v);  // half-row mirror
  v += dpp_move<0x140>(v);  // row mirror
  return (read_lane(v, 0) + read_lane(v, 16)) + (read_lane(v, 32) + read_lane(v, 48));
}

constexpr int kTargetBlocks = 2048;  // workgroups a dot launch aims for
constexpr int kMinChunk = 256;       // shortest x chunk of a dot workgroup

void dot_chunks(int64_t len, int na, int* nch, int64_t* per, int target = kTargetBlocks) {
  const int64_t ablk = (na + 63) / 64;
  int64_t want = std::max<int64_t>(1, target / ablk);
  want = std::min<int64_t>(want, std::max<int64_t>(1, (len + kMinChunk - 1) / kMinChunk));
  int64_t p = (len + want - 1) / want;
  p = (p + 63) / 64 * 64;
  *per = p;
  *nch = (int)((len + p - 1) / p);
}

// Partial sums of A^T B over one x chunk.  Work items (chunk, 64 rows of A) are
// chunk-major and every XCD takes a contiguous range of them (workgroup w runs on
// XCD w % 8), so the row groups of one chunk share that XCD's L2 copy of B's chunk.
// The chunk is walked 64 entries at a time: the 64 A rows and the (<= 32) B columns
// of the step go to LDS as whole 512-byte row segments (every load issued before the
// first store, clamped into the vectors and masked), then wavefront w multiplies
// its 16 A rows against both 16-column B tiles in 16 matrix-core steps (step q takes
// entries 4q .. 4q+3).  part[(b * na + a) * nch + chunk].
constexpr int kDotLd = 68;  // LDS row stride in elements (rows land apart in the banks)
// BR: B rows loaded (8, 16 or 32; with 8 the lanes of tile columns 8 .. 15 feed zeros
// to the matrix cores instead of reading LDS); A is staged in its own precision
template <typename AT, int BR>
__global__ __launch_bounds__(256) void k_bg_dot(const AT* __restrict__ A, int na, const double* __restrict__ B,
                                                int nb, int64_t len, int64_t per, int nch, int items,
                                                double* __restrict__ part) {
  __shared__ AT As[64 * kDotLd];
  __shared__ double Bs[BR * kDotLd];
  const int ablk = (na + 63) / 64;
  const int per_xcd = (int)(gridDim.x / 8);
  const int item = (int)(blockIdx.x % 8) * per_xcd + (int)(blockIdx.x / 8);
  if (item >= items) return;  // uniform over the workgroup
  const int chunk = item / ablk, ab = item - chunk * ablk;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int64_t x0 = (int64_t)chunk * per;
  const int64_t x1 = min(len, x0 + per);
  const bool two = BR > 16 && nb > 16;
  const bool active = ab * 64 + wave * 16 < na;
  bg_v4d acc0 = {0.0, 0.0, 0.0, 0.0}, acc1 = {0.0, 0.0, 0.0, 0.0};
  for (int64_t xb = x0; xb < x1; xb += 64) {
    const int64_t gx = xb + lane;
    const bool xok = gx < x1;
    const int64_t xc = xok ? gx : x0;
    AT av[16];
    double bv[BR / 4];
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      const int ar = ab * 64 + wave + 4 * i;
      av[i] = A[(int64_t)(ar < na ? ar : 0) * len + xc];
    }
#pragma unroll
    for (int i = 0; i < BR / 4; ++i) {
      const int br = wave + 4 * i;
      bv[i] = B[(int64_t)(br < nb ? br : 0) * len + xc];
    }
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      const int row = wave + 4 * i;
      As[row * kDotLd + lane] = xok && ab * 64 + row < na ? av[i] : AT(0);
    }
#pragma unroll
    for (int i = 0; i < BR / 4; ++i) {
      const int row = wave + 4 * i;
      Bs[row * kDotLd + lane] = xok && row < nb ? bv[i] : 0.0;
    }
    __syncthreads();
    if (active) {
      const AT* ar = As + (wave * 16 + (lane & 15)) * kDotLd + (lane >> 4);
      const bool bz = BR < 16 && (lane & 15) >= BR;  // tile column past the loaded rows
      const double* b0 = Bs + ((lane & 15) % BR) * kDotLd + (lane >> 4);
      const double* b1 = Bs + ((BR > 16 ? 16 : 0) + (lane & 15)) * kDotLd + (lane >> 4);
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        const double a = (double)ar[4 * q];
        acc0 = bg_mma(a, bz ? 0.0 : b0[4 * q], acc0);
        if (two) acc1 = bg_mma(a, b1[4 * q], acc1);
      }
    }
    __syncthreads();
  }
  if (!active) return;
  const int a0 = ab * 64 + wave * 16, bc = lane & 15;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int a = a0 + (lane >> 4) + 4 * v;
    if (a >= na) continue;
    if (bc < nb) part[((int64_t)bc * na + a) * nch + chunk] = acc0[v];
    if (two && 16 + bc < nb) part[((int64_t)(16 + bc) * na + a) * nch + chunk] = acc1[v];
  }
}

// A^T B for na <= 16 (the Gram matrices of a block): 16 A rows are staged, and the
// four wavefronts split every 64-entry step (wavefront w takes entries 16w .. 16w+15
// in four matrix-core steps), each keeping its own sums: part[(b * na + a) * nch + 4
// chunk + w] with nch four times the chunk count.
template <typename AT, int BR>
__global__ __launch_bounds__(256) void k_bg_dot16(const AT* __restrict__ A, int na, const double* __restrict__ B,
                                                  int nb, int64_t len, int64_t per, int nch4, int items,
                                                  double* __restrict__ part) {
  __shared__ AT As[16 * kDotLd];
  __shared__ double Bs[BR * kDotLd];
  const int per_xcd = (int)(gridDim.x / 8);
  const int chunk = (int)(blockIdx.x % 8) * per_xcd + (int)(blockIdx.x / 8);
  if (chunk >= items) return;  // uniform over the workgroup
  const int tid = threadIdx.x, wave = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
  const int64_t x0 = (int64_t)chunk * per;
  const int64_t x1 = min(len, x0 + per);
  const bool two = BR > 16 && nb > 16;
  bg_v4d acc0 = {0.0, 0.0, 0.0, 0.0}, acc1 = {0.0, 0.0, 0.0, 0.0};
  for (int64_t xb = x0; xb < x1; xb += 64) {
    const int64_t gx = xb + lane;
    const bool xok = gx < x1;
    const int64_t xc = xok ? gx : x0;
    AT av[4];
    double bv[BR / 4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int ar = wave + 4 * i;
      av[i] = A[(int64_t)(ar < na ? ar : 0) * len + xc];
    }
#pragma unroll
    for (int i = 0; i < BR / 4; ++i) {
      const int br = wave + 4 * i;
      bv[i] = B[(int64_t)(br < nb ? br : 0) * len + xc];
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int row = wave + 4 * i;
      As[row * kDotLd + lane] = xok && row < na ? av[i] : AT(0);
    }
#pragma unroll
    for (int i = 0; i < BR / 4; ++i) {
      const int row = wave + 4 * i;
      Bs[row * kDotLd + lane] = xok && row < nb ? bv[i] : 0.0;
    }
    __syncthreads();
    {
      const int e0 = 16 * wave + (lane >> 4);
      const AT* ar = As + (lane & 15) * kDotLd + e0;
      const double* b0 = Bs + (lane & 15) * kDotLd + e0;
      const double* b1 = Bs + ((BR > 16 ? 16 : 0) + (lane & 15)) * kDotLd + e0;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const double a = (double)ar[4 * q];
        acc0 = bg_mma(a, b0[4 * q], acc0);
        if (two) acc1 = bg_mma(a, b1[4 * q], acc1);
      }
    }
    __syncthreads();
  }
  const int bc = lane & 15, slot = 4 * chunk + wave;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int a = (lane >> 4) + 4 * v;
    if (a >= na) continue;
    if (bc < nb) part[((int64_t)bc * na + a) * nch4 + slot] = acc0[v];
    if (two && 16 + bc < nb) part[((int64_t)(16 + bc) * na + a) * nch4 + slot] = acc1[v];
  }
}

// One wavefront per output: lanes take the chunks c = lane, lane + 64, ... in order,
// then a fixed butterfly.  out[b * ldo + a] (and, with outT, outT[a * kBgMaxCols + b]).
__global__ __launch_bounds__(256) void k_bg_dot_final(const double* __restrict__ part, int na, int nb, int nch,
                                                      double* __restrict__ out, int ldo, double beta,
                                                      double* __restrict__ outT) {
  const int o = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (o >= na * nb) return;
  const int a = o % na, b = o / na;
  const double* p = part + (int64_t)o * nch;
  double acc = 0.0;
  for (int c = lane; c < nch; c += 64) acc += p[c];
  acc = wave_sum(acc);
  if (lane == 0) {
    double* d = out + (int64_t)b * ldo + a;
    const double v = beta != 0.0 ? beta * *d + acc : acc;
    *d = v;
    if (outT) outT[(int64_t)a * kBgMaxCols + b] = v;
  }
}

// out = beta win + alpha A H: workgroup of four wavefronts, each 16 consecutive x
// against all (<= 32) columns; the contraction runs over the na vectors of A in
// groups of 16 (four matrix-core steps, a = ab + 4q + l/16).
template <typename AT, typename OT>
__global__ __launch_bounds__(256) void k_bg_update(const AT* __restrict__ A, int na, const double* __restrict__ H,
                                                   int64_t sa, int64_t sb, double alpha, const OT* win,
                                                   double beta, OT* out, int nb, int64_t len) {
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const int64_t x0 = ((int64_t)blockIdx.x * 4 + wave) * 16;
  if (x0 >= len) return;
  const int64_t xr = x0 + (lane & 15);
  const int64_t xc = xr < len ? xr : x0;
  const int kq = lane >> 4, bc = lane & 15;
  const bool two = nb > 16;
  const bool b0ok = bc < nb, b1ok = 16 + bc < nb;
  const double* h0 = H + (b0ok ? bc : 0) * sb;
  const double* h1 = H + (b1ok ? 16 + bc : 0) * sb;
  bg_v4d acc0 = {0.0, 0.0, 0.0, 0.0}, acc1 = {0.0, 0.0, 0.0, 0.0};
  for (int ab = 0; ab < na; ab += 16) {
    double av[4], hv0[4], hv1[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int a = ab + 4 * q + kq;
      const int ac = a < na ? a : 0;
      av[q] = (double)A[(int64_t)ac * len + xc];
      hv0[q] = h0[ac * sa];
      hv1[q] = two ? h1[ac * sa] : 0.0;
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const bool ok = ab + 4 * q + kq < na;
      const double a = ok ? av[q] : 0.0;
      acc0 = bg_mma(a, b0ok ? hv0[q] : 0.0, acc0);
      if (two) acc1 = bg_mma(a, b1ok ? hv1[q] : 0.0, acc1);
    }
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int64_t x = x0 + (lane >> 4) + 4 * v;
    if (x >= len) continue;
    if (b0ok) {
      const int64_t o = (int64_t)bc * len + x;
      out[o] = (OT)(beta != 0.0 ? beta * (double)win[o] + alpha * acc0[v] : alpha * acc0[v]);
    }
    if (two && b1ok) {
      const int64_t o = (int64_t)(16 + bc) * len + x;
      out[o] = (OT)(beta != 0.0 ? beta * (double)win[o] + alpha * acc1[v] : alpha * acc1[v]);
    }
  }
}

// The same product for an FP32 A over an even length: each wavefront takes 32
// consecutive entries, lane m the pair x0 + 2m, x0 + 2m + 1 with one 8-byte load (so a
// row load covers a whole 128-byte line), and runs the even entries and the odd ones
// as two matrix-core tiles.
template <typename OT, bool TWO>
__global__ __launch_bounds__(256) void k_bg_update_f2(const float* __restrict__ A, int na,
                                                      const double* __restrict__ H, int64_t sa, int64_t sb,
                                                      double alpha, const OT* win, double beta, OT* out, int nb,
                                                      int64_t len) {
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const int64_t x0 = ((int64_t)blockIdx.x * 4 + wave) * 32;
  if (x0 >= len) return;
  const int64_t xp = x0 + 2 * (lane & 15);  // even, and len is even: xp < len covers the pair
  const bool pok = xp < len;
  const int64_t xc = pok ? xp : x0;
  const int kq = lane >> 4, bc = lane & 15;
  const bool two = TWO && nb > 16;  // a second 16-column tile (TWO false: none, fewer registers)
  const bool b0ok = bc < nb, b1ok = 16 + bc < nb;
  const double* h0 = H + (b0ok ? bc : 0) * sb;
  const double* h1 = H + (b1ok ? 16 + bc : 0) * sb;
  bg_v4d e0 = {0.0, 0.0, 0.0, 0.0}, o0 = {0.0, 0.0, 0.0, 0.0};
  bg_v4d e1 = {0.0, 0.0, 0.0, 0.0}, o1 = {0.0, 0.0, 0.0, 0.0};
  for (int ab = 0; ab < na; ab += 16) {
    float2 av[4];
    double hv0[4], hv1[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int a = ab + 4 * q + kq;
      const int ac = a < na ? a : 0;
      av[q] = *reinterpret_cast<const float2*>(A + (int64_t)ac * len + xc);
      hv0[q] = h0[ac * sa];
      hv1[q] = two ? h1[ac * sa] : 0.0;
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const bool ok = pok && ab + 4 * q + kq < na;
      const double ae = ok ? (double)av[q].x : 0.0, ao = ok ? (double)av[q].y : 0.0;
      const double g0 = b0ok ? hv0[q] : 0.0;
      e0 = bg_mma(ae, g0, e0);
      o0 = bg_mma(ao, g0, o0);
      if (two) {
        const double g1 = b1ok ? hv1[q] : 0.0;
        e1 = bg_mma(ae, g1, e1);
        o1 = bg_mma(ao, g1, o1);
      }
    }
  }
  auto put = [&](int b, int64_t x, double v) {
    const int64_t o = (int64_t)b * len + x;
    out[o] = (OT)(beta != 0.0 ? beta * (double)win[o] + alpha * v : alpha * v);
  };
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int64_t xe = x0 + 2 * ((lane >> 4) + 4 * v);
    if (xe >= len) continue;  // len even: the odd partner is in range too
    if (b0ok) {
      put(bc, xe, e0[v]);
      put(bc, xe + 1, o0[v]);
    }
    if (two && b1ok) {
      put(16 + bc, xe, e1[v]);
      put(16 + bc, xe + 1, o1[v]);
    }
  }
}

// The same product for an FP32 A, an even length and at most 8 columns, on FP64
// vector FMAs: a 16-column matrix-core tile would spend half its products on absent
// columns, and the vector units have the same FP64 rate.  Lane m takes the pair
// 2m, 2m + 1 of its workgroup's 512 entries (one 8-byte load per row) and keeps both
// entries' sums for every column; H is read as scalars (uniform over the
// wavefront).  Each sum runs over the rows of A in increasing order.
template <typename OT>
__global__ __launch_bounds__(256) void k_bg_update_v8(const float* __restrict__ A, int na,
                                                      const double* __restrict__ H, int64_t sa, int64_t sb,
                                                      double alpha, const OT* win, double beta, OT* out, int nb,
                                                      int64_t len) {
  const int64_t xp = ((int64_t)blockIdx.x * 256 + threadIdx.x) * 2;
  if (xp >= len) return;  // len even: xp + 1 < len as well
  double e[8], o[8];
#pragma unroll
  for (int b = 0; b < 8; ++b) e[b] = o[b] = 0.0;
  auto rows = [&](const float2* av, int a0, int cnt) {
    for (int u = 0; u < cnt; ++u) {
      const double ae = (double)av[u].x, ao = (double)av[u].y;
      const double* hr = H + (int64_t)(a0 + u) * sa;
#pragma unroll
      for (int b = 0; b < 8; ++b) {
        const double h = b < nb ? hr[b * sb] : 0.0;
        e[b] = fma(ae, h, e[b]);
        o[b] = fma(ao, h, o[b]);
      }
    }
  };
  int a = 0;
  for (; a + 8 <= na; a += 8) {
    float2 av[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) av[u] = *reinterpret_cast<const float2*>(A + (int64_t)(a + u) * len + xp);
    rows(av, a, 8);
  }
  for (; a < na; ++a) {
    const float2 av = *reinterpret_cast<const float2*>(A + (int64_t)a * len + xp);
    rows(&av, a, 1);
  }
#pragma unroll
  for (int b = 0; b < 8; ++b) {
    if (b >= nb) break;
    const int64_t q = (int64_t)b * len + xp;
    out[q] = (OT)(beta != 0.0 ? beta * (double)win[q] + alpha * e[b] : alpha * e[b]);
    out[q + 1] = (OT)(beta != 0.0 ? beta * (double)win[q + 1] + alpha * o[b] : alpha * o[b]);
  }
}

// Cholesky QR pass (one workgroup; see launch_bg_chol), right-looking: once column i
// yields a vector, the remaining Gram entries and the remaining columns' coefficient
// vectors (Es column l = e_l minus its parts on the kept vectors) are updated at once.
// As[i + 32 j]: Gram matrix being reduced, Gd: its original diagonal, Rs[c + 32 l] =
// R_cl, Ts[i + 32 c] = T_ic.
__global__ __launch_bounds__(256) void k_bg_chol(const double* __restrict__ G, int m, double drop,
                                                 const int* __restrict__ cnt_in, const double* __restrict__ rprev,
                                                 int* __restrict__ cnt, double* __restrict__ T,
                                                 double* __restrict__ R) {
  constexpr int C = kBgMaxCols;
  __shared__ double As[C * C], Es[C * C], Rs[C * C], Ts[C * C], Gd[C];
  const int tid = threadIdx.x;
  const int mm = cnt_in ? min(*cnt_in, m) : m;
  for (int q = tid; q < C * C; q += 256) {
    const int i = q % C, j = q / C;
    As[q] = i < m && j < m ? G[i + m * j] : 0.0;
    Es[q] = i == j ? 1.0 : 0.0;
    Rs[q] = 0.0;
    Ts[q] = 0.0;
  }
  if (tid < C) Gd[tid] = tid < m ? G[tid + m * tid] : 0.0;
  __syncthreads();
  int kept = 0;
  for (int i = 0; i < mm; ++i) {
    const double d = As[i + C * i], gii = Gd[i];
    // NaN fails every comparison: such a column is dropped
    const bool keep = gii > 0.0 && d > 0.0 && d > drop * drop * gii;
    if (!keep) continue;  // uniform over the workgroup
    const double rho = sqrt(d);
    if (tid < C) {
      const int l = tid;
      if (l > i && l < mm) Rs[kept + C * l] = As[i + C * l] / rho;
      if (l == i) Rs[kept + C * l] = rho;
      if (l < m) Ts[l + C * kept] = Es[l + C * i] / rho;
    }
    __syncthreads();
    for (int q = tid; q < C * C; q += 256) {
      const int u = q % C, l = q / C;
      if (l > i && l < mm) {
        if (u > i && u < mm) As[u + C * l] -= Rs[kept + C * u] * Rs[kept + C * l];
        if (u < m) Es[u + C * l] -= Rs[kept + C * l] * Ts[u + C * kept];
      }
    }
    ++kept;
    __syncthreads();
  }
  if (tid == 0) *cnt = kept;
  for (int q = tid; q < m * m; q += 256) T[q] = Ts[(q % m) + C * (q / m)];
  for (int q = tid; q < C * C; q += 256) {
    const int c = q % C, i = q / C;
    double v = 0.0;
    if (c < kept && i < m) {
      if (rprev) {
        for (int cp = 0; cp < mm; ++cp) v += Rs[c + C * cp] * rprev[cp + C * i];
      } else {
        v = Rs[c + C * i];
      }
    }
    R[q] = v;
  }
}

constexpr int kLsqWaves = 16;  // wavefronts of the least-squares kernel

// Block step of the Householder least-squares update (one workgroup, 16 wavefronts).
// Work slots: the r new columns of Hbar, then the s columns of G; wavefront w owns
// slots w, w + 16, w + 32, w + 48.  A slot keeps a 64-row window of its column in
// registers, row rho in lane rho % 64, so a reflection of rows p .. p+63 is one
// multiply-add and one wavefront sum per lane; when p advances, the row leaving the
// window is stored and the row entering it loaded.  Reflections are at most 64 rows
// long (a column's rows below its diagonal are the r + cnt of its block step).
__global__ __launch_bounds__(64 * kLsqWaves) void k_bg_lsq(BgLsq L, int n0, int r, int nv,
                                                          const double* __restrict__ h, int ldh,
                                                          const double* __restrict__ R, const int* __restrict__ cnts,
                                                          double* host_res, int* host_cnt) {
  __shared__ double vsh[64];
  __shared__ double bsh;
  __shared__ double rgrp[64 * 64], bgrp[64];  // 64 earlier reflections at a time
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int cnt = cnts[1];
  const int rows = nv + cnt;
  const int s = L.s;
  const int64_t ld = L.ldH;
  // the new columns of Hbar
  for (int q = tid; q < r * rows; q += 64 * kLsqWaves) {
    const int c = q / rows, row = q % rows;
    L.H[(int64_t)(n0 + c) * ld + row] = row < nv ? h[(int64_t)c * ldh + row] : R[(row - nv) + kBgMaxCols * c];
  }
  __syncthreads();
  const int nslot = r + s;
  double* col[4];
  double reg[4];
  bool own[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int q = wave + kLsqWaves * u;
    own[u] = q < nslot;
    col[u] = q < r ? L.H + (int64_t)(n0 + q) * ld : L.G + (int64_t)(own[u] ? q - r : 0) * ld;
    // H slots start their window at row 0, G slots at row n0 (earlier reflections
    // were applied to G in earlier steps)
    const int base = q < r ? 0 : n0;
    const int row = base + ((lane - base) & 63);
    reg[u] = own[u] && row < rows ? col[u][row] : 0.0;
  }
  // advance the window of slot u past row p, to the row loaded ahead into nxt[u]
  double nxt[4] = {0.0, 0.0, 0.0, 0.0};
  auto advance = [&](int u, int p) {
    if (lane == (p & 63)) {
      col[u][p] = reg[u];
      reg[u] = nxt[u];
    }
  };
  // earlier reflections on the new columns, 64 at a time: the group's reflection
  // vectors and factors are staged in LDS by the whole workgroup, and the rows
  // entering the windows during the group are loaded at once (row p0 + 64 + lane)
  for (int p = 0; p < n0; ++p) {
    if ((p & 63) == 0) {
      __syncthreads();  // the previous group's reflections are applied
      const int ng = min(64, n0 - p);
      for (int i = tid; i < 64 * 64; i += 64 * kLsqWaves)
        rgrp[i] = i < ng * 64 ? L.refl[(int64_t)p * 64 + i] : 0.0;
      if (tid < 64) bgrp[tid] = tid < ng ? L.rbeta[p + tid] : 0.0;
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int q = wave + kLsqWaves * u;
        const int row = p + 64 + lane;
        nxt[u] = own[u] && q < r && row < rows ? col[u][row] : 0.0;
      }
      __syncthreads();
    }
    const double v = rgrp[(p & 63) * 64 + ((lane - p) & 63)];
    const double be = bgrp[p & 63];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int q = wave + kLsqWaves * u;
      if (!own[u] || q >= r) continue;
      if (be != 0.0) {
        const double dt = wave_sum(v * reg[u]);
        reg[u] -= be * dt * v;
      }
      if (lane == (p & 63)) {
        col[u][p] = reg[u];
        reg[u] = nxt[u];
      }
    }
  }
  // the new columns' own reflections, applied to the later new columns and to G.  The
  // windows hold rows n0 .. n0+63 (lane l row n0 + ((l - n0) & 63)); the rows entering
  // them during these r < 64 steps are p + 64 for p < n0 + r, which nothing here
  // writes, so they are loaded at once
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int pl = n0 + ((lane - n0) & 63);
    nxt[u] = own[u] && pl < n0 + r && pl + 64 < rows ? col[u][pl + 64] : 0.0;
  }
  for (int c = 0; c < r; ++c) {
    const int p = n0 + c;
    const int t = (lane - p) & 63;
    const int len = rows - p;
    if (wave == c % kLsqWaves) {
      const int u = c / kLsqWaves;
      const double x = t < len ? reg[u] : 0.0;
      const double sig = wave_sum(t >= 1 ? x * x : 0.0);
      const double x0 = __shfl(x, p & 63);
      double v = 0.0, be = 0.0, alpha = x0;
      if (sig > 0.0) {
        const double nrm = sqrt(x0 * x0 + sig);
        alpha = x0 >= 0.0 ? -nrm : nrm;
        const double v0 = x0 - alpha;
        v = t == 0 ? v0 : x;
        be = 2.0 / (v0 * v0 + sig);
      }
      vsh[t] = v;
      if (lane == 0) bsh = be;
      L.refl[(int64_t)p * 64 + t] = v;
      if (lane == 0) L.rbeta[p] = be;
      if (lane == (p & 63)) col[u][p] = alpha;
    }
    __syncthreads();
    const double v = vsh[t];
    const double be = bsh;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int q = wave + kLsqWaves * u;
      if (!own[u] || q <= c) continue;
      if (be != 0.0) {
        const double dt = wave_sum(v * reg[u]);
        reg[u] -= be * dt * v;
      }
      advance(u, p);
    }
    __syncthreads();  // vsh is rewritten by the next column
  }
  // G: store the window (rows nv .. rows-1 hold the residual block) and the residuals
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int q = wave + kLsqWaves * u;
    if (!own[u] || q < r) continue;
    const int row = nv + ((lane - nv) & 63);
    if (row < rows) col[u][row] = reg[u];
    const double rs = sqrt(wave_sum(row < rows ? reg[u] * reg[u] : 0.0));
    if (lane == 0) {
      L.res[q - r] = rs;
      host_res[q - r] = rs;
    }
  }
  if (tid == 0) {
    host_cnt[0] = cnts[0];
    host_cnt[1] = cnt;
  }
}

// Y = triangle(H)^{-1} G[0 .. ncol) by blocks of 32 rows from the bottom (one
// workgroup): a block's triangle and right-hand sides are solved in LDS, then the
// rows above it are updated with the block's solution.
__global__ __launch_bounds__(1024) void k_bg_backsolve(BgLsq L, int ncol, double* __restrict__ Y, int ldy) {
  constexpr int C = kBgMaxCols;
  __shared__ double tri[C * (C + 1)], yb[C * (C + 1)];  // tri[r + 33 c] = H[i0 + r][i0 + c], yb[r + 33 g]
  const int tid = threadIdx.x;
  const int s = L.s;
  const int64_t ld = L.ldH;
  for (int q = tid; q < ncol * s; q += 1024) {
    const int row = q % ncol, g = q / ncol;
    Y[(int64_t)g * ldy + row] = L.G[(int64_t)g * ld + row];
  }
  __syncthreads();
  for (int i1 = ncol; i1 > 0; i1 -= C) {
    const int i0 = max(0, i1 - C), nb = i1 - i0;
    for (int q = tid; q < C * C; q += 1024) {
      const int r = q % C, c = q / C;
      tri[r + (C + 1) * c] = r < nb && c < nb && r <= c ? L.H[(int64_t)(i0 + c) * ld + i0 + r] : 0.0;
      yb[r + (C + 1) * c] = r < nb && c < s ? Y[(int64_t)c * ldy + i0 + r] : 0.0;
    }
    __syncthreads();
    for (int rr = nb - 1; rr >= 0; --rr) {
      if (tid < s) {
        const double dg = tri[rr + (C + 1) * rr];
        yb[rr + (C + 1) * tid] = dg != 0.0 ? yb[rr + (C + 1) * tid] / dg : 0.0;
      }
      __syncthreads();
      if (tid < rr * s) {
        const int r = tid % rr, g = tid / rr;
        yb[r + (C + 1) * g] -= tri[r + (C + 1) * rr] * yb[rr + (C + 1) * g];
      }
      __syncthreads();
    }
    for (int q = tid; q < nb * s; q += 1024) {
      const int r = q % nb, g = q / nb;
      Y[(int64_t)g * ldy + i0 + r] = yb[r + (C + 1) * g];
    }
    for (int q = tid; q < i0 * s; q += 1024) {
      const int row = q % i0, g = q / i0;
      double acc = 0.0;
      for (int c = 0; c < nb; ++c) acc += L.H[(int64_t)(i0 + c) * ld + row] * yb[c + (C + 1) * g];
      Y[(int64_t)g * ldy + row] -= acc;
    }
    __syncthreads();
  }
}

__global__ void k_bg_widen(const float* __restrict__ a, double* __restrict__ b, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = (double)a[i];
}

__global__ void k_bg_lsq_start(BgLsq L, const double* __restrict__ R0, const int* __restrict__ m) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= L.ldH * L.s) return;
  const int row = (int)(idx % L.ldH), g = (int)(idx / L.ldH);
  L.G[idx] = row < *m ? R0[row + kBgMaxCols * g] : 0.0;
}

}  // namespace

int64_t bg_dot_part_size() { return (int64_t)(kTargetBlocks + 64) * 64 * kBgMaxCols; }

constexpr int kMaxDevices = 64;

// Workgroup count a k_bg_dot<AT, BR> launch aims for: the largest whole number of
// rounds of the workgroups the device holds at once that fits in kTargetBlocks (a
// partial last round leaves most of the chip idle at the end).  Per device, computed
// once; kTargetBlocks where the query fails.
template <typename AT, int BR>
int dot_target() {
  static std::atomic<int> cache[kMaxDevices];
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return kTargetBlocks;
  int t = cache[dev].load(std::memory_order_relaxed);
  if (t == 0) {
    int per_cu = 0, ncu = 0;
    t = kTargetBlocks;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_bg_dot<AT, BR>, 256, 0) == hipSuccess &&
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess) {
      const int cap = per_cu * ncu;
      if (cap > 0 && cap <= kTargetBlocks) t = kTargetBlocks / cap * cap;
    }
    cache[dev].store(t, std::memory_order_relaxed);
  }
  return t;
}

template <typename AT>
void launch_bg_dot(const AT* A, int na, const double* B, int nb, int64_t len, double* part, double* out, int ldo,
                   double beta, hipStream_t s, double* outT) {
  if (na <= 0 || nb <= 0) return;
  int nch;
  int64_t per;
  const int tot = na * nb;
  if (na <= 16) {
    // the four wavefronts split each step; their sums stay apart (4 nch partial sums,
    // so a quarter of the chunks)
    dot_chunks(len, na, &nch, &per, kTargetBlocks / 4);
    const int grid16 = (nch + 7) / 8 * 8;
    if (nb <= 16)
      hipLaunchKernelGGL((k_bg_dot16<AT, 16>), dim3(grid16), dim3(256), 0, s, A, na, B, nb, len, per, 4 * nch, nch,
                         part);
    else
      hipLaunchKernelGGL((k_bg_dot16<AT, 32>), dim3(grid16), dim3(256), 0, s, A, na, B, nb, len, per, 4 * nch, nch,
                         part);
    hipLaunchKernelGGL(k_bg_dot_final, dim3((tot + 3) / 4), dim3(256), 0, s, part, na, nb, 4 * nch, out, ldo, beta,
                       outT);
    return;
  }
  const int target = nb <= 8 ? dot_target<AT, 8>() : nb <= 16 ? dot_target<AT, 16>() : dot_target<AT, 32>();
  dot_chunks(len, na, &nch, &per, target);
  const int items = nch * ((na + 63) / 64);
  const int grid = (items + 7) / 8 * 8;
  if (nb <= 8)
    hipLaunchKernelGGL((k_bg_dot<AT, 8>), dim3(grid), dim3(256), 0, s, A, na, B, nb, len, per, nch, items, part);
  else if (nb <= 16)
    hipLaunchKernelGGL((k_bg_dot<AT, 16>), dim3(grid), dim3(256), 0, s, A, na, B, nb, len, per, nch, items, part);
  else
    hipLaunchKernelGGL((k_bg_dot<AT, 32>), dim3(grid), dim3(256), 0, s, A, na, B, nb, len, per, nch, items, part);
  hipLaunchKernelGGL(k_bg_dot_final, dim3((tot + 3) / 4), dim3(256), 0, s, part, na, nb, nch, out, ldo, beta, outT);
}

template <typename AT, typename OT>
void launch_bg_update(const AT* A, int na, const double* H, int64_t sa, int64_t sb, double alpha, const OT* win,
                      double beta, OT* out, int nb, int64_t len, hipStream_t s) {
  if (nb <= 0) return;
  if constexpr (std::is_same<AT, float>::value) {
    if (len % 2 == 0 && nb <= 8) {
      hipLaunchKernelGGL((k_bg_update_v8<OT>), dim3((unsigned)((len + 511) / 512)), dim3(256), 0, s, A, na, H, sa,
                         sb, alpha, win, beta, out, nb, len);
      return;
    }
    if (len % 2 == 0) {
      const int64_t blocks2 = (len + 127) / 128;
      if (nb > 16)
        hipLaunchKernelGGL((k_bg_update_f2<OT, true>), dim3((unsigned)blocks2), dim3(256), 0, s, A, na, H, sa, sb,
                           alpha, win, beta, out, nb, len);
      else
        hipLaunchKernelGGL((k_bg_update_f2<OT, false>), dim3((unsigned)blocks2), dim3(256), 0, s, A, na, H, sa, sb,
                           alpha, win, beta, out, nb, len);
      return;
    }
  }
  const int64_t blocks = (len + 63) / 64;
  hipLaunchKernelGGL((k_bg_update<AT, OT>), dim3((unsigned)blocks), dim3(256), 0, s, A, na, H, sa, sb, alpha, win,
                     beta, out, nb, len);
}

template void launch_bg_dot<double>(const double*, int, const double*, int, int64_t, double*, double*, int, double,
                                    hipStream_t, double*);
template void launch_bg_dot<float>(const float*, int, const double*, int, int64_t, double*, double*, int, double,
                                   hipStream_t, double*);
template void launch_bg_update<double, double>(const double*, int, const double*, int64_t, int64_t, double,
                                               const double*, double, double*, int, int64_t, hipStream_t);
template void launch_bg_update<float, double>(const float*, int, const double*, int64_t, int64_t, double,
                                              const double*, double, double*, int, int64_t, hipStream_t);
template void launch_bg_update<double, float>(const double*, int, const double*, int64_t, int64_t, double,
                                              const float*, double, float*, int, int64_t, hipStream_t);

void launch_bg_widen(const float* a, double* b, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_bg_widen, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, a, b, n);
}

void launch_bg_chol(const double* G, int m, double drop, const int* cnt_in, const double* rprev, int* cnt, double* T,
                    double* R, hipStream_t s) {
  hipLaunchKernelGGL(k_bg_chol, dim3(1), dim3(256), 0, s, G, m, drop, cnt_in, rprev, cnt, T, R);
}

void launch_bg_lsq(const BgLsq& L, int n0, int r, int nv, const double* h, int ldh, const double* R,
                   const int* cnts, double* host_res, int* host_cnt, hipStream_t s) {
  hipLaunchKernelGGL(k_bg_lsq, dim3(1), dim3(64 * kLsqWaves), 0, s, L, n0, r, nv, h, ldh, R, cnts, host_res,
                     host_cnt);
}

void launch_bg_backsolve(const BgLsq& L, int ncol, double* Y, int ldy, hipStream_t s) {
  if (ncol <= 0) return;
  hipLaunchKernelGGL(k_bg_backsolve, dim3(1), dim3(1024), 0, s, L, ncol, Y, ldy);
}

void launch_bg_lsq_start(const BgLsq& L, const double* R0, const int* m, hipStream_t s) {
  const int64_t tot = (int64_t)L.ldH * L.s;
  hipLaunchKernelGGL(k_bg_lsq_start, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, L, R0, m);
}

}  // namespace smpm
