// gfx950 kernels of the SMPM deflated Schur complement solver (FP64 path).
//
// Mapping.  Element-local operators run one 64-lane wavefront per element:
// lanes index the outputs (side x node along the side), the operator is stored
// with that index fastest so each step of the contraction is one coalesced
// read, and the neighbour data the contraction needs is staged in LDS.  Vector
// reductions are two-stage (per-chunk partials, then a fixed-order sum), so
// every FP64 result is deterministic from run to run.
#include <hip/hip_runtime.h>

#include <atomic>

#include "smpm_kernels.h"
#include "smpm_plan.h"  // kDenseCoarseMax

namespace smpm {

namespace {

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

// Sum over each row of 16 lanes, the same value on the row's lanes: a butterfly on
// DPP lane moves (partners lane ^ 1, lane ^ 2, then the half-row and row mirrors,
// 7 - i and 15 - i).  A fixed order.
__device__ __forceinline__ double row_sum16(double v) {
  v += dpp_move<0xB1>(v);   // quad permutation 1 0 3 2
  v += dpp_move<0x4E>(v);   // quad permutation 2 3 0 1
  v += dpp_move<0x141>(v);  // half-row mirror
  v += dpp_move<0x140>(v);  // row mirror
  return v;
}

// Sum over the 64 lanes, the same value on every lane: the row sums, then the four
// of them read as scalars.  A fixed order.  All 64 lanes must be active.
__device__ __forceinline__ double wave_sum(double v) {
  v = row_sum16(v);
  return (read_lane(v, 0) + read_lane(v, 16)) + (read_lane(v, 32) + read_lane(v, 48));
}

__device__ __forceinline__ int side_node(int n, int s, int t) {
  return s == 0 ? t * n : s == 1 ? t * n + (n - 1) : s == 2 ? t : (n - 1) * n + t;
}

// ------------------------------------------------------------------ Schur apply


constexpr int kPrefetch = 8;  // independent operator loads in flight per lane

// t = y + B A^{-1} E y (Eq. schur_complement_system), pushed from senders.
// One wavefront takes a group of up to kGroup elements of one class J: their
// slots are staged in LDS, lane (s, i) holds row i of J's outgoing flux W_{J,s}
// and accumulates it against all elements of the group, so each operator entry
// is read once per group.  Sender e's side-s flux lands in the facing slots of
// its neighbour, which have no other writer.
template <int G, typename OpT>
__global__ __launch_bounds__(256) void k_schur_fwd(DevPlan P, const double* __restrict__ y,
                                                   double* __restrict__ t, const int* __restrict__ active,
                                                   double* __restrict__ side_sums) {
  using Acc = typename AccOf<OpT>::type;
  extern __shared__ double lds[];
  const int col = blockIdx.y;
  if (active && !active[col]) return;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int g = xcd_block(blockIdx.x, gridDim.x) * 4 + wave;
  const int n = P.n, ld = 4 * n;
  double* ysd = lds + (size_t)wave * G * ld;   // this wave's region (G*ld doubles)
  Acc* ys = reinterpret_cast<Acc*>(ysd);
  const double* yc = y + (int64_t)col * P.k;
  double* tc = t + (int64_t)col * P.k;
  int elem[G];
  int J = 0, ns = 0;
  if (g < P.ngrp) {
    J = P.grp_cls[g];
    ns = P.cls_nslots[J];
#pragma unroll
    for (int u = 0; u < G; ++u) {
      elem[u] = P.grp_elem[g * kGroup + u];
      if (elem[u] >= 0) {
        const int base = P.slot_off[elem[u]];
        for (int c = lane; c < ns; c += 64) ys[u * ld + c] = (Acc)yc[base + c];
      }
    }
  }
  __syncthreads();
  const bool valid = g < P.ngrp;
  double tv[G];
#pragma unroll
  for (int u = 0; u < G; ++u) tv[u] = 0.0;
  for (int o = lane; o < 4 * n && valid; o += 64) {
    const int s = o / n, i = o - s * n;
    if (P.cls_sidecol[J * 4 + s] < 0) continue;
    const OpT* Wp = schur_op<OpT>(P, true) + P.W_off[J * 4 + s];
    Acc acc[G];
#pragma unroll
    for (int u = 0; u < G; ++u) acc[u] = 0;
    // operator loads are issued kPrefetch at a time so they overlap
    for (int c0 = 0; c0 < ns; c0 += kPrefetch) {
      Acc wv[kPrefetch];
#pragma unroll
      for (int q = 0; q < kPrefetch; ++q) wv[q] = c0 + q < ns ? to_acc(Wp[(c0 + q) * n + i]) : Acc(0);
#pragma unroll
      for (int q = 0; q < kPrefetch; ++q) {
        if (c0 + q >= ns) break;
#pragma unroll
        for (int u = 0; u < G; ++u) acc[u] = fma(wv[q], ys[u * ld + c0 + q], acc[u]);
      }
    }
#pragma unroll
    for (int u = 0; u < G; ++u) {
      if (elem[u] < 0) break;
      const int recv = P.nbr[elem[u] * 4 + s];
      const int slot = P.side_slot[recv * 4 + (s ^ 1)] + i;
      tv[u] = yc[slot] + (double)acc[u];
      tc[slot] = tv[u];
    }
  }
  if (!side_sums) return;
  // Sum of t over each receiving side (4n <= 64: lane o = s*n + i owns one row).
  // The values go through this wave's LDS region, then lane s adds its side's n
  // entries in order.
  __syncthreads();
  if (valid && lane < 4 * n) {
    const int s = lane / n;
    if (P.cls_sidecol[J * 4 + s] >= 0) {
#pragma unroll
      for (int u = 0; u < G; ++u) ysd[u * ld + lane] = tv[u];
    }
  }
  __syncthreads();
  if (valid && lane < 4 && P.cls_sidecol[J * 4 + lane] >= 0) {
    const int s = lane;
    double* ss = side_sums + (int64_t)col * P.nsides;
#pragma unroll
    for (int u = 0; u < G; ++u) {
      if (elem[u] < 0) break;
      double acc = 0.0;
      for (int i = 0; i < n; ++i) acc += ysd[u * ld + s * n + i];
      const int recv = P.nbr[elem[u] * 4 + s];
      ss[P.side_slot[recv * 4 + (s ^ 1)] / n] = acc;
    }
  }
}

// t = y + E^T A^{-T} B^T y for a group of same-class elements: element e collects
// W_{J,s}^T applied to the slots its side-s flux feeds.  Lane = slot column c.
template <int G, typename OpT>
__global__ __launch_bounds__(256) void k_schur_adj(DevPlan P, const double* __restrict__ y,
                                                   double* __restrict__ t, const int* __restrict__ active) {
  using Acc = typename AccOf<OpT>::type;
  extern __shared__ double lds[];
  const int col = blockIdx.y;
  if (active && !active[col]) return;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int g = xcd_block(blockIdx.x, gridDim.x) * 4 + wave;
  const int n = P.n, ld = 4 * n;
  Acc* yr = reinterpret_cast<Acc*>(lds + (size_t)wave * G * ld);  // [u][s*n + i]
  const double* yc = y + (int64_t)col * P.k;
  double* tc = t + (int64_t)col * P.k;
  int elem[G];
  int J = 0, ns = 0;
  if (g < P.ngrp) {
    J = P.grp_cls[g];
    ns = P.cls_nslots[J];
#pragma unroll
    for (int u = 0; u < G; ++u) {
      elem[u] = P.grp_elem[g * kGroup + u];
      if (elem[u] >= 0) {
        for (int q = lane; q < ld; q += 64) {
          const int s = q / n, i = q - s * n;
          const int j = P.nbr[elem[u] * 4 + s];
          yr[u * ld + q] = j >= 0 ? (Acc)yc[P.side_slot[j * 4 + (s ^ 1)] + i] : Acc(0);
        }
      }
    }
  }
  __syncthreads();
  if (g >= P.ngrp) return;
  for (int c = lane; c < ns; c += 64) {
    Acc acc[G];
#pragma unroll
    for (int u = 0; u < G; ++u) acc[u] = 0;
    for (int s = 0; s < 4; ++s) {
      if (P.cls_sidecol[J * 4 + s] < 0) continue;
      const OpT* Wp = schur_op<OpT>(P, false) + P.W_off[J * 4 + s];
      for (int i0 = 0; i0 < n; i0 += kPrefetch) {
        Acc wv[kPrefetch];
#pragma unroll
        for (int q = 0; q < kPrefetch; ++q) wv[q] = i0 + q < n ? to_acc(Wp[(i0 + q) * ns + c]) : Acc(0);
#pragma unroll
        for (int q = 0; q < kPrefetch; ++q) {
          if (i0 + q >= n) break;
#pragma unroll
          for (int u = 0; u < G; ++u) acc[u] = fma(wv[q], yr[u * ld + s * n + i0 + q], acc[u]);
        }
      }
    }
#pragma unroll
    for (int u = 0; u < G; ++u) {
      if (elem[u] < 0) break;
      const int slot = P.slot_off[elem[u]] + c;
      tc[slot] = yc[slot] + (double)acc[u];
    }
  }
}

// ------------------------------------------------------------------ Schur apply on matrix cores
//
// For a class J the element-local part of S is one dense map per element, from its
// ns slots to the 4n nodes of the sides its fluxes reach (rows o = s*n + i).  A tile
// of up to 16 same-class elements turns it into the product
//     T[o][u] = sum_c W_J[o][c] Y[c][u]         (forward; u = element of the tile)
//     T[c][u] = sum_o W_J[o][c] Y[o][u]         (transpose: Y gathered from the
//                                                neighbours' facing slots)
// done with 16x16x4 MFMA tiles: wavefront w of the workgroup owns output rows
// 16w..16w+15, the operator fragments come from the class copy (L2-resident, shared
// by every tile of the class) and the Y tile is staged in LDS as [k][u].

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

template <typename Acc>
struct Mma;
template <>
struct Mma<double> {
  using V = v4d;
  static __device__ __forceinline__ V mma(double a, double b, V c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  // row of the 16x16 result held in register v of lane l (column = l % 16)
  static __device__ __forceinline__ int row(int l, int v) { return (l >> 4) + 4 * v; }
};
template <>
struct Mma<float> {
  using V = v4f;
  static __device__ __forceinline__ V mma(float a, float b, V c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int l, int v) { return 4 * (l >> 4) + v; }
};

constexpr int kTileLd = kTile + 1;  // LDS row stride of the staged Y tile

// KT = 4-deep steps (4*KT >= 4n, KT = 4 * row tiles), workgroup = 16*KT threads,
// NC right-hand-side columns per workgroup (the operator fragments, held in
// registers, serve all of them).  Every index the tile needs comes from its slot
// tables, so each gather is one load after one table load, and all of a thread's
// loads are issued before the first wait.  The 16x16 results go back through LDS
// so that 16 lanes write 16 consecutive rows (one receiving side, or the element's
// own slots) with one coalesced store.
template <bool ADJ, int KT, int NC, typename OpT, bool NTS = false>
__global__ __launch_bounds__(256) void k_schur_mfma(DevPlan P, const double* __restrict__ y,
                                                    double* __restrict__ t, int nrhs,
                                                    const int* __restrict__ active,
                                                    double* __restrict__ side_sums) {
  using Acc = typename AccOf<OpT>::type;
  using M = Mma<Acc>;
  constexpr int kRows = 4 * KT;                    // staged Y rows (contraction index, zero padded)
  constexpr int kPer = kTile * kRows / (16 * KT);  // staged values per thread and column (= 4)
  constexpr int kWaves = KT / 4;
  extern __shared__ double lds[];
  const int c0 = blockIdx.y * NC;
  const int tile = xcd_block(blockIdx.x, gridDim.x);
  if (tile >= P.ntile) return;
  // Nothing below waits for the columns' activity or the class's slot count until
  // the staged values are written: the table loads, the operator fragments and the
  // y gathers (in-bounds, masked afterwards) are all in flight first.
  const int n = P.n, no = 4 * n;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int J = P.tile_cls[tile];
  // ys: the staged Y tiles [NC][kRows][kTileLd]; after the products the same space
  // holds the result tiles [NC][kWaves][kTile][kTileLd] (as many entries)
  Acc* ys = reinterpret_cast<Acc*>(lds);
  double* part = lds + (NC * kRows * kTileLd * sizeof(Acc) + 7) / 8;  // [NC][kTile][4][kWaves]
  const int* src = P.tile_src + tile * kTile;
  const int* dst = P.tile_dst + tile * kTile * 4;

  // operator fragments: one coalesced load per step
  const OpT* Af = mma_op<OpT>(P, ADJ) + ((int64_t)(J * P.mma_mt + wave) * KT) * 64 + lane;
  Acc a[KT];
#pragma unroll
  for (int q = 0; q < KT; ++q) a[q] = to_acc(Af[q * 64]);

  // Output mapping after the transpose: lane l writes row mr = 16*wave + l%16 of
  // tile columns (elements) uu = l/16 + 4v.  Table entries are loaded first
  // (unconditional, in-bounds), then every y gather at once; an invalid gather
  // reads y[0] and is masked, so no load waits on a branch.
  const int row = lane & 15, mr = wave * 16 + row;
  const int srow = min(mr / n, 3);
  int tb[4], sb[kPer];
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int uu = (lane >> 4) + 4 * v;
    tb[v] = ADJ ? src[uu] : dst[uu * 4 + srow];
  }
#pragma unroll
  for (int j = 0; j < kPer; ++j) {
    const int q = tid + j * 16 * KT;
    const int uu = q / kRows, kk = q - uu * kRows;
    sb[j] = ADJ ? dst[uu * 4 + min(kk / n, 3)] : src[uu];
  }
  // the output slots (row mr of the tile's elements; the transpose's rows end at the
  // class's slot count, known later), clamped into the vector for the gathers of y
  int slotg[4];
#pragma unroll
  for (int v = 0; v < 4; ++v)
    slotg[v] = tb[v] >= 0 ? (int)min((int64_t)tb[v] + (ADJ ? mr : mr - srow * n), P.k - 1) : -1;
  // the Y tile as [kk][u]: forward gathers the element's own slots, transpose the
  // neighbours' slots facing it (the gather index is clamped into the vector; entries
  // past the contraction length kdim are masked once it is known)
  int gi[kPer];
#pragma unroll
  for (int j = 0; j < kPer; ++j) {
    const int q = tid + j * 16 * KT;
    const int uu = q / kRows, kk = q - uu * kRows;
    const int s = kk / n;
    gi[j] = sb[j] >= 0 ? (int)min((int64_t)sb[j] + (ADJ ? kk - s * n : kk), P.k - 1) : -1;
  }
  double yv[NC][4], st[NC][kPer];
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    const double* yc = y + (int64_t)(c0 + c < nrhs ? c0 + c : 0) * P.k;
#pragma unroll
    for (int j = 0; j < kPer; ++j) st[c][j] = yc[max(gi[j], 0)];
#pragma unroll
    for (int v = 0; v < 4; ++v) yv[c][v] = yc[max(slotg[v], 0)];
  }
  bool on[NC];
  bool any = false;
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    on[c] = c0 + c < nrhs && (!active || active[c0 + c]);
    any = any || on[c];
  }
  if (!any) return;
  const int ns = P.cls_nslots[J];
  const int kdim = ADJ ? no : ns;
  const bool row_ok = ADJ ? mr < ns : mr < no;
  int slot[4];
#pragma unroll
  for (int v = 0; v < 4; ++v) slot[v] = row_ok && tb[v] >= 0 ? tb[v] + (ADJ ? mr : mr - srow * n) : -1;
#pragma unroll
  for (int c = 0; c < NC; ++c)
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
      const int q = tid + j * 16 * KT;
      const int uu = q / kRows, kk = q - uu * kRows;
      ys[(c * kRows + kk) * kTileLd + uu] = gi[j] >= 0 && kk < kdim ? (Acc)st[c][j] : Acc(0);
    }
  __syncthreads();

  typename M::V acc[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    acc[c] = typename M::V{0, 0, 0, 0};
#pragma unroll
    for (int q = 0; q < KT; ++q)
      acc[c] = M::mma(a[q], ys[(c * kRows + 4 * q + (lane >> 4)) * kTileLd + (lane & 15)], acc[c]);
  }
  __syncthreads();  // every wave is done reading ys
#pragma unroll
  for (int c = 0; c < NC; ++c)
#pragma unroll
    for (int v = 0; v < 4; ++v)
      ys[((c * kWaves + wave) * kTile + (lane & 15)) * kTileLd + M::row(lane, v)] = acc[c][v];
  __syncthreads();

  // receiving sides met by this wave's 16 rows (several when n < 16)
  const int s_lo = min((wave * 16) / n, 3), s_hi = min((wave * 16 + 15) / n, 3);
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    if (!on[c]) continue;
    double* tc = t + (int64_t)(c0 + c) * P.k;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int uu = (lane >> 4) + 4 * v;
      const double tv = yv[c][v] + (double)ys[((c * kWaves + wave) * kTile + uu) * kTileLd + row];
      if (slot[v] >= 0) {
        if constexpr (NTS)  // an output that goes back to the caller: streamed past the caches
          __builtin_nontemporal_store(tv, &tc[slot[v]]);
        else
          tc[slot[v]] = tv;
      }
      if (!ADJ && side_sums) {
        // sums over the rows of each receiving side: 16-lane butterflies, fixed order
        double* pp = part + (c * kTile + uu) * 4 * kWaves;
        if (row == 0)
#pragma unroll
          for (int s = 0; s < 4; ++s)
            if (s < s_lo || s > s_hi) pp[s * kWaves + wave] = 0.0;
        for (int s = s_lo; s <= s_hi; ++s) {
          const double x = row_sum16(slot[v] >= 0 && srow == s ? tv : 0.0);
          if (row == 0) pp[s * kWaves + wave] = x;
        }
      }
    }
  }
  if (ADJ || !side_sums) return;
  __syncthreads();
  if (tid < 4 * kTile) {
    const int uu = tid >> 2, s = tid & 3;
    const int b = dst[uu * 4 + s];
    if (b >= 0)
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        if (!on[c]) continue;
        double sum = 0.0;
        for (int w = 0; w < kWaves; ++w) sum += part[((c * kTile + uu) * 4 + s) * kWaves + w];
        side_sums[(int64_t)(c0 + c) * P.nsides + b / n] = sum;
      }
  }
}

// Persistent, software-pipelined variant (no side sums).  Work items are (tile,
// column group) pairs, tile-major; each XCD walks one contiguous slice of them (its
// blocks are those with blockIdx.x % 8 equal to the XCD) with one item per block in
// turn.  While the products and stores of one item run, the next item's y is already
// being loaded into registers, and the class operator fragments stay in registers
// across items of one class.  Results go through a separate LDS region, so the
// staged Y tile is only rewritten after a barrier.
template <bool ADJ, int KT, int NC, typename OpT>
__global__ __launch_bounds__(256) void k_schur_mfma_pers(DevPlan P, const double* __restrict__ y,
                                                         double* __restrict__ t, int nrhs,
                                                         const int* __restrict__ active, int ncg) {
  using Acc = typename AccOf<OpT>::type;
  using M = Mma<Acc>;
  constexpr int kRows = 4 * KT;
  constexpr int kPer = kTile * kRows / (16 * KT);
  constexpr int kWaves = KT / 4;
  extern __shared__ double lds[];
  Acc* ys = reinterpret_cast<Acc*>(lds);          // [NC][kRows][kTileLd]
  Acc* rs = ys + NC * kRows * kTileLd;             // [NC][kWaves][kTile][kTileLd]
  const int n = P.n, no = 4 * n;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int row = lane & 15, mr = wave * 16 + row;
  const int srow = min(mr / n, 3);
  const int64_t nitems = (int64_t)P.ntile * ncg;
  const int xcd = blockIdx.x & 7, nbx = gridDim.x >> 3;
  const int64_t hi = nitems * (xcd + 1) / 8;
  int64_t item = nitems * xcd / 8 + (blockIdx.x >> 3);
  if (item >= hi) return;

  // index tables and y loads of one item (see k_schur_mfma for the mappings)
  auto prepare = [&](int64_t it, int& c0, int& J, bool (&on)[NC], int (&slot)[4], int (&gi)[kPer]) {
    const int tile = (int)(it / ncg);
    c0 = (int)(it - (int64_t)tile * ncg) * NC;
#pragma unroll
    for (int c = 0; c < NC; ++c) on[c] = c0 + c < nrhs && (!active || active[c0 + c]);
    J = P.tile_cls[tile];
    const int ns = P.cls_nslots[J];
    const int kdim = ADJ ? no : ns;
    const int* src = P.tile_src + tile * kTile;
    const int* dst = P.tile_dst + tile * kTile * 4;
    int tb[4], sb[kPer];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int uu = (lane >> 4) + 4 * v;
      tb[v] = ADJ ? src[uu] : dst[uu * 4 + srow];
    }
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
      const int q = tid + j * 16 * KT;
      const int uu = q / kRows, kk = q - uu * kRows;
      sb[j] = ADJ ? dst[uu * 4 + min(kk / n, 3)] : src[uu];
    }
    const bool row_ok = ADJ ? mr < ns : mr < no;
#pragma unroll
    for (int v = 0; v < 4; ++v) slot[v] = row_ok && tb[v] >= 0 ? tb[v] + (ADJ ? mr : mr - srow * n) : -1;
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
      const int q = tid + j * 16 * KT;
      const int uu = q / kRows, kk = q - uu * kRows;
      const int s = kk / n;
      const bool ok = sb[j] >= 0 && kk < kdim;
      gi[j] = ok ? sb[j] + (ADJ ? kk - s * n : kk) : -1;
    }
  };
  auto load = [&](int c0, const bool (&on)[NC], const int (&slot)[4], const int (&gi)[kPer],
                  double (&st)[NC][kPer], double (&yv)[NC][4]) {
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      const double* yc = y + (int64_t)(on[c] ? c0 + c : 0) * P.k;
#pragma unroll
      for (int j = 0; j < kPer; ++j) st[c][j] = yc[max(gi[j], 0)];
#pragma unroll
      for (int v = 0; v < 4; ++v) yv[c][v] = yc[max(slot[v], 0)];
    }
  };

  int c0, J;
  bool on[NC];
  int slot[4], gi[kPer];
  double st[NC][kPer], yv[NC][4];
  prepare(item, c0, J, on, slot, gi);
  load(c0, on, slot, gi, st, yv);
  int Ja = -1;
  Acc a[KT];
  while (true) {
    if (J != Ja) {  // uniform over the workgroup
      const OpT* Af = mma_op<OpT>(P, ADJ) + ((int64_t)(J * P.mma_mt + wave) * KT) * 64 + lane;
#pragma unroll
      for (int q = 0; q < KT; ++q) a[q] = to_acc(Af[q * 64]);
      Ja = J;
    }
    __syncthreads();  // the previous item is done with ys and rs
#pragma unroll
    for (int c = 0; c < NC; ++c)
#pragma unroll
      for (int j = 0; j < kPer; ++j) {
        const int q = tid + j * 16 * KT;
        const int uu = q / kRows, kk = q - uu * kRows;
        ys[(c * kRows + kk) * kTileLd + uu] = gi[j] >= 0 ? (Acc)st[c][j] : Acc(0);
      }
    __syncthreads();
    // the next item's loads fly while this item's products and stores run
    const int64_t nxt = item + nbx;
    const bool more = nxt < hi;
    int c0n = 0, Jn = J;
    bool onn[NC];
    int slotn[4], gin[kPer];
    double stn[NC][kPer], yvn[NC][4];
    if (more) {
      prepare(nxt, c0n, Jn, onn, slotn, gin);
      load(c0n, onn, slotn, gin, stn, yvn);
    }
    typename M::V acc[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      acc[c] = typename M::V{0, 0, 0, 0};
#pragma unroll
      for (int q = 0; q < KT; ++q)
        acc[c] = M::mma(a[q], ys[(c * kRows + 4 * q + (lane >> 4)) * kTileLd + (lane & 15)], acc[c]);
    }
#pragma unroll
    for (int c = 0; c < NC; ++c)
#pragma unroll
      for (int v = 0; v < 4; ++v)
        rs[((c * kWaves + wave) * kTile + (lane & 15)) * kTileLd + M::row(lane, v)] = acc[c][v];
    __syncthreads();
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      if (!on[c]) continue;
      double* tc = t + (int64_t)(c0 + c) * P.k;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int uu = (lane >> 4) + 4 * v;
        const double tv = yv[c][v] + (double)rs[((c * kWaves + wave) * kTile + uu) * kTileLd + row];
        if (slot[v] >= 0) tc[slot[v]] = tv;
      }
    }
    if (!more) break;
    item = nxt;
    c0 = c0n;
    J = Jn;
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      on[c] = onn[c];
#pragma unroll
      for (int j = 0; j < kPer; ++j) st[c][j] = stn[c][j];
#pragma unroll
      for (int v = 0; v < 4; ++v) yv[c][v] = yvn[c][v];
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) slot[v] = slotn[v];
#pragma unroll
    for (int j = 0; j < kPer; ++j) gi[j] = gin[j];
  }
}

// Column-pipelined variant (no side sums): one workgroup per tile and group of up to
// cpw columns, taken one column per pass.  The operator fragments and the tile's index
// tables are loaded once; the gathers of column c+1 are issued before the products of
// column c (the pass loop is unrolled, so the two register sets are indexed
// statically), so each workgroup keeps loads in flight while its matrix cores run.  Y
// tiles are double-buffered in LDS, the result tile has its own buffer; two barriers
// per pass, the same count for every thread.  Every column gets the arithmetic of
// k_schur_mfma.
template <bool ADJ, int KT, int CPW, typename OpT, bool NTS>
__global__ __launch_bounds__(256) void k_schur_cols(DevPlan P, const double* __restrict__ y,
                                                    double* __restrict__ t, int nrhs,
                                                    const int* __restrict__ active) {
  using Acc = typename AccOf<OpT>::type;
  using M = Mma<Acc>;
  constexpr int kRows = 4 * KT;
  constexpr int kPer = kTile * kRows / (16 * KT);  // staged values per thread (= 4)
  constexpr int kBuf = kRows * kTileLd;
  extern __shared__ double lds[];
  Acc* ybuf = reinterpret_cast<Acc*>(lds);         // [2][kRows][kTileLd]
  Acc* rbuf = ybuf + 2 * kBuf;                     // [kWaves][kTile][kTileLd]
  const int tile = xcd_block(blockIdx.x, gridDim.x);
  if (tile >= P.ntile) return;
  const int c0 = blockIdx.y * CPW;
  const int passes = min(CPW, nrhs - c0);
  if (passes <= 0) return;
  const int n = P.n, no = 4 * n;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int J = P.tile_cls[tile];
  const int ns = P.cls_nslots[J];
  const int kdim = ADJ ? no : ns;
  const int* src = P.tile_src + tile * kTile;
  const int* dst = P.tile_dst + tile * kTile * 4;
  const OpT* Af = mma_op<OpT>(P, ADJ) + ((int64_t)(J * P.mma_mt + wave) * KT) * 64 + lane;
  Acc a[KT];
#pragma unroll
  for (int q = 0; q < KT; ++q) a[q] = to_acc(Af[q * 64]);
  const int row = lane & 15, mr = wave * 16 + row;
  const int srow = min(mr / n, 3);
  int tb[4], sb[kPer];
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int uu = (lane >> 4) + 4 * v;
    tb[v] = ADJ ? src[uu] : dst[uu * 4 + srow];
  }
#pragma unroll
  for (int j = 0; j < kPer; ++j) {
    const int q = tid + j * 16 * KT;
    const int uu = q / kRows, kk = q - uu * kRows;
    sb[j] = ADJ ? dst[uu * 4 + min(kk / n, 3)] : src[uu];
  }
  const bool row_ok = ADJ ? mr < ns : mr < no;
  int slot[4], gi[kPer];
#pragma unroll
  for (int v = 0; v < 4; ++v) slot[v] = row_ok && tb[v] >= 0 ? tb[v] + (ADJ ? mr : mr - srow * n) : -1;
#pragma unroll
  for (int j = 0; j < kPer; ++j) {
    const int q = tid + j * 16 * KT;
    const int uu = q / kRows, kk = q - uu * kRows;
    const int sd = kk / n;
    const bool ok = sb[j] >= 0 && kk < kdim;
    gi[j] = ok ? sb[j] + (ADJ ? kk - sd * n : kk) : -1;
  }
  // column loads into register set b (statically indexed after unrolling)
  double st[2][kPer], yv[2][4];
  auto load = [&](int c, int b) {
    const double* yc = y + (int64_t)c * P.k;
#pragma unroll
    for (int j = 0; j < kPer; ++j) st[b][j] = yc[max(gi[j], 0)];
#pragma unroll
    for (int v = 0; v < 4; ++v) yv[b][v] = yc[max(slot[v], 0)];
  };
  load(c0, 0);
#pragma unroll
  for (int p = 0; p < CPW; ++p) {
    if (p >= passes) break;  // uniform over the workgroup
    const int c = c0 + p, b = p & 1;
    Acc* yb = ybuf + b * kBuf;
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
      const int q = tid + j * 16 * KT;
      const int uu = q / kRows, kk = q - uu * kRows;
      yb[kk * kTileLd + uu] = gi[j] >= 0 ? (Acc)st[b][j] : Acc(0);
    }
    // the next column's gathers fly during this column's products and stores
    if (p + 1 < passes) load(c + 1, b ^ 1);
    __syncthreads();
    typename M::V acc = typename M::V{0, 0, 0, 0};
#pragma unroll
    for (int q = 0; q < KT; ++q) acc = M::mma(a[q], yb[(4 * q + (lane >> 4)) * kTileLd + (lane & 15)], acc);
#pragma unroll
    for (int v = 0; v < 4; ++v) rbuf[(wave * kTile + (lane & 15)) * kTileLd + M::row(lane, v)] = acc[v];
    __syncthreads();
    if (!active || active[c]) {
      double* tc = t + (int64_t)c * P.k;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int uu = (lane >> 4) + 4 * v;
        const double tv = yv[b][v] + (double)rbuf[(wave * kTile + uu) * kTileLd + row];
        if (slot[v] >= 0) {
          if constexpr (NTS)
            __builtin_nontemporal_store(tv, &tc[slot[v]]);
          else
            tc[slot[v]] = tv;
        }
      }
    }
  }
}

// Warp-specialized persistent variant (no side sums): a workgroup of 2 x kWaves
// wavefronts walks its (tile, column group) items as the persistent kernel does.
// The first kWaves ("compute") run the matrix-core products of item s from one LDS
// Y buffer into one LDS result buffer; meanwhile the other kWaves ("memory") store
// the results of item s-1 (plus its identity term, loaded one step earlier), load
// the identity-term values of item s and gather the Y tile of item s+1 into the
// other Y buffer.  One barrier per step, count + 1 steps for count items, taken by
// every wavefront.  The products and the loads and stores of neighbouring items so
// overlap inside one workgroup; every column gets the arithmetic of k_schur_mfma.
template <bool ADJ, int KT, int NC, typename OpT, bool NTS>
__global__ __launch_bounds__(32 * KT) void k_schur_ws(DevPlan P, const double* __restrict__ y,
                                                      double* __restrict__ t, int nrhs,
                                                      const int* __restrict__ active, int ncg) {
  using Acc = typename AccOf<OpT>::type;
  using M = Mma<Acc>;
  constexpr int kThr = 16 * KT;                    // threads of one role
  constexpr int kRows = 4 * KT;
  constexpr int kPer = kTile * kRows / kThr;       // staged values per thread and column (= 4)
  constexpr int kWaves = KT / 4;
  constexpr int kBuf = NC * kRows * kTileLd;       // one Y tile set (or result tile set)
  extern __shared__ double lds[];
  Acc* ybuf = reinterpret_cast<Acc*>(lds);         // [2][kBuf]
  Acc* rbuf = ybuf + 2 * kBuf;                     // [2][kBuf]: [NC][kWaves][kTile][kTileLd]
  const int n = P.n, no = 4 * n;
  const bool mem = threadIdx.x >= kThr;
  const int tid = (int)threadIdx.x - (mem ? kThr : 0), wave = tid >> 6, lane = tid & 63;
  const int row = lane & 15, mr = wave * 16 + row;
  const int srow = min(mr / n, 3);
  const int64_t nitems = (int64_t)P.ntile * ncg;
  const int xcd = blockIdx.x & 7, nbx = gridDim.x >> 3;
  const int64_t hi = nitems * (xcd + 1) / 8;
  const int64_t first = nitems * xcd / 8 + (blockIdx.x >> 3);
  const int count = first < hi ? (int)((hi - first + nbx - 1) / nbx) : 0;
  if (count == 0) return;  // uniform over the workgroup

  // tables of item it (memory role): columns, output slots, gather indices
  auto tables = [&](int64_t it, int& c0, bool (&on)[NC], int (&slot)[4], int (&gi)[kPer]) {
    const int tile = (int)(it / ncg);
    c0 = (int)(it - (int64_t)tile * ncg) * NC;
#pragma unroll
    for (int c = 0; c < NC; ++c) on[c] = c0 + c < nrhs && (!active || active[c0 + c]);
    const int J = P.tile_cls[tile];
    const int ns = P.cls_nslots[J];
    const int kdim = ADJ ? no : ns;
    const int* src = P.tile_src + tile * kTile;
    const int* dst = P.tile_dst + tile * kTile * 4;
    int tb[4], sb[kPer];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int uu = (lane >> 4) + 4 * v;
      tb[v] = ADJ ? src[uu] : dst[uu * 4 + srow];
    }
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
      const int q = tid + j * kThr;
      const int uu = q / kRows, kk = q - uu * kRows;
      sb[j] = ADJ ? dst[uu * 4 + min(kk / n, 3)] : src[uu];
    }
    const bool row_ok = ADJ ? mr < ns : mr < no;
#pragma unroll
    for (int v = 0; v < 4; ++v) slot[v] = row_ok && tb[v] >= 0 ? tb[v] + (ADJ ? mr : mr - srow * n) : -1;
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
      const int q = tid + j * kThr;
      const int uu = q / kRows, kk = q - uu * kRows;
      const int s = kk / n;
      const bool ok = sb[j] >= 0 && kk < kdim;
      gi[j] = ok ? sb[j] + (ADJ ? kk - s * n : kk) : -1;
    }
  };
  // gather the Y tile of an item into an LDS buffer as [c][kk][u]
  auto gather = [&](int c0, const bool (&on)[NC], const int (&gi)[kPer], Acc* yb) {
    double st[NC][kPer];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      const double* yc = y + (int64_t)(on[c] ? c0 + c : 0) * P.k;
#pragma unroll
      for (int j = 0; j < kPer; ++j) st[c][j] = yc[max(gi[j], 0)];
    }
#pragma unroll
    for (int c = 0; c < NC; ++c)
#pragma unroll
      for (int j = 0; j < kPer; ++j) {
        const int q = tid + j * kThr;
        const int uu = q / kRows, kk = q - uu * kRows;
        yb[(c * kRows + kk) * kTileLd + uu] = gi[j] >= 0 ? (Acc)st[c][j] : Acc(0);
      }
  };

  if (mem) {
    // memory role: prologue gathers item 0; step s stores item s-1, loads the identity
    // term of item s and gathers item s+1
    int c0p = 0, c0c = 0;
    bool onp[NC], onc[NC];
    int slotp[4], slotc[4], gic[kPer];
    double yv[NC][4];
    tables(first, c0c, onc, slotc, gic);
    gather(c0c, onc, gic, ybuf);
    __syncthreads();
    for (int s = 0; s <= count; ++s) {
      if (s >= 1) {
        const Acc* rb = rbuf + ((s - 1) & 1) * kBuf;
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          if (!onp[c]) continue;
          double* tc = t + (int64_t)(c0p + c) * P.k;
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int uu = (lane >> 4) + 4 * v;
            const double tv = yv[c][v] + (double)rb[((c * kWaves + wave) * kTile + uu) * kTileLd + row];
            if (slotp[v] >= 0) {
              if constexpr (NTS)
                __builtin_nontemporal_store(tv, &tc[slotp[v]]);
              else
                tc[slotp[v]] = tv;
            }
          }
        }
      }
      if (s < count) {
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          const double* yc = y + (int64_t)(onc[c] ? c0c + c : 0) * P.k;
#pragma unroll
          for (int v = 0; v < 4; ++v) yv[c][v] = yc[max(slotc[v], 0)];
        }
        c0p = c0c;
#pragma unroll
        for (int c = 0; c < NC; ++c) onp[c] = onc[c];
#pragma unroll
        for (int v = 0; v < 4; ++v) slotp[v] = slotc[v];
        if (s + 1 < count) {
          tables(first + (int64_t)(s + 1) * nbx, c0c, onc, slotc, gic);
          gather(c0c, onc, gic, ybuf + ((s + 1) & 1) * kBuf);
        }
      }
      __syncthreads();
    }
  } else {
    // compute role: products of item s from Y buffer s % 2 into result buffer s % 2
    int Ja = -1;
    Acc a[KT];
    __syncthreads();
    for (int s = 0; s <= count; ++s) {
      if (s < count) {
        const int tile = (int)((first + (int64_t)s * nbx) / ncg);
        const int J = P.tile_cls[tile];
        if (J != Ja) {  // uniform over the workgroup
          const OpT* Af = mma_op<OpT>(P, ADJ) + ((int64_t)(J * P.mma_mt + wave) * KT) * 64 + lane;
#pragma unroll
          for (int q = 0; q < KT; ++q) a[q] = to_acc(Af[q * 64]);
          Ja = J;
        }
        const Acc* yb = ybuf + (s & 1) * kBuf;
        Acc* rb = rbuf + (s & 1) * kBuf;
        typename M::V acc[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          acc[c] = typename M::V{0, 0, 0, 0};
#pragma unroll
          for (int q = 0; q < KT; ++q)
            acc[c] = M::mma(a[q], yb[(c * kRows + 4 * q + (lane >> 4)) * kTileLd + (lane & 15)], acc[c]);
        }
#pragma unroll
        for (int c = 0; c < NC; ++c)
#pragma unroll
          for (int v = 0; v < 4; ++v)
            rb[((c * kWaves + wave) * kTile + (lane & 15)) * kTileLd + M::row(lane, v)] = acc[c][v];
      }
      __syncthreads();
    }
  }
}

// ------------------------------------------------------------------ B A^{-1} and its transpose

__global__ __launch_bounds__(64) void k_flux(DevPlan P, const double* __restrict__ f, double* __restrict__ b) {
  extern __shared__ double fs[];  // 4 * n2
  const int e = blockIdx.x, col = blockIdx.y, lane = threadIdx.x;
  const int n = P.n, n2 = P.n2;
  const double* fc = f + (int64_t)col * P.r;
  double* bc = b + (int64_t)col * P.k;
  for (int s = 0; s < 4; ++s) {
    const int j = P.nbr[e * 4 + s];
    if (j < 0) continue;
    for (int l = lane; l < n2; l += 64) fs[s * n2 + l] = fc[(int64_t)j * n2 + l];
  }
  __syncthreads();
  for (int o = lane; o < 4 * n; o += 64) {
    const int s = o / n, i = o - s * n;
    const int j = P.nbr[e * 4 + s];
    if (j < 0) continue;
    const double* Hp = P.Hc + P.H_off[P.cls[j] * 4 + (s ^ 1)];
    double acc = 0.0;
    // 32 operator loads in flight per batch (in bounds), the products in order
    for (int l0 = 0; l0 < n2; l0 += 32) {
      double h[32];
#pragma unroll
      for (int u = 0; u < 32; ++u) h[u] = Hp[min(l0 + u, n2 - 1) * n + i];
#pragma unroll
      for (int u = 0; u < 32; ++u)
        if (l0 + u < n2) acc = fma(h[u], fs[s * n2 + l0 + u], acc);
    }
    bc[P.side_slot[e * 4 + s] + i] = acc;
  }
}

__global__ __launch_bounds__(256) void k_flux_adj(DevPlan P, const double* __restrict__ x, double* __restrict__ y) {
  __shared__ double xr[4][kMaxN];
  const int e = blockIdx.x, col = blockIdx.y, tid = threadIdx.x;
  const int n = P.n, n2 = P.n2;
  const double* xc = x + (int64_t)col * P.k;
  double* yc = y + (int64_t)col * P.r;
  if (tid < 4 * n) {
    const int s = tid / n, i = tid - s * n;
    const int j = P.nbr[e * 4 + s];
    xr[s][i] = j >= 0 ? xc[P.side_slot[j * 4 + (s ^ 1)] + i] : 0.0;
  }
  __syncthreads();
  const int J = P.cls[e];
  for (int l = tid; l < n2; l += 256) {
    double acc = 0.0;
    for (int s = 0; s < 4; ++s) {
      if (P.nbr[e * 4 + s] < 0) continue;
      const double* Hp = P.Hr + P.H_off[J * 4 + s];
#pragma unroll 8
      for (int i = 0; i < n; ++i) acc = fma(Hp[i * n2 + l], xr[s][i], acc);
    }
    yc[(int64_t)e * n2 + l] = acc;
  }
}

// ------------------------------------------------------------------ element solves

// u_e = A_e^{-1} (f_e - E_e x): corner nodes on two inter-element sides lose both slots.
__global__ __launch_bounds__(256) void k_backsub(DevPlan P, const double* __restrict__ f, const double* __restrict__ x,
                                                 double* __restrict__ u) {
  extern __shared__ double zs[];  // n2
  const int e = blockIdx.x, col = blockIdx.y, tid = threadIdx.x;
  const int n = P.n, n2 = P.n2;
  const double* fc = f + (int64_t)col * P.r;
  const double* xc = x + (int64_t)col * P.k;
  double* uc = u + (int64_t)col * P.r;
  for (int l = tid; l < n2; l += 256) zs[l] = fc[(int64_t)e * n2 + l];
  __syncthreads();
  for (int pass = 0; pass < 2; ++pass) {  // W/E sides touch disjoint nodes, then S/N
    for (int q = tid; q < 2 * n; q += 256) {
      const int s = 2 * pass + q / n, tt = q % n;
      const int base = P.side_slot[e * 4 + s];
      if (base >= 0) zs[side_node(n, s, tt)] -= xc[base + tt];
    }
    __syncthreads();
  }
  const double* Ap = P.AinvT + (int64_t)P.cls[e] * n2 * n2;
  for (int l = tid; l < n2; l += 256) {
    double acc = 0.0;
    // 32 operator loads in flight per batch (in bounds), the products in order
    for (int m0 = 0; m0 < n2; m0 += 32) {
      double a[32];
#pragma unroll
      for (int u = 0; u < 32; ++u) a[u] = Ap[(int64_t)min(m0 + u, n2 - 1) * n2 + l];
#pragma unroll
      for (int u = 0; u < 32; ++u)
        if (m0 + u < n2) acc = fma(a[u], zs[m0 + u], acc);
    }
    uc[(int64_t)e * n2 + l] = acc;
  }
}

// ---- element applies on the matrix cores (n <= 16): one block takes a tile of up to
// 16 elements of one class, stages their vectors in LDS ([contraction][element]) and
// multiplies by the class operator with FP64 16x16x4 MFMAs, so the operator is read
// once per tile instead of once per element.  Lane l supplies A[l % 16][l / 16] and
// B[l / 16][l % 16]; register v of lane l holds C[(l >> 4) + 4v][l % 16].  Results
// go back through LDS so that consecutive lanes store consecutive rows.
constexpr int kMmaN2 = 256;  // largest n^2 of these kernels (n <= 16)
constexpr int kMmaBatch = 32;  // operator loads in flight per lane

// A operand row `row` (clamped in) of a row-major source, loaded for k-steps
// m0 + 4q + kk, q < kMmaBatch; entries past `len` or of invalid rows are zero
template <typename Ld>
__device__ __forceinline__ void mma_load_a(double (&a)[kMmaBatch], int m0, int kk, int len, bool rok, Ld ld) {
#pragma unroll
  for (int q = 0; q < kMmaBatch; ++q) a[q] = ld(min(m0 + 4 * q + kk, len - 1));
#pragma unroll
  for (int q = 0; q < kMmaBatch; ++q)
    if (!rok || m0 + 4 * q + kk >= len) a[q] = 0.0;
}

// b_S = B A^{-1} f on element tiles: rows (side s, node i) of the class's side
// operators H_{J,s} (4n x n^2, stored [l][i] per side) times the tile's f; row
// (s, i) of element u lands on the neighbour's slot facing side s (tile_dst).
// With pu != nullptr the staged values are ft = f - pdot[col] * pscale * pu (written
// to ft as well): the projection that precedes B A^{-1} in the solve.
// With du != nullptr each wave also writes the partial sum of du . b over the slots it
// stores to part[col][block][wave] (zeros for idle waves and padding blocks).
__global__ __launch_bounds__(256) void k_flux_mfma(DevPlan P, const double* __restrict__ f, double* __restrict__ b,
                                                   const double* __restrict__ pu, const double* __restrict__ pdot,
                                                   double pscale, double* __restrict__ ft,
                                                   const double* __restrict__ du, double* __restrict__ part) {
  __shared__ double fs[kMmaN2 * kTileLd];
  __shared__ double os[4][kTile * kTileLd];
  const int col = blockIdx.y;
  double* pw = du ? part + ((int64_t)col * gridDim.x + blockIdx.x) * 4 + (threadIdx.x >> 6) : nullptr;
  const int tile = xcd_block(blockIdx.x, gridDim.x);
  if (tile >= P.ntile) {
    if (pw && (threadIdx.x & 63) == 0) *pw = 0.0;
    return;
  }
  const int n = P.n, n2 = P.n2, tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int J = P.tile_cls[tile];
  const int* el = P.tile_elem + tile * kTile;
  const int* dst = P.tile_dst + tile * kTile * 4;
  const double* fc = f + (int64_t)col * P.r;
  const int kr = (n2 + 3) & ~3;
  for (int q = tid; q < kr * kTile; q += 256) {
    const int u = q / kr, l = q - u * kr;
    const int e = el[u];
    double v = 0.0;
    if (e >= 0 && l < n2) {
      const int64_t x = (int64_t)e * n2 + l;
      v = fc[x];
      if (pu) {
        v = v - pdot[col] * pscale * pu[x];
        ft[(int64_t)col * P.r + x] = v;
      }
    }
    fs[l * kTileLd + u] = v;
  }
  __syncthreads();
  // 4n <= 64 rows: row tile `wave` (waves past the row count only join the barrier)
  const int r = lane & 15, kk = lane >> 4;
  const int rt = wave;
  const bool act = rt * 16 < 4 * n;
  if (act) {
    const int row = rt * 16 + r;
    const int s = min(row / n, 3), i = min(row - s * n, n - 1);
    const int64_t ho = P.H_off[J * 4 + s];
    const bool rok = row < 4 * n && ho >= 0;
    const double* Hp = P.Hc + (ho >= 0 ? ho : 0);
    v4d acc = {0.0, 0.0, 0.0, 0.0};
    for (int m0 = 0; m0 < kr; m0 += 4 * kMmaBatch) {
      double a[kMmaBatch];
      mma_load_a(a, m0, kk, n2, rok, [&](int m) { return Hp[(int64_t)m * n + i]; });
#pragma unroll
      for (int q = 0; q < kMmaBatch; ++q)
        if (m0 + 4 * q < kr) acc = Mma<double>::mma(a[q], fs[(m0 + 4 * q + kk) * kTileLd + r], acc);
    }
    // the 16 x 16 result as [element][row] in this wave's LDS
#pragma unroll
    for (int v = 0; v < 4; ++v) os[wave][r * kTileLd + Mma<double>::row(lane, v)] = acc[v];
  }
  __syncthreads();
  if (!act) {
    if (pw && lane == 0) *pw = 0.0;
    return;
  }
  // row-contiguous stores: row (s, i) of element u to the neighbour's slot facing s
  double* bc = b + (int64_t)col * P.k;
  double dsum = 0.0;
  for (int q = lane; q < kTile * 16; q += 64) {
    const int u = q >> 4, rr = q & 15;
    const int orow = rt * 16 + rr;
    if (orow >= 4 * n || el[u] < 0) continue;
    const int os_ = orow / n, oi = orow - os_ * n;
    const int base = dst[u * 4 + os_];
    if (base >= 0) {
      const double v = os[wave][u * kTileLd + rr];
      bc[base + oi] = v;
      if (du) dsum = fma(du[base + oi], v, dsum);
    }
  }
  if (!pw) return;
  for (int off = 32; off > 0; off >>= 1) dsum += __shfl_xor(dsum, off);
  if (lane == 0) *pw = dsum;
}

// u_e = A_e^{-1} (f_e - E_e x) on element tiles: the tile's right-hand sides are
// staged (the slot values subtracted as k_backsub does, W/E sides then S/N), then
// rows [64 g, 64 g + 64) of the class's A^{-1} (stored transposed, [m][l]) multiply
// them, one 16-row tile per wave.
// With wq != nullptr each block also writes the partial sum of wq . u over its outputs
// to part[col][block] (blocks in launch order), for the mean of u.
__global__ __launch_bounds__(256) void k_backsub_mfma(DevPlan P, const double* __restrict__ f,
                                                      const double* __restrict__ x, double* __restrict__ u,
                                                      const double* __restrict__ wq, double* __restrict__ part) {
  __shared__ double zs[kMmaN2 * kTileLd];
  __shared__ double os[4][kTile * kTileLd];
  __shared__ double red[4];
  const int col = blockIdx.z;
  const int nblk = gridDim.x * gridDim.y, blk = blockIdx.y * gridDim.x + blockIdx.x;
  const int tile = xcd_block(blockIdx.x, gridDim.x);
  if (tile >= P.ntile) {
    if (wq && threadIdx.x == 0) part[(int64_t)col * nblk + blk] = 0.0;
    return;
  }
  const int n = P.n, n2 = P.n2, tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int J = P.tile_cls[tile];
  const int* el = P.tile_elem + tile * kTile;
  const double* fc = f + (int64_t)col * P.r;
  const double* xc = x + (int64_t)col * P.k;
  const int kr = (n2 + 3) & ~3;
  for (int q = tid; q < kr * kTile; q += 256) {
    const int uu = q / kr, l = q - uu * kr;
    const int e = el[uu];
    zs[l * kTileLd + uu] = e >= 0 && l < n2 ? fc[(int64_t)e * n2 + l] : 0.0;
  }
  __syncthreads();
  for (int pass = 0; pass < 2; ++pass) {  // W/E sides touch disjoint nodes, then S/N
    for (int q = tid; q < kTile * 2 * n; q += 256) {
      const int uu = q / (2 * n), qq = q - uu * 2 * n;
      const int s = 2 * pass + qq / n, tt = qq % n;
      const int e = el[uu];
      if (e < 0) continue;
      const int base = P.side_slot[e * 4 + s];
      if (base >= 0) zs[side_node(n, s, tt) * kTileLd + uu] -= xc[base + tt];
    }
    __syncthreads();
  }
  const int r = lane & 15, kk = lane >> 4;
  const int row = blockIdx.y * 64 + wave * 16 + r;
  const bool rok = row < n2;
  const double* Ap = P.AinvT + (int64_t)J * n2 * n2 + min(row, n2 - 1);
  v4d acc = {0.0, 0.0, 0.0, 0.0};
  for (int m0 = 0; m0 < kr; m0 += 4 * kMmaBatch) {
    double a[kMmaBatch];
    mma_load_a(a, m0, kk, n2, rok, [&](int m) { return Ap[(int64_t)m * n2]; });
#pragma unroll
    for (int q = 0; q < kMmaBatch; ++q)
      if (m0 + 4 * q < kr) acc = Mma<double>::mma(a[q], zs[(m0 + 4 * q + kk) * kTileLd + r], acc);
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) os[wave][r * kTileLd + Mma<double>::row(lane, v)] = acc[v];
  __syncthreads();
  double* uc = u + (int64_t)col * P.r;
  const int row0 = blockIdx.y * 64 + wave * 16;
  double wsum = 0.0;
  for (int q = lane; q < kTile * 16; q += 64) {
    const int uu = q >> 4, rr = q & 15;
    const int e = el[uu];
    if (e >= 0 && row0 + rr < n2) {
      const int64_t o = (int64_t)e * n2 + row0 + rr;
      const double v = os[wave][uu * kTileLd + rr];
      uc[o] = v;
      if (wq) wsum = fma(wq[o], v, wsum);
    }
  }
  if (!wq) return;
  for (int off = 32; off > 0; off >>= 1) wsum += __shfl_xor(wsum, off);
  if (lane == 0) red[wave] = wsum;
  __syncthreads();
  if (threadIdx.x == 0) part[(int64_t)col * nblk + blk] = (red[0] + red[1]) + (red[2] + red[3]);
}

// out = A^{-T} c  (to_slots = 0, r-vector) or E^T A^{-T} c (to_slots = 1, k-vector).
__global__ __launch_bounds__(256) void k_local_adj(DevPlan P, const double* __restrict__ c, double* __restrict__ out,
                                                   int to_slots) {
  extern __shared__ double sm[];  // 2 * n2
  const int e = blockIdx.x, col = blockIdx.y, tid = threadIdx.x;
  const int n = P.n, n2 = P.n2;
  double* cs = sm;
  double* ws = sm + n2;
  const double* cc = c + (int64_t)col * P.r;
  for (int l = tid; l < n2; l += 256) cs[l] = cc[(int64_t)e * n2 + l];
  __syncthreads();
  const double* Ap = P.Ainv + (int64_t)P.cls[e] * n2 * n2;
  for (int l = tid; l < n2; l += 256) {
    double acc = 0.0;
    for (int m0 = 0; m0 < n2; m0 += 32) {
      double a[32];
#pragma unroll
      for (int u = 0; u < 32; ++u) a[u] = Ap[(int64_t)min(m0 + u, n2 - 1) * n2 + l];
#pragma unroll
      for (int u = 0; u < 32; ++u)
        if (m0 + u < n2) acc = fma(a[u], cs[m0 + u], acc);
    }
    if (to_slots)
      ws[l] = acc;
    else
      out[(int64_t)col * P.r + (int64_t)e * n2 + l] = acc;
  }
  if (!to_slots) return;
  __syncthreads();
  for (int s = 0; s < 4; ++s) {
    const int base = P.side_slot[e * 4 + s];
    if (base < 0) continue;
    for (int tt = tid; tt < n; tt += 256) out[(int64_t)col * P.k + base + tt] = ws[side_node(n, s, tt)];
  }
}

// ------------------------------------------------------------------ block-Jacobi

template <typename OpT>
__global__ __launch_bounds__(256) void k_precond(DevPlan P, const double* __restrict__ x, double* __restrict__ y,
                                                 int transpose, const int* __restrict__ active) {
  using Acc = typename AccOf<OpT>::type;
  __shared__ Acc xs[8 * kMaxN];
  __shared__ Acc part[256];
  const int b = gridDim.x % 8 == 0 ? xcd_block(blockIdx.x, gridDim.x) : blockIdx.x;
  const int col = blockIdx.y, tid = threadIdx.x;
  if (active && !active[col]) return;
  const double* xc = x + (int64_t)col * P.k;
  double* yc = y + (int64_t)col * P.k;
  const int o = P.blk_off[b], sb = P.blk_off[b + 1] - o;
  const int bc = P.blk_cls[b];
  for (int i = tid; i < sb; i += 256) xs[i] = (Acc)xc[P.blk_slots[o + i]];
  __syncthreads();
  const OpT* Mp = minv_op<OpT>(P, transpose != 0) + P.bcls_off[bc];
  block_jacobi_apply<1>(Mp, xs, 0, sb, part, [&](int, int r, Acc v) { yc[P.blk_slots[o + r]] = (double)v; });
}

// The same for NC columns per workgroup: each block inverse is read once for all of
// them (block_jacobi_apply<NC> gives every column the bits of the one-column kernel).
template <typename OpT, int NC>
__global__ __launch_bounds__(256) void k_precond_n(DevPlan P, const double* __restrict__ x, double* __restrict__ y,
                                                   int nrhs, int transpose, const int* __restrict__ active) {
  using Acc = typename AccOf<OpT>::type;
  __shared__ Acc xs[NC][8 * kMaxN];
  __shared__ Acc part[NC * 256];
  const int b = gridDim.x % 8 == 0 ? xcd_block(blockIdx.x, gridDim.x) : blockIdx.x;
  const int c0 = blockIdx.y * NC, tid = threadIdx.x;
  const int o = P.blk_off[b], sb = P.blk_off[b + 1] - o;
  const int bc = P.blk_cls[b];
  bool on[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) on[c] = c0 + c < nrhs && (!active || active[c0 + c]);
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    const double* xc = x + (int64_t)(on[c] ? c0 + c : 0) * P.k;
    for (int i = tid; i < sb; i += 256) xs[c][i] = on[c] ? (Acc)xc[P.blk_slots[o + i]] : Acc(0);
  }
  __syncthreads();
  const OpT* Mp = minv_op<OpT>(P, transpose != 0) + P.bcls_off[bc];
  block_jacobi_apply<NC>(Mp, &xs[0][0], 8 * kMaxN, sb, part, [&](int c, int r, Acc v) {
    if (on[c]) y[(int64_t)(c0 + c) * P.k + P.blk_slots[o + r]] = (double)v;
  });
}

// ------------------------------------------------------------------ deflation

// c_j = sum of t over the 2n slots of interface j: one wavefront per interface,
// lanes over slots, fixed shuffle tree.
__global__ __launch_bounds__(256) void k_iface_sum(DevPlan P, const double* __restrict__ t, double* __restrict__ c,
                                                   const int* __restrict__ active, const double* __restrict__ a,
                                                   double sb) {
  const int col = blockIdx.y;
  if (active && !active[col]) return;
  const int n = P.n;
  // with 2n <= 32 a wavefront takes two interfaces, one per half (the halves' trees
  // are the 64-lane tree without its first step, which only added zeros)
  const bool pack = 2 * n <= 32;
  const int lane = threadIdx.x & 63;
  const int j = pack ? blockIdx.x * 8 + (threadIdx.x >> 6) * 2 + (lane >> 5) : blockIdx.x * 4 + (threadIdx.x >> 6);
  const int l = pack ? lane & 31 : lane;
  if (j >= P.d) return;  // a whole wave, or a whole half whose partners are in it
  const double* tc = t + (int64_t)col * P.k;
  const double* ac = a ? a + (int64_t)col * P.k : nullptr;  // sums of a + sb t instead of t
  double acc = 0.0;
  for (int q = l; q < 2 * n; q += 64) {
    const int h = q / n, i = q - h * n;
    const int64_t x = (int64_t)P.iface_side[2 * j + h] * n + i;
    acc += ac ? ac[x] + sb * tc[x] : tc[x];
  }
  for (int off = pack ? 16 : 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
  if (l == 0) c[(int64_t)col * P.d + j] = acc;
}

// c2 = G c (or G^T c): one wavefront per row, lanes over the row, fixed reduction tree.
__global__ __launch_bounds__(256) void k_coarse(DevPlan P, const double* __restrict__ c, double* __restrict__ c2,
                                                int transpose, const int* __restrict__ active) {
  const int col = blockIdx.y;
  if (active && !active[col]) return;
  const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int d = P.d;
  if (i >= d) return;
  const double* Gp = (transpose ? P.GT : P.G) + (int64_t)i * d;  // row i of G (or of G^T)
  const double* cc = c + (int64_t)col * d;
  double acc = 0.0;
  for (int j = lane; j < d; j += 64) acc = fma(Gp[j], cc[j], acc);
  acc = wave_sum(acc);
  if (lane == 0) c2[(int64_t)col * d + i] = acc;
}

// ---- substructured coarse solve: per-column scratch = [patch parts | r | lambda]

__device__ __forceinline__ int64_t sub_part_len(const DevPlan& P) {
  return P.sub_B_off[P.sub_npatch] + (int64_t)P.sub_npatch * P.sub_border;
}

// y_p = K_pp^{-1} c_p into c2 (interior interfaces); q_p = R_p c_p (transpose:
// K_pp^{-T} c_p and F_p^T c_p) into the patch's part of the scratch.
__global__ __launch_bounds__(256) void k_sub_patch1(DevPlan P, const double* __restrict__ c, double* __restrict__ c2,
                                                    int transpose, const int* __restrict__ active) {
  extern __shared__ double cl[];
  const int pp = blockIdx.x, col = blockIdx.y;
  if (active && !active[col]) return;
  const int i0 = P.sub_I_off[pp], ni = P.sub_I_off[pp + 1] - i0;
  const int nb = P.sub_B_off[pp + 1] - P.sub_B_off[pp], nbb = nb + P.sub_border;
  const double* cc = c + (int64_t)col * P.d;
  for (int j = threadIdx.x; j < ni; j += blockDim.x) cl[j] = cc[P.sub_I[i0 + j]];
  __syncthreads();
  const double* K = (transpose ? P.sub_Kr : P.sub_Kc) + P.sub_K_off[pp];
  const double* M = (transpose ? P.sub_Fr : P.sub_Rc) + P.sub_FR_off[pp];
  double* part = P.cws + (int64_t)col * P.cws_stride + P.sub_B_off[pp] + (int64_t)pp * P.sub_border;
  for (int row = threadIdx.x; row < ni + nbb; row += blockDim.x) {
    // row of K_pp^{-1} (interior) or of R_p (separator part): its entries loaded
    // 32 at a time (clamped in the last batch), the products in order
    const bool interior = row < ni;
    const double* src = interior ? K + row : M + (row - ni);
    const int64_t ld = interior ? ni : nbb;
    double acc = 0.0;
    for (int j0 = 0; j0 < ni; j0 += 32) {
      double kv[32];
#pragma unroll
      for (int u = 0; u < 32; ++u) kv[u] = src[(int64_t)min(j0 + u, ni - 1) * ld];
#pragma unroll
      for (int u = 0; u < 32; ++u)
        if (j0 + u < ni) acc = fma(kv[u], cl[j0 + u], acc);
    }
    if (interior)
      c2[(int64_t)col * P.d + P.sub_I[i0 + row]] = acc;
    else
      part[row - ni] = acc;
  }
}

// r = c_B - (parts of the two patches of each separator); r_lambda = -(sum of the patches'
// lambda parts, in patch order)
__global__ __launch_bounds__(256) void k_sub_rhs(DevPlan P, const double* __restrict__ c,
                                                 const int* __restrict__ active) {
  const int col = blockIdx.y;
  if (active && !active[col]) return;
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  const int nS = P.sub_nsep + P.sub_border;
  if (b >= nS) return;
  const double* ws = P.cws + (int64_t)col * P.cws_stride;
  double* r = P.cws + (int64_t)col * P.cws_stride + sub_part_len(P);
  if (b < P.sub_nsep) {
    const int* wo = P.sub_sep_woff + (int64_t)b * 2;
    const double qa = ws[wo[0]];
    const double qb = ws[wo[1]];
    r[b] = c[(int64_t)col * P.d + P.sub_sep_iface[b]] - qa - qb;
  } else {
    // lambda part = last of each patch; sixteen patches' loads at a time, sums in order
    const int np = P.sub_npatch;
    double acc = 0.0;
    for (int p0 = 0; p0 < np; p0 += 16) {
      int off[16];
#pragma unroll
      for (int u = 0; u < 16; ++u) off[u] = P.sub_B_off[min(p0 + u, np - 1) + 1];
      double v[16];
#pragma unroll
      for (int u = 0; u < 16; ++u) v[u] = ws[off[u] + (int64_t)min(p0 + u, np - 1) * P.sub_border];
#pragma unroll
      for (int u = 0; u < 16; ++u)
        if (p0 + u < np) acc += v[u];
    }
    r[b] = -acc;
  }
}

// x_B = S_B^{-1} r (transpose: S_B^{-T} r): wave per row, r staged in LDS.
template <int NC>
__global__ __launch_bounds__(256) void k_sub_sep(DevPlan P, double* __restrict__ c2, int transpose, int nrhs,
                                                 const int* __restrict__ active) {
  // x_B = S_B^{-1} r for NC columns at once: each row of S_B^{-1} is read once for
  // all of them; r comes through the caches (per column, the same sums in the same
  // order as for one column)
  const int c0 = blockIdx.y * NC;
  bool on[NC];
  bool any = false;
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    on[c] = c0 + c < nrhs && (!active || active[c0 + c]);
    any = any || on[c];
  }
  if (!any) return;
  const int nS = P.sub_nsep + P.sub_border;
  const double* r[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) r[c] = P.cws + (int64_t)(on[c] ? c0 + c : c0) * P.cws_stride + sub_part_len(P);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const double* Si = transpose ? P.sub_SiT : P.sub_Si;
  // the wave's four rows advance together (rows past nS repeat the last row, in
  // bounds, results not stored), so their loads are in flight at once
  const int a0 = (blockIdx.x * 4 + wave) * 4;
  if (a0 >= nS) return;
  const double* row[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) row[q] = Si + (int64_t)min(a0 + q, nS - 1) * nS;
  double acc[4][NC];
#pragma unroll
  for (int q = 0; q < 4; ++q)
#pragma unroll
    for (int c = 0; c < NC; ++c) acc[q][c] = 0.0;
#pragma unroll 2
  for (int j = lane; j < nS; j += 64) {
    double m[4], rv[NC];
#pragma unroll
    for (int q = 0; q < 4; ++q) m[q] = row[q][j];
#pragma unroll
    for (int c = 0; c < NC; ++c) rv[c] = r[c][j];
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int c = 0; c < NC; ++c) acc[q][c] = fma(m[q], rv[c], acc[q][c]);
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int a = a0 + q;
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      const double v = wave_sum(acc[q][c]);
      if (lane == 0 && on[c] && a < nS) {
        if (a < P.sub_nsep)
          c2[(int64_t)(c0 + c) * P.d + P.sub_sep_iface[a]] = v;
        else
          P.cws[(int64_t)(c0 + c) * P.cws_stride + sub_part_len(P) + nS] = v;  // lambda
      }
    }
  }
}

// x_p = y_p - F_p [x_B; lambda] (transpose: - R_p^T [x_B; lambda]) over the interior.
__global__ __launch_bounds__(256) void k_sub_patch2(DevPlan P, double* __restrict__ c2, int transpose,
                                                    const int* __restrict__ active) {
  extern __shared__ double xl[];
  const int pp = blockIdx.x, col = blockIdx.y;
  if (active && !active[col]) return;
  const int i0 = P.sub_I_off[pp], ni = P.sub_I_off[pp + 1] - i0;
  const int b0 = P.sub_B_off[pp], nb = P.sub_B_off[pp + 1] - b0, nbb = nb + P.sub_border;
  double* cc = c2 + (int64_t)col * P.d;
  const double* ws = P.cws + (int64_t)col * P.cws_stride;
  for (int l = threadIdx.x; l < nbb; l += blockDim.x)
    xl[l] = l < nb ? cc[P.sub_B_iface[b0 + l]] : ws[sub_part_len(P) + P.sub_nsep + P.sub_border];
  __syncthreads();
  const double* M = (transpose ? P.sub_Rr : P.sub_Fc) + P.sub_FR_off[pp];
  for (int row = threadIdx.x; row < ni; row += blockDim.x) {
    double acc = cc[P.sub_I[i0 + row]];
    // the row's entries 32 at a time (clamped in the last batch), products in order
    for (int l0 = 0; l0 < nbb; l0 += 32) {
      double mv[32];
#pragma unroll
      for (int u = 0; u < 32; ++u) mv[u] = M[(int64_t)min(l0 + u, nbb - 1) * ni + row];
#pragma unroll
      for (int u = 0; u < 32; ++u)
        if (l0 + u < nbb) acc = fma(-mv[u], xl[l0 + u], acc);
    }
    cc[P.sub_I[i0 + row]] = acc;
  }
}

// c2 = G c with c_j = side_sums[a_j] + side_sums[b_j] (the two sides of interface j).
__global__ __launch_bounds__(256) void k_coarse_sides(DevPlan P, const double* __restrict__ ss,
                                                      double* __restrict__ c2, int transpose,
                                                      const int* __restrict__ active) {
  __shared__ double cs[kDenseCoarseMax];
  const int col = blockIdx.y;
  const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int d = P.d;
  // the first 512 entries of this wave's row of G (or G^T): they need nothing else,
  // so their loads are issued before the column's activity and the sums are read
  const double* Gp = (transpose ? P.GT : P.G) + (int64_t)min(i, d - 1) * d;
  double g0[8];
#pragma unroll
  for (int u = 0; u < 8; ++u) g0[u] = Gp[min(lane + u * 64, d - 1)];
  // the first round's interface side indices, also before the activity check
  int sa0[4], sb0[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int j = min((int)threadIdx.x + u * 256, d - 1);
    sa0[u] = P.iface_side[2 * j];
    sb0[u] = P.iface_side[2 * j + 1];
  }
  if (active && !active[col]) return;
  const double* sc = ss + (int64_t)col * P.nsides;
  // the interface sums c_j = s(side a) + s(side b) into LDS, four per thread and
  // round: the index loads, then the gathers, are issued together
  for (int j0 = threadIdx.x; j0 < d; j0 += 4 * 256) {
    int sa[4], sb[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int j = min(j0 + u * 256, d - 1);
      sa[u] = j0 == (int)threadIdx.x ? sa0[u] : P.iface_side[2 * j];
      sb[u] = j0 == (int)threadIdx.x ? sb0[u] : P.iface_side[2 * j + 1];
    }
    double va[4], vb[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      va[u] = sc[sa[u]];
      vb[u] = sc[sb[u]];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (j0 + u * 256 < d) cs[j0 + u * 256] = va[u] + vb[u];
  }
  __syncthreads();
  if (i >= d) return;
  // the row's products in lane order (j = lane, lane + 64, ...), its loads eight at a time
  double acc = 0.0;
#pragma unroll
  for (int u = 0; u < 8; ++u)
    if (lane + u * 64 < d) acc = fma(g0[u], cs[lane + u * 64], acc);
  for (int j0 = lane + 8 * 64; j0 < d; j0 += 8 * 64) {
    double g[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) g[u] = Gp[min(j0 + u * 64, d - 1)];
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (j0 + u * 64 < d) acc = fma(g[u], cs[j0 + u * 64], acc);
  }
  acc = wave_sum(acc);
  if (lane == 0) c2[(int64_t)col * d + i] = acc;
}

// w = t + sign * (Z c2 + {0, S Z c2, S^T Z c2})
__global__ void k_prolong(DevPlan P, const double* __restrict__ t, const double* __restrict__ c2,
                          double* __restrict__ w, int sz, double sign, const int* __restrict__ active) {
  const int col = blockIdx.y;
  if (active && !active[col]) return;
  const int64_t slot = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (slot >= P.k) return;
  const double* cc = c2 + (int64_t)col * P.d;
  double acc;
  if (sz == 1 || sz == 2) {
    acc = deflation(P, cc, slot, sz == 2);
  } else {
    const int si = (int)(slot / P.n);
    acc = cc[P.iface[P.side_elem[si] * 4 + P.side_dir[si]]];
  }
  const int64_t o = (int64_t)col * P.k + slot;
  w[o] = t[o] + sign * acc;
}

// ------------------------------------------------------------------ boundary data

__global__ void k_copy(const double* __restrict__ a, double* __restrict__ b, int64_t len) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < len) b[i] = a[i];
}

// deterministic test pattern in (-1, 1) (hash of the index), for timing runs
__global__ void k_fill_pattern(double* __restrict__ b, int64_t len) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= len) return;
  uint64_t h = (uint64_t)i * 0x9E3779B97F4A7C15ull;
  h ^= h >> 31;
  h *= 0xBF58476D1CE4E5B9ull;
  h ^= h >> 29;
  b[i] = (double)(h >> 11) * (2.0 / 9007199254740992.0) - 1.0;
}

// b = a, and *flag = 1 if an entry of a is not finite (threads that see one store 1;
// the flag is cleared by the caller)
__global__ void k_copy_check(const double* __restrict__ a, double* __restrict__ b, int64_t len, int* flag) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= len) return;
  const double v = a[i];
  b[i] = v;
  if (!isfinite(v)) *flag = 1;
}

__global__ void k_check_finite(const double* __restrict__ a, int64_t len, int* flag) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < len && !isfinite(a[i])) *flag = 1;
}

// rhs[node] += tau g over boundary entries [b0, b1) (a range whose nodes are distinct);
// *flag = 1 for a non-finite g entry
__global__ void k_bdry_add(DevPlan P, const double* __restrict__ g, double* __restrict__ rhs, int64_t b0, int64_t b1,
                           int* flag) {
  const int col = blockIdx.y;
  const int64_t b = b0 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= b1) return;
  const double gv = g[(int64_t)col * P.nbdry + b];
  if (!isfinite(gv)) *flag = 1;
  rhs[(int64_t)col * P.r + P.bdry_node[b]] += P.bdry_tau[b] * gv;
}

__global__ void k_bdry_adj(DevPlan P, const double* __restrict__ mu, double* __restrict__ dg) {
  const int col = blockIdx.y;
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= P.nbdry) return;
  dg[(int64_t)col * P.nbdry + b] = P.bdry_tau[b] * mu[(int64_t)col * P.r + P.bdry_node[b]];
}

// ------------------------------------------------------------------ results to pinned host memory

// Device values copied by a kernel into pinned host memory (mapped, coherent): one
// small launch instead of a DMA copy.  The host reads them after an event/stream wait.
__global__ void k_publish(const double* __restrict__ src, int n, double* dst) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = src[i];
}
__global__ void k_publish_i(const int* __restrict__ src, int n, int* dst) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = src[i];
}
__global__ __launch_bounds__(256) void k_publish_set(PublishSet p) {
  for (int q = 0; q < 8; ++q)
    for (int i = threadIdx.x; i < p.n[q]; i += 256) p.dst[q][i] = p.src[q][i];
  for (int i = threadIdx.x; i < p.in; i += 256) p.idst[i] = p.isrc[i];
}
// ------------------------------------------------------------------ vector kernels

constexpr int kChunk = 2048;   // elements per reduction chunk (256 threads x 8)
constexpr int kVecGroup = 8;   // vectors per block in the multi-dot

__device__ __forceinline__ double block_sum_256(double v, double* red) {
  v = wave_sum(v);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  return (red[0] + red[1]) + (red[2] + red[3]);
}

__global__ __launch_bounds__(256) void k_mdot_part(const double* __restrict__ A, int64_t a_vs, int64_t a_cs, int nvec,
                                                   const double* __restrict__ b, int64_t b_cs,
                                                   const double* __restrict__ wt, int64_t len, int nchunks,
                                                   double* __restrict__ part, const int* __restrict__ active) {
  __shared__ double red[4];
  const int chunk = blockIdx.x, grp = blockIdx.y, col = blockIdx.z;
  if (active && !active[col]) return;
  const int64_t x0 = (int64_t)chunk * kChunk;
  double bv[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const int64_t x = x0 + q * 256 + threadIdx.x;
    double v = x < len ? b[(int64_t)col * b_cs + x] : 0.0;
    if (wt && x < len) v *= wt[x];
    bv[q] = v;
  }
  const int i0 = grp * kVecGroup;
  const int i1 = min(nvec, i0 + kVecGroup);
  for (int i = i0; i < i1; ++i) {
    const double* a = A + (int64_t)col * a_cs + (int64_t)i * a_vs;
    double acc = 0.0;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int64_t x = x0 + q * 256 + threadIdx.x;
      if (x < len) acc = fma(a[x], bv[q], acc);
    }
    const double s = block_sum_256(acc, red);
    if (threadIdx.x == 0) part[((int64_t)col * nvec + i) * nchunks + chunk] = s;
  }
}

__global__ void k_mdot_final(const double* __restrict__ part, int nvec, int nchunks, int nrhs,
                             double* __restrict__ out, const int* __restrict__ active) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= nvec * nrhs) return;
  const int col = idx / nvec;
  if (active && !active[col]) return;
  const double* p = part + (int64_t)idx * nchunks;
  double acc = 0.0;
  for (int c = 0; c < nchunks; ++c) acc += p[c];
  out[idx] = acc;
}

// Partial sums of |a + sb b|^2 over the chunk of k_mdot_part (same element order and
// tree as k_mdot_part of that vector with itself).
__global__ __launch_bounds__(256) void k_norm2_diff_part(const double* __restrict__ a, const double* __restrict__ b,
                                                         double sb, int64_t len, int nchunks,
                                                         double* __restrict__ part) {
  __shared__ double red[4];
  const int chunk = blockIdx.x, col = blockIdx.y;
  const int64_t x0 = (int64_t)chunk * kChunk;
  double dv[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const int64_t x = x0 + q * 256 + threadIdx.x;
    dv[q] = x < len ? a[(int64_t)col * len + x] + sb * b[(int64_t)col * len + x] : 0.0;
  }
  double acc = 0.0;
#pragma unroll
  for (int q = 0; q < 8; ++q)
    if (x0 + q * 256 + threadIdx.x < len) acc = fma(dv[q], dv[q], acc);
  const double sum = block_sum_256(acc, red);
  if (threadIdx.x == 0) part[(int64_t)col * nchunks + chunk] = sum;
}

// y = x - dot[col] * scale * u written, with the partial sums of |y|^2 as above
// (with sides != nullptr, also the sums of y over each run of n consecutive entries,
// n a power of two <= 64: the per-side sums of a slot vector)
__global__ __launch_bounds__(256) void k_axpy_norm2_part(const double* __restrict__ xv, const double* __restrict__ u,
                                                         const double* __restrict__ dot, double scale,
                                                         double* __restrict__ y, int64_t len, int nchunks,
                                                         double* __restrict__ part, double* __restrict__ sides,
                                                         int n) {
  __shared__ double red[4];
  const int chunk = blockIdx.x, col = blockIdx.y;
  const int64_t x0 = (int64_t)chunk * kChunk;
  double yv[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const int64_t x = x0 + q * 256 + threadIdx.x;
    yv[q] = 0.0;
    if (x < len) {
      yv[q] = xv[(int64_t)col * len + x] - dot[col] * scale * u[x];
      y[(int64_t)col * len + x] = yv[q];
    }
  }
  double acc = 0.0;
#pragma unroll
  for (int q = 0; q < 8; ++q)
    if (x0 + q * 256 + threadIdx.x < len) acc = fma(yv[q], yv[q], acc);
  if (sides) {
    // n consecutive lanes hold one side's entries for each q: a butterfly over them
    const int64_t nsides = len / n;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      double v = yv[q];
      for (int off = n >> 1; off > 0; off >>= 1) v += __shfl_xor(v, off);
      const int64_t x = x0 + q * 256 + threadIdx.x;
      if ((threadIdx.x & (n - 1)) == 0 && x / n < nsides) sides[(int64_t)col * nsides + x / n] = v;
    }
  }
  const double sum = block_sum_256(acc, red);
  if (threadIdx.x == 0) part[(int64_t)col * nchunks + chunk] = sum;
}

__global__ __launch_bounds__(256) void k_mupdate(double* __restrict__ w, int64_t w_cs, const double* __restrict__ A,
                                                 int64_t a_vs, int64_t a_cs, int nvec, const double* __restrict__ coef,
                                                 double scale, int64_t len, const int* __restrict__ active) {
  const int col = blockIdx.y;
  if (active && !active[col]) return;
  const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= len) return;
  const double* a = A + (int64_t)col * a_cs + x;
  const double* cf = coef + (int64_t)col * nvec;
  double acc = 0.0;
  for (int i = 0; i < nvec; ++i) acc = fma(cf[i], a[(int64_t)i * a_vs], acc);
  w[(int64_t)col * w_cs + x] -= scale * acc;
}

__global__ void k_axpy_shared(const double* __restrict__ x, int64_t x_cs, const double* __restrict__ u,
                              const double* __restrict__ dot, double scale, double* __restrict__ y, int64_t len) {
  const int col = blockIdx.y;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= len) return;
  y[(int64_t)col * len + i] = x[(int64_t)col * x_cs + i] - dot[col] * scale * u[i];
}

__global__ void k_scale_inv(const double* __restrict__ x, int64_t x_cs, const double* __restrict__ nrm, int sq,
                            double* __restrict__ y, int64_t y_cs, int64_t len, const int* __restrict__ active) {
  const int col = blockIdx.y;
  if (active && !active[col]) return;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= len) return;
  const double v = sq ? sqrt(nrm[col]) : nrm[col];
  y[(int64_t)col * y_cs + i] = v > 0.0 ? x[(int64_t)col * x_cs + i] / v : 0.0;
}

__global__ void k_add(const double* __restrict__ a, const double* __restrict__ b, double sb,
                      double* __restrict__ y, int64_t len) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < len) y[i] = a[i] + sb * b[i];
}

// ------------------------------------------------------------------ GMRES small work

__global__ void k_givens(double* H, int ldh, int maxit, double* cs, double* sn, double* g, const double* hnew,
                         const double* nrm2, int j, int nrhs, double* res, const int* active) {
  const int col = blockIdx.x * blockDim.x + threadIdx.x;
  if (col >= nrhs) return;
  if (active && !active[col]) return;
  double* Hc = H + (int64_t)col * ldh * maxit + (int64_t)j * ldh;
  double* csc = cs + (int64_t)col * ldh;
  double* snc = sn + (int64_t)col * ldh;
  double* gc = g + (int64_t)col * ldh;
  for (int i = 0; i <= j; ++i) Hc[i] = hnew[(int64_t)col * (j + 1) + i];
  Hc[j + 1] = sqrt(nrm2[col]);
  for (int i = 0; i < j; ++i) {
    const double a = Hc[i], b = Hc[i + 1];
    Hc[i] = csc[i] * a + snc[i] * b;
    Hc[i + 1] = -snc[i] * a + csc[i] * b;
  }
  const double a = Hc[j], b = Hc[j + 1];
  const double rr = hypot(a, b);
  const double c = rr > 0.0 ? a / rr : 1.0;
  const double s = rr > 0.0 ? b / rr : 0.0;
  csc[j] = c;
  snc[j] = s;
  Hc[j] = rr;
  Hc[j + 1] = 0.0;
  gc[j + 1] = -s * gc[j];
  gc[j] = c * gc[j];
  res[col] = fabs(gc[j + 1]);
}

__global__ void k_lsq(const double* H, int ldh, int maxit, const double* g, const int* jcount, double* y, int nrhs) {
  const int col = blockIdx.x * blockDim.x + threadIdx.x;
  if (col >= nrhs) return;
  const int J = jcount[col];
  const double* Hc = H + (int64_t)col * ldh * maxit;
  const double* gc = g + (int64_t)col * ldh;
  double* yc = y + (int64_t)col * maxit;
  for (int i = J; i < maxit; ++i) yc[i] = 0.0;
  for (int i = J - 1; i >= 0; --i) {
    double acc = gc[i];
    for (int m = i + 1; m < J; ++m) acc -= Hc[(int64_t)m * ldh + i] * yc[m];
    yc[i] = acc / Hc[(int64_t)i * ldh + i];
  }
}

inline dim3 grid1(int64_t len, int bs, int ny = 1) { return dim3((unsigned)((len + bs - 1) / bs), ny); }

}  // namespace

// ------------------------------------------------------------------ launchers

size_t sub_patch_lds(const DevPlan& P) { return (size_t)P.sub_lds_max * sizeof(double); }

bool schur_has_side_sums(const DevPlan& P) { return 4 * P.n <= 64; }

// Persistent Schur apply when there are enough work items for every resident workgroup
// to take at least two (or when forced by a positive P.schur_pers of the class).  Returns false if the plain
// launch should be used instead.
template <int KT, int NC, typename T>
static bool pers_launch(const DevPlan& P, const double* y, double* t, int nrhs, bool transpose,
                        const int* active, hipStream_t s) {
  const size_t lds = (size_t)2 * NC * 4 * KT * kTileLd * sizeof(typename AccOf<T>::type);
  const int ncg = (nrhs + NC - 1) / NC;
  const int64_t nitems = (int64_t)P.ntile * ncg;
  static std::atomic<int> occ[2] = {0, 0};  // resident workgroups per CU, per direction
  int oc = occ[transpose ? 1 : 0].load(std::memory_order_relaxed);
  if (oc == 0) {
    int v = 0;
    const hipError_t e = transpose
        ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&v, k_schur_mfma_pers<true, KT, NC, T>, 16 * KT, lds)
        : hipOccupancyMaxActiveBlocksPerMultiprocessor(&v, k_schur_mfma_pers<false, KT, NC, T>, 16 * KT, lds);
    oc = (e == hipSuccess && v > 0) ? v : 1;
    occ[transpose ? 1 : 0].store(oc, std::memory_order_relaxed);
  }
  const int64_t resident = (int64_t)P.num_cu * oc;
  if (P.schur_pers[schur_nc_class(nrhs)] == 0 && nitems < 2 * resident) return false;
  int64_t blocks = std::min<int64_t>(resident, nitems);
  blocks = (blocks + 7) / 8 * 8;
  const dim3 g((unsigned)blocks), b(16 * KT);
  if (transpose)
    hipLaunchKernelGGL((k_schur_mfma_pers<true, KT, NC, T>), g, b, lds, s, P, y, t, nrhs, active, ncg);
  else
    hipLaunchKernelGGL((k_schur_mfma_pers<false, KT, NC, T>), g, b, lds, s, P, y, t, nrhs, active, ncg);
  return true;
}

template <int KT, typename T>
static bool pers_nc(const DevPlan& P, const double* y, double* t, int nrhs, bool tr, const int* active,
                    hipStream_t s) {
  return nrhs >= 2 ? pers_launch<KT, 2, T>(P, y, t, nrhs, tr, active, s)
                   : pers_launch<KT, 1, T>(P, y, t, nrhs, tr, active, s);
}

template <int KT>
static bool pers_prec(const DevPlan& P, const double* y, double* t, int nrhs, bool tr, const int* active,
                      hipStream_t s, int prec) {
  if (prec == PREC_F32) return pers_nc<KT, float>(P, y, t, nrhs, tr, active, s);
  if (prec == PREC_BF16) return pers_nc<KT, bf16s>(P, y, t, nrhs, tr, active, s);
  return pers_nc<KT, double>(P, y, t, nrhs, tr, active, s);
}

// Column-pipelined Schur apply (no side sums): one workgroup per (tile, group of cpw
// columns, cpw = 1, 2, 4 or 8); cpw from the tuned value of the column-count class, else 8.
template <int KT, typename T, bool NTS>
static void cols_launch(const DevPlan& P, const double* y, double* t, int nrhs, bool transpose, const int* active,
                        hipStream_t s, int cpw) {
  const size_t lds = (size_t)3 * 4 * KT * kTileLd * sizeof(typename AccOf<T>::type);
  const int c = cpw >= 8 ? 8 : cpw >= 4 ? 4 : cpw >= 2 ? 2 : 1;
  const dim3 g((P.ntile + 7) / 8 * 8, (nrhs + c - 1) / c), b(16 * KT);
#define SMPM_COLS_LAUNCH(C)                                                                                    \
  if (transpose)                                                                                               \
    hipLaunchKernelGGL((k_schur_cols<true, KT, C, T, NTS>), g, b, lds, s, P, y, t, nrhs, active);              \
  else                                                                                                         \
    hipLaunchKernelGGL((k_schur_cols<false, KT, C, T, NTS>), g, b, lds, s, P, y, t, nrhs, active);
  if (c == 8) {
    SMPM_COLS_LAUNCH(8)
  } else if (c == 4) {
    SMPM_COLS_LAUNCH(4)
  } else if (c == 2) {
    SMPM_COLS_LAUNCH(2)
  } else {
    SMPM_COLS_LAUNCH(1)
  }
#undef SMPM_COLS_LAUNCH
}

template <int KT>
static void cols_prec(const DevPlan& P, const double* y, double* t, int nrhs, bool tr, const int* active,
                      hipStream_t s, int prec, int cpw, bool nts) {
  if (prec == PREC_F32)
    cols_launch<KT, float, false>(P, y, t, nrhs, tr, active, s, cpw);
  else if (prec == PREC_BF16)
    cols_launch<KT, bf16s, false>(P, y, t, nrhs, tr, active, s, cpw);
  else if (nts)
    cols_launch<KT, double, true>(P, y, t, nrhs, tr, active, s, cpw);
  else
    cols_launch<KT, double, false>(P, y, t, nrhs, tr, active, s, cpw);
}

static void launch_schur_cols(const DevPlan& P, const double* y, double* t, int nrhs, bool transpose,
                              const int* active, hipStream_t s, int prec, bool nts) {
  const int tuned = P.schur_cpw[schur_nc_class(nrhs)];
  const int cpw = tuned > 0 ? tuned : 8;
  switch (4 * P.mma_mt) {
    case 4: cols_prec<4>(P, y, t, nrhs, transpose, active, s, prec, cpw, nts); break;
    case 8: cols_prec<8>(P, y, t, nrhs, transpose, active, s, prec, cpw, nts); break;
    case 12: cols_prec<12>(P, y, t, nrhs, transpose, active, s, prec, cpw, nts); break;
    default: cols_prec<16>(P, y, t, nrhs, transpose, active, s, prec, cpw, nts); break;
  }
}

// Warp-specialized persistent Schur apply (no side sums): one workgroup per resident
// slot of the device, items (tile, column group) split over the XCDs.
template <int KT, int NC, typename T, bool NTS>
static void ws_launch(const DevPlan& P, const double* y, double* t, int nrhs, bool transpose, const int* active,
                      hipStream_t s) {
  const size_t lds = (size_t)4 * NC * 4 * KT * kTileLd * sizeof(typename AccOf<T>::type);
  const int ncg = (nrhs + NC - 1) / NC;
  const int64_t nitems = (int64_t)P.ntile * ncg;
  static std::atomic<int> occ[2] = {0, 0};  // resident workgroups per CU, per direction
  int oc = occ[transpose ? 1 : 0].load(std::memory_order_relaxed);
  if (oc == 0) {
    int v = 0;
    const hipError_t e = transpose
        ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&v, k_schur_ws<true, KT, NC, T, NTS>, 32 * KT, lds)
        : hipOccupancyMaxActiveBlocksPerMultiprocessor(&v, k_schur_ws<false, KT, NC, T, NTS>, 32 * KT, lds);
    oc = (e == hipSuccess && v > 0) ? v : 1;
    occ[transpose ? 1 : 0].store(oc, std::memory_order_relaxed);
  }
  int64_t blocks = std::min<int64_t>((int64_t)P.num_cu * oc, nitems);
  blocks = (blocks + 7) / 8 * 8;
  const dim3 g((unsigned)blocks), b(32 * KT);
  if (transpose)
    hipLaunchKernelGGL((k_schur_ws<true, KT, NC, T, NTS>), g, b, lds, s, P, y, t, nrhs, active, ncg);
  else
    hipLaunchKernelGGL((k_schur_ws<false, KT, NC, T, NTS>), g, b, lds, s, P, y, t, nrhs, active, ncg);
}

template <int KT, typename T, bool NTS>
static void ws_nc(const DevPlan& P, const double* y, double* t, int nrhs, bool tr, const int* active,
                  hipStream_t s, int nc) {
  if (nc >= 4 && nrhs >= 4)
    ws_launch<KT, 4, T, NTS>(P, y, t, nrhs, tr, active, s);
  else if (nc >= 2 && nrhs >= 2)
    ws_launch<KT, 2, T, NTS>(P, y, t, nrhs, tr, active, s);
  else
    ws_launch<KT, 1, T, NTS>(P, y, t, nrhs, tr, active, s);
}

template <int KT>
static void ws_prec(const DevPlan& P, const double* y, double* t, int nrhs, bool tr, const int* active,
                    hipStream_t s, int prec, int nc, bool nts) {
  if (prec == PREC_F32)
    ws_nc<KT, float, false>(P, y, t, nrhs, tr, active, s, nc);
  else if (prec == PREC_BF16)
    ws_nc<KT, bf16s, false>(P, y, t, nrhs, tr, active, s, nc);
  else if (nts)
    ws_nc<KT, double, true>(P, y, t, nrhs, tr, active, s, nc);
  else
    ws_nc<KT, double, false>(P, y, t, nrhs, tr, active, s, nc);
}

static void launch_schur_ws(const DevPlan& P, const double* y, double* t, int nrhs, bool transpose,
                            const int* active, hipStream_t s, int prec, bool nts) {
  const int tuned = P.schur_nc[schur_nc_class(nrhs)];
  const int nc = tuned > 0 ? tuned : 2;
  switch (4 * P.mma_mt) {
    case 4: ws_prec<4>(P, y, t, nrhs, transpose, active, s, prec, nc, nts); break;
    case 8: ws_prec<8>(P, y, t, nrhs, transpose, active, s, prec, nc, nts); break;
    case 12: ws_prec<12>(P, y, t, nrhs, transpose, active, s, prec, nc, nts); break;
    default: ws_prec<16>(P, y, t, nrhs, transpose, active, s, prec, nc, nts); break;
  }
}

bool launch_schur_pers(const DevPlan& P, const double* y, double* t, int nrhs, bool transpose, const int* active,
                       hipStream_t s, int prec) {
  switch (4 * P.mma_mt) {
    case 4: return pers_prec<4>(P, y, t, nrhs, transpose, active, s, prec);
    case 8: return pers_prec<8>(P, y, t, nrhs, transpose, active, s, prec);
    case 12: return pers_prec<12>(P, y, t, nrhs, transpose, active, s, prec);
    default: return pers_prec<16>(P, y, t, nrhs, transpose, active, s, prec);
  }
}

int schur_nc_class(int nrhs) { return nrhs <= 1 ? 0 : nrhs <= 3 ? 1 : nrhs <= 7 ? 2 : 3; }

void launch_schur(const DevPlan& P, const double* y, double* t, int nrhs, bool transpose, const int* active,
                  hipStream_t s) {
  launch_schur_ex(P, y, t, nrhs, transpose, active, nullptr, s);
}

void launch_schur_ex(const DevPlan& P, const double* y, double* t, int nrhs, bool transpose, const int* active,
                     double* side_sums, hipStream_t s, int prec, bool stream_out) {
  if (transpose || !schur_has_side_sums(P)) side_sums = nullptr;
  if (P.mma_mt > 0 && !side_sums && P.schur_pers[schur_nc_class(nrhs)] == 2) {
    launch_schur_ws(P, y, t, nrhs, transpose, active, s, prec, stream_out);
    return;
  }
  if (P.mma_mt > 0 && !side_sums && P.schur_pers[schur_nc_class(nrhs)] == 3) {
    launch_schur_cols(P, y, t, nrhs, transpose, active, s, prec, stream_out);
    return;
  }
  if (P.mma_mt > 0 && !side_sums && P.schur_pers[schur_nc_class(nrhs)] >= 0 && launch_schur_pers(P, y, t, nrhs, transpose, active, s, prec))
    return;
  if (P.mma_mt > 0) {
    // matrix-core path: one workgroup per tile and NC columns, one wavefront per 16 rows
    const int kt = 4 * P.mma_mt;
    // columns per workgroup: the tuned value of this column-count class, capped at nrhs
    const int tuned = P.schur_nc[schur_nc_class(nrhs)];
    int nc = tuned > 0 ? tuned : (nrhs >= 4 ? 4 : nrhs >= 2 ? 2 : 1);
    while (nc > 1 && nc > nrhs) nc >>= 1;
    const size_t acc = prec == PREC_F64 ? sizeof(double) : sizeof(float);
    // side-sum partials only when side sums are requested
    const size_t lds = ((size_t)nc * 4 * kt * kTileLd * acc + 7) / 8 * 8 +
                       (side_sums ? (size_t)nc * kTile * 4 * (kt / 4) * sizeof(double) : 0);
    const dim3 g((P.ntile + 7) / 8 * 8, (nrhs + nc - 1) / nc);
    const dim3 b(16 * kt);
#define SMPM_MFMA_LAUNCH(KT, NC, T, NTS)                                                                       \
  if (transpose)                                                                                               \
    hipLaunchKernelGGL((k_schur_mfma<true, KT, NC, T, NTS>), g, b, lds, s, P, y, t, nrhs, active, nullptr);    \
  else                                                                                                         \
    hipLaunchKernelGGL((k_schur_mfma<false, KT, NC, T, NTS>), g, b, lds, s, P, y, t, nrhs, active, side_sums);
#define SMPM_MFMA_NC(KT, T, NTS)            \
  if (nc == 4) {                            \
    SMPM_MFMA_LAUNCH(KT, 4, T, NTS)         \
  } else if (nc == 2) {                     \
    SMPM_MFMA_LAUNCH(KT, 2, T, NTS)         \
  } else {                                  \
    SMPM_MFMA_LAUNCH(KT, 1, T, NTS)         \
  }
#define SMPM_MFMA_PREC(KT)              \
  if (prec == PREC_F32) {               \
    SMPM_MFMA_NC(KT, float, false)      \
  } else if (prec == PREC_BF16) {       \
    SMPM_MFMA_NC(KT, bf16s, false)      \
  } else if (stream_out) {              \
    SMPM_MFMA_NC(KT, double, true)      \
  } else {                              \
    SMPM_MFMA_NC(KT, double, false)     \
  }
    switch (kt) {
      case 4: SMPM_MFMA_PREC(4) break;
      case 8: SMPM_MFMA_PREC(8) break;
      case 12: SMPM_MFMA_PREC(12) break;
      default: SMPM_MFMA_PREC(16) break;
    }
#undef SMPM_MFMA_PREC
#undef SMPM_MFMA_NC
#undef SMPM_MFMA_LAUNCH
    return;
  }
  const int blocks = ((P.ngrp + 3) / 4 + 7) / 8 * 8;  // a multiple of the 8 XCDs
  const size_t lds = (size_t)4 * P.grp_size * 4 * P.n * sizeof(double);
  dim3 g(blocks, nrhs);
#define SMPM_SCHUR_LAUNCH(G, T)                                                       \
  if (transpose)                                                                      \
    hipLaunchKernelGGL((k_schur_adj<G, T>), g, dim3(256), lds, s, P, y, t, active);   \
  else                                                                                \
    hipLaunchKernelGGL((k_schur_fwd<G, T>), g, dim3(256), lds, s, P, y, t, active, side_sums);
#define SMPM_SCHUR_PREC(G)                                  \
  if (prec == PREC_F32) {                                   \
    SMPM_SCHUR_LAUNCH(G, float)                             \
  } else if (prec == PREC_BF16) {                           \
    SMPM_SCHUR_LAUNCH(G, bf16s)                             \
  } else {                                                  \
    SMPM_SCHUR_LAUNCH(G, double)                            \
  }
  switch (P.grp_size) {
    case 1: SMPM_SCHUR_PREC(1) break;
    case 2: SMPM_SCHUR_PREC(2) break;
    case 4: SMPM_SCHUR_PREC(4) break;
    default: SMPM_SCHUR_PREC(8) break;
  }
#undef SMPM_SCHUR_PREC
#undef SMPM_SCHUR_LAUNCH
}

void launch_flux(const DevPlan& P, const double* f, double* b, int nrhs, hipStream_t s) {
  if (P.mma_mt > 0 && P.n2 <= kMmaN2) {
    // a multiple of 8 workgroups, so that the XCD-aware order is a permutation of the tiles
    hipLaunchKernelGGL(k_flux_mfma, dim3((P.ntile + 7) / 8 * 8, nrhs), dim3(256), 0, s, P, f, b,
                       (const double*)nullptr, (const double*)nullptr, 0.0, (double*)nullptr, (const double*)nullptr,
                       (double*)nullptr);
    return;
  }
  hipLaunchKernelGGL(k_flux, dim3(P.nel, nrhs), dim3(64), 4 * P.n2 * sizeof(double), s, P, f, b);
}

bool launch_backsub_dot(const DevPlan& P, const double* f, const double* x, double* u, const double* wq, int nrhs,
                        double* part, double* out, hipStream_t s) {
  if (!(P.mma_mt > 0 && P.n2 <= kMmaN2)) return false;
  const dim3 g((P.ntile + 7) / 8 * 8, (P.n2 + 63) / 64, nrhs);
  hipLaunchKernelGGL(k_backsub_mfma, g, dim3(256), 0, s, P, f, x, u, wq, part);
  const int nblk = (int)(g.x * g.y);
  hipLaunchKernelGGL(k_mdot_final, grid1((int64_t)nrhs, 128), dim3(128), 0, s, part, 1, nblk, nrhs, out,
                     (const int*)nullptr);
  return true;
}

bool launch_flux_projected(const DevPlan& P, const double* f, const double* u, const double* dot, double scale,
                           double* ft, double* b, int nrhs, hipStream_t s, const double* du, double* part,
                           double* dout) {
  if (!(P.mma_mt > 0 && P.n2 <= kMmaN2)) return false;
  const int nb = (P.ntile + 7) / 8 * 8;
  hipLaunchKernelGGL(k_flux_mfma, dim3(nb, nrhs), dim3(256), 0, s, P, f, b, u, dot, scale, ft, du, part);
  if (du)
    hipLaunchKernelGGL(k_mdot_final, grid1((int64_t)nrhs, 128), dim3(128), 0, s, part, 1, 4 * nb, nrhs, dout,
                       (const int*)nullptr);
  return true;
}

void launch_flux_adj(const DevPlan& P, const double* x, double* y, int nrhs, hipStream_t s) {
  hipLaunchKernelGGL(k_flux_adj, dim3(P.nel, nrhs), dim3(256), 0, s, P, x, y);
}

void launch_backsub(const DevPlan& P, const double* f, const double* x, double* u, int nrhs, hipStream_t s) {
  if (P.mma_mt > 0 && P.n2 <= kMmaN2) {
    hipLaunchKernelGGL(k_backsub_mfma, dim3((P.ntile + 7) / 8 * 8, (P.n2 + 63) / 64, nrhs), dim3(256), 0, s, P, f,
                       x, u, (const double*)nullptr, (double*)nullptr);
    return;
  }
  hipLaunchKernelGGL(k_backsub, dim3(P.nel, nrhs), dim3(256), P.n2 * sizeof(double), s, P, f, x, u);
}

void launch_local_adj(const DevPlan& P, const double* c, double* out, int nrhs, bool to_slots, hipStream_t s) {
  hipLaunchKernelGGL(k_local_adj, dim3(P.nel, nrhs), dim3(256), 2 * P.n2 * sizeof(double), s, P, c, out,
                     to_slots ? 1 : 0);
}

void launch_precond(const DevPlan& P, const double* x, double* y, int nrhs, bool transpose, const int* active,
                    hipStream_t s, int prec) {
  if (nrhs > 1) {
    // four columns per workgroup, each block inverse read once for them
    const dim3 g4(P.nblk, (nrhs + 3) / 4);
    const int tr = transpose ? 1 : 0;
    if (prec == PREC_F32)
      hipLaunchKernelGGL((k_precond_n<float, 4>), g4, dim3(256), 0, s, P, x, y, nrhs, tr, active);
    else if (prec == PREC_BF16)
      hipLaunchKernelGGL((k_precond_n<bf16s, 4>), g4, dim3(256), 0, s, P, x, y, nrhs, tr, active);
    else
      hipLaunchKernelGGL((k_precond_n<double, 4>), g4, dim3(256), 0, s, P, x, y, nrhs, tr, active);
    return;
  }
  const dim3 g(P.nblk, nrhs);
  if (prec == PREC_F32)
    hipLaunchKernelGGL(k_precond<float>, g, dim3(256), 0, s, P, x, y, transpose ? 1 : 0, active);
  else if (prec == PREC_BF16)
    hipLaunchKernelGGL(k_precond<bf16s>, g, dim3(256), 0, s, P, x, y, transpose ? 1 : 0, active);
  else
    hipLaunchKernelGGL(k_precond<double>, g, dim3(256), 0, s, P, x, y, transpose ? 1 : 0, active);
}

void launch_iface_sum(const DevPlan& P, const double* t, double* c, int nrhs, const int* active, hipStream_t s) {
  if (P.d == 0 || !P.has_coarse) return;
  hipLaunchKernelGGL(k_iface_sum, grid1(P.d, 2 * P.n <= 32 ? 8 : 4, nrhs), dim3(256), 0, s, P, t, c, active,
                     (const double*)nullptr, 0.0);
}

void launch_iface_sum_diff(const DevPlan& P, const double* a, const double* t, double sb, double* c, int nrhs,
                           hipStream_t s) {
  if (P.d == 0 || !P.has_coarse) return;
  hipLaunchKernelGGL(k_iface_sum, grid1(P.d, 2 * P.n <= 32 ? 8 : 4, nrhs), dim3(256), 0, s, P, t, c,
                     (const int*)nullptr, a, sb);
}

void launch_coarse(const DevPlan& P, const double* c, double* c2, int nrhs, bool transpose, const int* active,
                   hipStream_t s) {
  if (P.d == 0 || !P.has_coarse) return;
  const int tr = transpose ? 1 : 0;
  if (P.coarse_mode == 2) {
    const int nS = P.sub_nsep + P.sub_border;
    hipLaunchKernelGGL(k_sub_patch1, dim3(P.sub_npatch, nrhs), dim3(256), sub_patch_lds(P), s, P, c, c2, tr,
                       active);
    if (nS > 0) {
      hipLaunchKernelGGL(k_sub_rhs, dim3((nS + 255) / 256, nrhs), dim3(256), 0, s, P, c, active);
      if (nrhs >= 4)
        hipLaunchKernelGGL(k_sub_sep<4>, dim3((nS + 15) / 16, (nrhs + 3) / 4), dim3(256), 0, s, P, c2, tr, nrhs,
                           active);
      else
        hipLaunchKernelGGL(k_sub_sep<1>, dim3((nS + 15) / 16, nrhs), dim3(256), 0, s, P, c2, tr, nrhs, active);
      hipLaunchKernelGGL(k_sub_patch2, dim3(P.sub_npatch, nrhs), dim3(256), sub_patch_lds(P), s, P, c2, tr,
                         active);
    }
    return;
  }
  hipLaunchKernelGGL(k_coarse, grid1(P.d, 4, nrhs), dim3(256), 0, s, P, c, c2, tr, active);
}

void launch_coarse_sides(const DevPlan& P, const double* side_sums, double* c2, int nrhs, bool transpose,
                         const int* active, hipStream_t s) {
  // dense mode only: d <= dense_coarse_limit() <= kDenseCoarseMax, the kernel's LDS
  if (P.d == 0 || !P.has_coarse || P.coarse_mode != 1) return;
  hipLaunchKernelGGL(k_coarse_sides, grid1(P.d, 4, nrhs), dim3(256), 0, s, P, side_sums, c2, transpose ? 1 : 0,
                     active);
}

void launch_prolong(const DevPlan& P, const double* t, const double* c2, double* w, int nrhs, int sz, double sign,
                    const int* active, hipStream_t s) {
  hipLaunchKernelGGL(k_prolong, grid1(P.k, 256, nrhs), dim3(256), 0, s, P, t, c2, w, sz, sign, active);
}

void launch_rhs(const DevPlan& P, const double* f, const double* g, double* rhs, int nrhs, int* flag,
                hipStream_t s) {
  const int64_t len = P.r * nrhs;
  hipLaunchKernelGGL(k_copy_check, grid1(len, 256), dim3(256), 0, s, f, rhs, len, flag);
  if (!g) return;
  // south + north edges first (distinct nodes), then west + east edges (distinct nodes);
  // a domain-corner node receives one term from each launch
  const int64_t sn = 2 * (int64_t)P.mx * P.n;
  hipLaunchKernelGGL(k_bdry_add, grid1(sn, 256, nrhs), dim3(256), 0, s, P, g, rhs, (int64_t)0, sn, flag);
  hipLaunchKernelGGL(k_bdry_add, grid1(P.nbdry - sn, 256, nrhs), dim3(256), 0, s, P, g, rhs, sn, P.nbdry, flag);
}

void launch_copy(const double* a, double* b, int64_t len, hipStream_t s) {
  hipLaunchKernelGGL(k_copy, grid1(len, 256), dim3(256), 0, s, a, b, len);
}

void launch_check_finite(const double* a, int64_t len, int* flag, hipStream_t s) {
  hipLaunchKernelGGL(k_check_finite, grid1(len, 256), dim3(256), 0, s, a, len, flag);
}

void launch_bdry_adj(const DevPlan& P, const double* mu, double* dg, int nrhs, hipStream_t s) {
  hipLaunchKernelGGL(k_bdry_adj, grid1(P.nbdry, 256, nrhs), dim3(256), 0, s, P, mu, dg);
}

int reduce_chunks(int64_t len) { return (int)((len + kChunk - 1) / kChunk); }

void launch_fill_pattern(double* b, int64_t len, hipStream_t s) {
  hipLaunchKernelGGL(k_fill_pattern, grid1(len, 256), dim3(256), 0, s, b, len);
}

void launch_publish(const double* src, int n, double* host_dst, hipStream_t s) {
  hipLaunchKernelGGL(k_publish, dim3((n + 255) / 256), dim3(256), 0, s, src, n, host_dst);
}
void launch_publish_i(const int* src, int n, int* host_dst, hipStream_t s) {
  hipLaunchKernelGGL(k_publish_i, dim3((n + 255) / 256), dim3(256), 0, s, src, n, host_dst);
}
void launch_publish_set(const PublishSet& p, hipStream_t s) {
  hipLaunchKernelGGL(k_publish_set, dim3(1), dim3(256), 0, s, p);
}
void launch_mdot(const double* A, int64_t a_vs, int64_t a_cs, int nvec, const double* b, int64_t b_cs,
                 const double* wt, int64_t len, int nrhs, double* part, double* out, const int* active,
                 hipStream_t s) {
  const int nch = reduce_chunks(len);
  dim3 g(nch, (nvec + kVecGroup - 1) / kVecGroup, nrhs);
  hipLaunchKernelGGL(k_mdot_part, g, dim3(256), 0, s, A, a_vs, a_cs, nvec, b, b_cs, wt, len, nch, part, active);
  hipLaunchKernelGGL(k_mdot_final, grid1((int64_t)nvec * nrhs, 128), dim3(128), 0, s, part, nvec, nch, nrhs, out,
                     active);
}

void launch_norm2_diff(const double* a, const double* b, double sb, int64_t len, int nrhs, double* part, double* out,
                       hipStream_t s) {
  const int nch = reduce_chunks(len);
  hipLaunchKernelGGL(k_norm2_diff_part, dim3(nch, nrhs), dim3(256), 0, s, a, b, sb, len, nch, part);
  hipLaunchKernelGGL(k_mdot_final, grid1((int64_t)nrhs, 128), dim3(128), 0, s, part, 1, nch, nrhs, out,
                     (const int*)nullptr);
}

void launch_axpy_norm2(const double* x, const double* u, const double* dot, double scale, double* y, int64_t len,
                       int nrhs, double* part, double* out, hipStream_t s, double* sides, int n) {
  const int nch = reduce_chunks(len);
  hipLaunchKernelGGL(k_axpy_norm2_part, dim3(nch, nrhs), dim3(256), 0, s, x, u, dot, scale, y, len, nch, part,
                     sides, n);
  hipLaunchKernelGGL(k_mdot_final, grid1((int64_t)nrhs, 128), dim3(128), 0, s, part, 1, nch, nrhs, out,
                     (const int*)nullptr);
}

void launch_mupdate(double* w, int64_t w_cs, const double* A, int64_t a_vs, int64_t a_cs, int nvec,
                    const double* coef, double scale, int64_t len, int nrhs, const int* active, hipStream_t s) {
  hipLaunchKernelGGL(k_mupdate, grid1(len, 256, nrhs), dim3(256), 0, s, w, w_cs, A, a_vs, a_cs, nvec, coef, scale,
                     len, active);
}

void launch_axpy_shared(const double* x, int64_t x_cs, const double* u, const double* dot, double scale, double* y,
                        int64_t len, int nrhs, hipStream_t s) {
  hipLaunchKernelGGL(k_axpy_shared, grid1(len, 256, nrhs), dim3(256), 0, s, x, x_cs, u, dot, scale, y, len);
}

void launch_scale_inv(const double* x, int64_t x_cs, const double* nrm, bool sq, double* y, int64_t y_cs,
                      int64_t len, int nrhs, const int* active, hipStream_t s) {
  hipLaunchKernelGGL(k_scale_inv, grid1(len, 256, nrhs), dim3(256), 0, s, x, x_cs, nrm, sq ? 1 : 0, y, y_cs, len,
                     active);
}

void launch_add(const double* a, const double* b, double sb, double* y, int64_t len, int nrhs, hipStream_t s) {
  const int64_t tot = len * nrhs;
  hipLaunchKernelGGL(k_add, grid1(tot, 256), dim3(256), 0, s, a, b, sb, y, tot);
}

void launch_givens(double* H, int ldh, double* cs, double* sn, double* g, const double* hnew, const double* nrm2,
                   int j, int nrhs, double* res, const int* active, hipStream_t s) {
  const int maxit = ldh - 1;
  hipLaunchKernelGGL(k_givens, grid1(nrhs, 64), dim3(64), 0, s, H, ldh, maxit, cs, sn, g, hnew, nrm2, j, nrhs, res,
                     active);
}

void launch_lsq(const double* H, int ldh, const double* g, const int* jcount, double* y, int nrhs, hipStream_t s) {
  const int maxit = ldh - 1;
  hipLaunchKernelGGL(k_lsq, grid1(nrhs, 64), dim3(64), 0, s, H, ldh, maxit, g, jcount, y, nrhs);
}

}  // namespace smpm
