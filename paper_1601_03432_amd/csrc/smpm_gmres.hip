// Device-resident GMRES iteration for the deflated Schur complement system.
//
// Arnoldi with classical Gram-Schmidt and delayed reorthogonalization (DCGS2, after
// Swirydowicz, Bielich, Langou, Thomas et al.): the operator is applied to the
// candidate vector u_j before it is reorthogonalized and normalized, and a single
// pass over the basis yields both the projections of w_j = A u_j and the
// reorthogonalization coefficients of u_j.  With Q_m = [q_0 .. q_{m-1}] the final
// basis and the candidate u_m stored in V_m:
//   dots   (d_i, c_i) = (q_i^T w_m, q_i^T u_m) for i < m, alpha = u_m^T w_m, nu = u_m^T u_m
//   rho    = sqrt(nu - |c|^2)                    (Pythagoras)
//   q_m    = (u_m - Q_m c) / rho                 Hessenberg column m-1 = h'_{m-1} + c, rho below
//   e      = q_m^T w_m = (alpha - c.d) / rho
//   u_{m+1}= (w_m - Q_m d - e q_m) / rho         (= A q_m projected once off Q_{m+1})
//   h'_m   = ([d; e] - H c) / rho                (= Q_{m+1}^T A q_m; H = the unrotated
//                                                 Hessenberg columns 0..m-1)
// so each step reads the basis twice (one dot pass, one update pass) instead of four
// times.  One step j is four kernels (five when the sums are pre-reduced) that read j
// from a device counter and keep every scalar on the device, so the host never waits
// inside the loop and a captured chunk of steps (hipGraph) replays for any j.  The
// counter is double-buffered: step q of a chunk reads slot q % 2 and its last kernel
// writes j + 1 into the other slot, so no kernel reads a value another block of it
// may be changing:
//   gm_update   (m = j - 1) rho, e from the previous dot pass; block 0 (alone)
//               applies the Givens rotations to Hessenberg column m-1, retires the
//               column once its residual estimate reaches tol * |b|, and forms h'_m;
//               the other blocks write q_m into V_m and u_{m+1} into V_{m+1} and
//               apply z = M^{-1} u_{m+1} (step 0: z = M^{-1} u_0)
//   Schur       t = S z, with the per-side sums of t for Z^T t
//   coarse      c2 = G Z^T t
//   gm_dots     w = t - Z c2 - S Z c2 (deflation); partial dots of V_0..V_j with w
//               and with u_j = V_j; next j
// Each block handles a chunk of rows.  Every block that needs a reduced value sums
// the previous kernel's per-chunk partials itself (or k_gm_reduce does it once per
// column), in one fixed order whatever the block shape, so results are
// deterministic and no inter-block fence is needed.  Basis loads become
// non-temporal once the part of the basis a pass reads outgrows the last-level cache.
#include <hip/hip_runtime.h>

#include "smpm_gmres.h"

#include <type_traits>

namespace smpm {

namespace {

constexpr int kThreads = 256;

// Basis entries are read once per pass.  Once the part of the basis a pass reads is
// larger than the last-level cache can keep (kStreamBytes; the 256 MB Infinity Cache
// also holds the other operands), caching it only evicts what is reused (block-Jacobi
// inverses, coefficients, partial sums): those loads are then non-temporal.  The
// choice is uniform over a launch.
constexpr int64_t kStreamBytes = 192ll << 20;
__device__ __forceinline__ bool stream_basis(int64_t nvec, int64_t vvs) { return nvec * vvs * 8 > kStreamBytes; }
template <bool NT, typename VT>
__device__ __forceinline__ double ld_basis(const VT* p) {
  if constexpr (NT)
    return (double)__builtin_nontemporal_load(p);
  else
    return (double)*p;
}
// The Krylov basis is stored in FP64, or in FP32 (a float view of the same buffer,
// same element strides) for the inner solves of mixed precision; all arithmetic is FP64.
template <typename VT>
__device__ __forceinline__ VT* basis(const GmState& S) {
  return reinterpret_cast<VT*>(S.V);
}
// kernels branch once on the choice and run a copy of their basis loops compiled for
// it (the tag is std::true_type or std::false_type)
template <typename Tag>
constexpr bool kNT = Tag::value;
constexpr int kWaves = kThreads / 64;
constexpr int kDotUnroll = 8;

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

// Sum over the 64 lanes, the same value on every lane: a butterfly inside each row of
// 16 lanes on DPP lane moves (partners lane ^ 1, lane ^ 2, then the half-row and row
// mirrors), then the four row sums read as scalars.  A fixed order, so every kernel
// that reduces the same lanes gets the same bits.  All 64 lanes must be active.
__device__ __forceinline__ double wave_sum(double v) {
  v += dpp_move<0xB1>(v);   // quad permutation 1 0 3 2
  v += dpp_move<0x4E>(v);   // quad permutation 2 3 0 1
  v += dpp_move<0x141>(v);  // half-row mirror
  v += dpp_move<0x140>(v);  // row mirror
  return (read_lane(v, 0) + read_lane(v, 16)) + (read_lane(v, 32) + read_lane(v, 48));
}

__device__ __forceinline__ double block_sum(double v, double* red) {
  v = wave_sum(v);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  return (red[0] + red[1]) + (red[2] + red[3]);
}

// oa[v] = sum_c pa[c*ld + v] and ob likewise, v < nvec (the dots' partials, one row of
// ld entries per chunk), with the loads of both arrays in flight together.  The
// order of the additions is fixed whatever the block shape: chunk c belongs to class
// c mod 16, a class sums its chunks in increasing c, and the class sums s_q are
// combined as (t_0 + t_1) + (t_2 + t_3) with t_r = (s_r + s_{r+4}) + (s_{r+8} +
// s_{r+12}); every block, of 4 or of 16 waves, obtains the same bits, and so does
// k_gm_reduce, which follows the same order with another lane mapping.  Lanes run
// over vectors (coalesced rows), the NW waves share the classes.  Vector groups
// g0, g0 + gstep, ... of 64.  lds: 2 * NW * 64 doubles.  Contains barriers: call from
// all threads of the block.
template <int NW>
__device__ void reduce_partials2(const double* __restrict__ pa, const double* __restrict__ pb, int nvec, int nch,
                                 int ld, double* oa, double* ob, double* lds, int g0 = 0, int gstep = 1) {
  static_assert(NW == 4 || NW == 16, "four or sixteen waves");
  constexpr int CPW = 16 / NW;  // classes of this wave: q = wave + NW * t
  constexpr int R = 16 / CPW;   // 16-chunk strides per batch: 2 * CPW * R = 32 loads in flight
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  for (int g = g0; g * 64 < nvec; g += gstep) {
    const int v = min(g * 64 + lane, nvec - 1);
    double sa[CPW], sb[CPW];
#pragma unroll
    for (int t = 0; t < CPW; ++t) sa[t] = sb[t] = 0.0;
    for (int c0 = 0; c0 < nch; c0 += 16 * R) {
      // chunks past nch repeat the last one (in bounds) and are not added
      double la[R][CPW], lb[R][CPW];
#pragma unroll
      for (int r = 0; r < R; ++r)
#pragma unroll
        for (int t = 0; t < CPW; ++t) {
          const int64_t at = (int64_t)min(c0 + 16 * r + wave + NW * t, nch - 1) * ld + v;
          la[r][t] = pa[at];
          lb[r][t] = pb[at];
        }
#pragma unroll
      for (int r = 0; r < R; ++r)
#pragma unroll
        for (int t = 0; t < CPW; ++t) {
          const bool ok = c0 + 16 * r + wave + NW * t < nch;
          sa[t] = ok ? sa[t] + la[r][t] : sa[t];
          sb[t] = ok ? sb[t] + lb[r][t] : sb[t];
        }
    }
    const int out = g * 64 + lane;
    if (NW == 4) {  // this wave holds s_w, s_{w+4}, s_{w+8}, s_{w+12}: t_w
      lds[wave * 64 + lane] = (sa[0] + sa[CPW > 1 ? 1 : 0]) + (sa[CPW > 2 ? 2 : 0] + sa[CPW > 3 ? 3 : 0]);
      lds[256 + wave * 64 + lane] = (sb[0] + sb[CPW > 1 ? 1 : 0]) + (sb[CPW > 2 ? 2 : 0] + sb[CPW > 3 ? 3 : 0]);
      __syncthreads();
      if (wave == 0 && out < nvec) {
        oa[out] = (lds[lane] + lds[64 + lane]) + (lds[128 + lane] + lds[192 + lane]);
        ob[out] = (lds[256 + lane] + lds[320 + lane]) + (lds[384 + lane] + lds[448 + lane]);
      }
    } else {  // this wave holds s_w
      lds[wave * 64 + lane] = sa[0];
      lds[1024 + wave * 64 + lane] = sb[0];
      __syncthreads();
      if (wave < 2 && out < nvec) {
        const double* q = lds + wave * 1024 + lane;
        double tr[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) tr[r] = (q[r * 64] + q[(r + 4) * 64]) + (q[(r + 8) * 64] + q[(r + 12) * 64]);
        (wave == 0 ? oa : ob)[out] = (tr[0] + tr[1]) + (tr[2] + tr[3]);
      }
    }
    __syncthreads();
  }
}

// Partial dots of the chunk held in LDS (wv and uv, `rows` rows) with
// V_0..V_{nvec-1}: one pass over the basis for both vectors.  Wave q handles groups
// of kDotUnroll basis vectors whose loads are all issued before the shuffle
// reductions; lanes run over rows.
template <bool NT, typename VT>
__device__ void chunk_dots2(const VT* __restrict__ V, int64_t vvs, int64_t x0, int rows, const double* wv,
                            const double* uv, int nvec, double* partw, double* partu, int ld, int chunk) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  for (int i0 = wave * kDotUnroll; i0 < nvec; i0 += kWaves * kDotUnroll) {
    double aw[kDotUnroll], au[kDotUnroll];
#pragma unroll
    for (int u = 0; u < kDotUnroll; ++u) aw[u] = au[u] = 0.0;
#pragma unroll 2
    for (int x = lane; x < rows; x += 64) {
      const double wx = wv[x], ux = uv[x];
      // vectors past nvec repeat the last one (in bounds, results never stored), so
      // every load is issued before the first product
      double vv[kDotUnroll];
#pragma unroll
      for (int u = 0; u < kDotUnroll; ++u) vv[u] = ld_basis<NT>(&V[(int64_t)min(i0 + u, nvec - 1) * vvs + x0 + x]);
#pragma unroll
      for (int u = 0; u < kDotUnroll; ++u) {
        aw[u] = fma(vv[u], wx, aw[u]);
        au[u] = fma(vv[u], ux, au[u]);
      }
    }
#pragma unroll
    for (int u = 0; u < kDotUnroll; ++u) {
      const double sw = wave_sum(aw[u]);
      const double su = wave_sum(au[u]);
      if (lane == 0 && i0 + u < nvec) {
        partw[(int64_t)chunk * ld + i0 + u] = sw;
        partu[(int64_t)chunk * ld + i0 + u] = su;
      }
    }
  }
}

// Givens step for Hessenberg column jc = j-1 of one right-hand side, run by
// block 0 of gm_update: H(:, jc) = h1 + h2 with beta below the diagonal (stored
// unrotated in Hu), rotated by the previous rotations; a new rotation zeroes beta.
// lds: the caller's LDS, kGivensLds doubles.
constexpr int kGivensLds = 3 * (kMaxIt + 2);
template <int B>
__device__ void givens_column(const GmState& S, int col, int j, double beta, const double* h2, double* lds) {
  double* hc = lds;
  double* csl = lds + (kMaxIt + 2);
  double* snl = lds + 2 * (kMaxIt + 2);
  const int tid = threadIdx.x;
  const int jc = j - 1;
  const double* h1 = S.h1 + (int64_t)col * S.ldv;
  double* csg = S.cs + (int64_t)col * S.ldv;
  double* sng = S.sn + (int64_t)col * S.ldv;
  double* Hu = S.Hu + (int64_t)col * S.ldv * S.maxit + (int64_t)jc * S.ldv;
  for (int i = tid; i <= jc; i += kThreads) {
    hc[i] = h1[i] + h2[i];
    Hu[i] = hc[i];  // the unrotated column, for the corrections of later steps
  }
  if (tid == 0) Hu[jc + 1] = beta;
  for (int i = tid; i < jc; i += kThreads) {
    csl[i] = csg[i];
    snl[i] = sng[i];
  }
  __syncthreads();
  if (tid == 0) {
    hc[jc + 1] = beta;
    // the entry carried from rotation i to i + 1 stays in a register; the operands
    // of B rotations are loaded before they are applied (rotation i reads hc[i + 1],
    // which only rotation i + 1 writes).  The same operations whatever B: the fused
    // multiply-adds are written out, so no instantiation is left to contract
    // c a + s b differently.
    double a = hc[0];
    for (int i0 = 0; i0 < jc; i0 += B) {
      double bb[B], ci[B], si[B];
#pragma unroll
      for (int u = 0; u < B; ++u) {
        const int i = min(i0 + u, jc - 1);
        bb[u] = hc[i + 1];
        ci[u] = csl[i];
        si[u] = snl[i];
      }
#pragma unroll
      for (int u = 0; u < B; ++u)
        if (i0 + u < jc) {
          const double sb = si[u] * bb[u], sa = si[u] * a;
          hc[i0 + u] = fma(ci[u], a, sb);
          a = fma(ci[u], bb[u], -sa);
        }
    }
    const double b = beta;
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
    // a column retires once its estimate meets the threshold, at maxit, on a breakdown,
    // or when the estimate is not finite (iterating on NaN is useless; the host's FP64
    // true residual then reports the column as not converged)
    if (res <= S.tolb[col] || !isfinite(res) || j >= S.maxit || !(beta > 0.0)) {
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

// Block-Jacobi staging of the Arnoldi update: up to kGroupBlocks consecutive blocks of
// one class (one size, adjacent slot lists), kStageSlots slots at most.
constexpr int kGroupBlocks = 8, kStageSlots = 1024;
// LDS of the single-column update: block 0's Givens step, or the other blocks'
// staged slots and the apply's partial sums
constexpr int kUpdLds = kStageSlots + kGroupBlocks * 256 > kGivensLds ? kStageSlots + kGroupBlocks * 256 : kGivensLds;
struct BlockGroup {
  int o0, sb, bc, nb;  // first slot-list entry, block size, class, blocks
};
// The group starting at block b of a run ending before bend; the class entries of
// the following blocks are loaded together.
__device__ __forceinline__ BlockGroup block_group(const DevPlan& P, int b, int bend) {
  BlockGroup g;
  g.o0 = P.blk_off[b];
  g.sb = P.blk_off[b + 1] - g.o0;
  g.bc = P.blk_cls[b];
  int cl[kGroupBlocks];
#pragma unroll
  for (int u = 1; u < kGroupBlocks; ++u) cl[u] = P.blk_cls[min(b + u, bend - 1)];
  g.nb = 1;
#pragma unroll
  for (int u = 1; u < kGroupBlocks; ++u)
    if (g.nb == u && b + u < bend && cl[u] == g.bc && (u + 1) * g.sb <= kStageSlots) g.nb = u + 1;
  return g;
}

// Step j's first kernel (see the file header; m = j - 1).  Step 0: z = M^{-1} u_0.
template <typename OpT, bool PRE, typename VT>
__global__ __launch_bounds__(256) void k_gm_update(DevPlan P, GmState S, int par, int use_precond, int transpose) {
  using Acc = typename AccOf<OpT>::type;
  constexpr int kGroup = kGroupBlocks;
  static_assert(kStageSlots >= 8 * kMaxN, "one block must fit the staging area");
  static_assert((kStageSlots + kGroup * 256) * sizeof(Acc) <= kUpdLds * sizeof(double), "LDS union");
  // block 0 uses wsp for the Givens step and then for the h' sums; the other blocks
  // (which never take the Givens step when the grid has more than one block) stage
  // their slots in it
  __shared__ double wsp[kUpdLds];
  __shared__ double red[2 * kWaves];
  __shared__ double ds[kMaxIt + 1];  // d_0..d_{m-1}, then alpha
  __shared__ double cs2[kMaxIt + 1]; // c_0..c_{m-1}, then nu
  double (*hsum)[64] = reinterpret_cast<double (*)[64]>(wsp);
  Acc* xs = reinterpret_cast<Acc*>(wsp);
  Acc* bpart = xs + kStageSlots;
  const int col = blockIdx.y, tid = threadIdx.x;
  // The slot blocks' run of block-Jacobi blocks and its first group: their table loads
  // depend on nothing, so they are issued before anything waits (the column's
  // activity, the step index); the tail reuses them.
  const bool slot_block = use_precond && (gridDim.x == 1 || blockIdx.x > 0);
  int wb = gridDim.x > 1 ? blockIdx.x - 1 : 0;
  const int nwb = gridDim.x > 1 ? gridDim.x - 1 : 1;
  if (nwb % 8 == 0) wb = xcd_block(wb, nwb);
  const int per = (P.nblk + nwb - 1) / nwb;
  const int b0 = wb * per, bend = min(P.nblk, (wb + 1) * per);
  BlockGroup g0 = {0, 0, 0, 0};
  if (slot_block && b0 < bend) g0 = block_group(P, b0, bend);
  if (!S.active[col]) return;
  const int j = S.jdev[par];
  const bool nt = S.stream > 0 || (S.stream < 0 && stream_basis(j > 1 ? j : 1, S.vvs));
  const int64_t k = P.k;
  double* zc = S.z + (int64_t)col * k;
  const VT* Vc = basis<VT>(S) + (int64_t)col * k;
  // The first group's inverse, and, when the group holds at most one slot per thread
  // and 1 <= m <= kPre, the thread's slot with its basis entries V_0..V_{m-1}, u_m and
  // w: loaded before the Gram-Schmidt sums are reduced (none of them needs a sum), so
  // the round trips overlap.
  constexpr int kPre = 32;
  double pv[kPre];
  double pvm = 0.0, pwc = 0.0;
  int64_t px = -1;
  const int mp = j - 1;
  int64_t mb0 = 0;
  if (slot_block && b0 < bend) mb0 = P.bcls_off[g0.bc];
  // uniform over the block
  const bool pre = slot_block && gridDim.x > 1 && b0 < bend && g0.nb * g0.sb <= kThreads && mp >= 1 &&
                   mp <= kPre && mp <= S.maxit;
  if (pre && tid < g0.nb * g0.sb) {
    px = P.blk_slots[g0.o0 + tid];
    auto load = [&](auto nt_) {
#pragma unroll
      for (int u = 0; u < kPre; ++u)
        pv[u] = ld_basis<kNT<decltype(nt_)>>(&Vc[(int64_t)min(u, mp - 1) * S.vvs + px]);
    };
    if (nt)
      load(std::true_type{});
    else
      load(std::false_type{});
    pvm = Vc[(int64_t)mp * S.vvs + px];
    pwc = S.w[(int64_t)col * k + px];
  }
  int m = -1;
  double inv = 0.0, e = 0.0;
  if (j > 0) {
    m = j - 1;
    if (m > S.maxit) return;
    if (PRE) {  // sums reduced once per column by k_gm_reduce
      for (int i = tid; i <= m; i += kThreads) {
        ds[i] = S.dw[(int64_t)col * S.ldv + i];
        cs2[i] = S.h2[(int64_t)col * S.ldv + i];
      }
    } else {
      reduce_partials2<kWaves>(S.part1 + (int64_t)col * S.ldv * S.nch, S.part2 + (int64_t)col * S.ldv * S.nch,
                               m + 1, S.nch, S.ldv, ds, cs2, wsp);
    }
    __syncthreads();
    if (tid < 64) {
      double cc = 0.0, cd = 0.0;
      for (int i = tid; i < m; i += 64) {
        cc = fma(cs2[i], cs2[i], cc);
        cd = fma(cs2[i], ds[i], cd);
      }
      cc = wave_sum(cc);
      cd = wave_sum(cd);
      if (tid == 0) {
        red[0] = sqrt(fmax(cs2[m] - cc, 0.0));  // rho
        red[1] = ds[m] - cd;                     // rho * e
      }
    }
    __syncthreads();
    const double rho = red[0];
    inv = rho > 0.0 ? 1.0 / rho : 0.0;
    e = red[1] * inv;
    if (blockIdx.x == 0) {
      if (m == 0) {
        if (tid == 0) {
          S.tolb[col] = S.tolv[0] * (S.bref2 ? sqrt(S.bref2[col]) : rho);
          S.g[(int64_t)col * S.ldv] = rho;
          S.res[col] = rho;
          if (!(rho > 0.0)) {
            S.active[col] = 0;
            S.iters[col] = 0;
          }
        }
      } else {
        givens_column<4>(S, col, m, rho, cs2, wsp);
      }
      // h'_m = ([d; e] - H c) / rho with the unrotated columns 0..m-1 (after the
      // Givens step has read h'_{m-1}): lanes take rows l, the waves split the
      // columns i, and the four partial sums are added in a fixed order
      __syncthreads();
      const double* Hu = S.Hu + (int64_t)col * S.ldv * S.maxit;
      double* hp = S.h1 + (int64_t)col * S.ldv;
      const int wave = tid >> 6, lane = tid & 63;
      for (int l0 = 0; l0 <= m; l0 += 64) {
        const int l = l0 + lane;
        double hc = 0.0;
        if (l <= m) {
          // this wave's columns i = ib, ib + 4, ...: clamped loads issued eight at a time
          const int ib = max(l - 1, 0) + ((wave - max(l - 1, 0)) & 3);
          for (int i0 = ib; i0 < m; i0 += 8 * kWaves) {
            double hv[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) hv[u] = Hu[(int64_t)min(i0 + u * kWaves, m - 1) * S.ldv + l];
#pragma unroll
            for (int u = 0; u < 8; ++u)
              if (i0 + u * kWaves < m) hc = fma(hv[u], cs2[i0 + u * kWaves], hc);
          }
        }
        hsum[wave][lane] = hc;
        __syncthreads();
        if (wave == 0 && l <= m)
          hp[l] = ((l < m ? ds[l] : e) - ((hsum[0][lane] + hsum[1][lane]) + (hsum[2][lane] + hsum[3][lane]))) * inv;
        __syncthreads();
      }
    }
    if (m >= S.maxit) return;
  }
  // q_m into V_m and u_{m+1} into V_{m+1} at one slot; returns u_{m+1} (step 0: u_0)
  const double* wc = S.w + (int64_t)col * k;
  VT* vm = basis<VT>(S) + (int64_t)max(m, 0) * S.vvs + (int64_t)col * k;
  VT* vn = basis<VT>(S) + (int64_t)(m + 1) * S.vvs + (int64_t)col * k;
  // the products from basis vector i_begin on, then q_m and u_{m+1} at slot x
  auto finish = [&](auto nt_, int64_t x, int i_begin, double sc, double sw) {
    // batches of 32: every load of a batch is issued before its products, which run in
    // order (same bits as a plain loop); the last, partial batch clamps and masks
    for (int i0 = i_begin; i0 < m; i0 += 32) {
      double v_[32];
      if (i0 + 32 <= m) {
#pragma unroll
        for (int u = 0; u < 32; ++u) {
          const int i = i0 + u;
          v_[u] = ld_basis<kNT<decltype(nt_)>>(&Vc[(int64_t)i * S.vvs + x]);
        }
#pragma unroll
        for (int u = 0; u < 32; ++u) {
          const int i = i0 + u;
          const double v = v_[u];
          sc = fma(-cs2[i], v, sc);
          sw = fma(-ds[i], v, sw);
        }
      } else {
#pragma unroll
        for (int u = 0; u < 32; ++u) {
          const int i = min(i0 + u, m - 1);
          v_[u] = ld_basis<kNT<decltype(nt_)>>(&Vc[(int64_t)i * S.vvs + x]);
        }
#pragma unroll
        for (int u = 0; u < 32; ++u) {
          const int i = i0 + u;
          if (i < m) {
            const double v = v_[u];
            sc = fma(-cs2[i], v, sc);
            sw = fma(-ds[i], v, sw);
          }
        }
      }
    }
    const double q = sc * inv;
    const double un = fma(-e, q, sw) * inv;
    vm[x] = (VT)q;
    vn[x] = (VT)un;
    return un;
  };
  auto update = [&](auto nt_, int64_t x) -> double {
    return m < 0 ? (double)vn[x] : finish(nt_, x, 0, (double)vm[x], wc[x]);
  };
  // the same from the prefetched entries (this thread's slot px, 1 <= m <= kPre): the
  // products in order, then q_m and u_{m+1} as finish() forms them
  auto update_pre = [&]() {
    double sc = pvm, sw = pwc;
#pragma unroll
    for (int u = 0; u < kPre; ++u)
      if (u < m) {
        sc = fma(-cs2[u], pv[u], sc);
        sw = fma(-ds[u], pv[u], sw);
      }
    const double q = sc * inv;
    const double un = fma(-e, q, sw) * inv;
    vm[px] = (VT)q;
    vn[px] = (VT)un;
    return un;
  };
  // the same at two slots, the loads of both in flight together (x1 is stored only
  // if st1; otherwise it must still be a valid slot)
  auto update2 = [&](auto nt_, int64_t x0, int64_t x1, bool st1, double& r0, double& r1) {
    if (m < 0) {
      r0 = vn[x0];
      r1 = vn[x1];
      return;
    }
    double sc0 = vm[x0], sw0 = wc[x0], sc1 = vm[x1], sw1 = wc[x1];
    // batches of 8: every load of a batch is issued before its products, which run in
    // order (same bits as a plain loop); the last, partial batch clamps and masks
    for (int i0 = 0; i0 < m; i0 += 8) {
      double v0_[8];
      double v1_[8];
      if (i0 + 8 <= m) {
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int i = i0 + u;
          v0_[u] = ld_basis<kNT<decltype(nt_)>>(&Vc[(int64_t)i * S.vvs + x0]);
          v1_[u] = ld_basis<kNT<decltype(nt_)>>(&Vc[(int64_t)i * S.vvs + x1]);
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int i = i0 + u;
          const double v0 = v0_[u];
          const double v1 = v1_[u];
          sc0 = fma(-cs2[i], v0, sc0);
          sw0 = fma(-ds[i], v0, sw0);
          sc1 = fma(-cs2[i], v1, sc1);
          sw1 = fma(-ds[i], v1, sw1);
        }
      } else {
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int i = min(i0 + u, m - 1);
          v0_[u] = ld_basis<kNT<decltype(nt_)>>(&Vc[(int64_t)i * S.vvs + x0]);
          v1_[u] = ld_basis<kNT<decltype(nt_)>>(&Vc[(int64_t)i * S.vvs + x1]);
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int i = i0 + u;
          if (i < m) {
            const double v0 = v0_[u];
            const double v1 = v1_[u];
            sc0 = fma(-cs2[i], v0, sc0);
            sw0 = fma(-ds[i], v0, sw0);
            sc1 = fma(-cs2[i], v1, sc1);
            sw1 = fma(-ds[i], v1, sw1);
          }
        }
      }
    }
    const double q0 = sc0 * inv, q1 = sc1 * inv;
    r0 = fma(-e, q0, sw0) * inv;
    r1 = fma(-e, q1, sw1) * inv;
    vm[x0] = (VT)q0;
    vn[x0] = (VT)r0;
    if (st1) {
      vm[x1] = (VT)q1;
      vn[x1] = (VT)r1;
    }
  };
  // block 0 takes the Givens step alone; blocks 1.. share the slots
  if (blockIdx.x == 0 && gridDim.x > 1) return;
  // the rest once per launch, with the basis loads compiled for the streaming choice
  auto tail = [&](auto nt_) {
    if (!use_precond) {
      const int wr = gridDim.x > 1 ? blockIdx.x - 1 : 0;  // row blocks in launch order
      for (int64_t x = (int64_t)wr * kThreads + tid; x < k; x += (int64_t)nwb * kThreads) zc[x] = update(nt_, x);
      return;
    }
    // a contiguous run of the (class-ordered) blocks per workgroup, runs of one XCD
    // adjacent; consecutive blocks of one class are staged together and share every
    // read of their inverse (the apply gives each block the same bits as alone)
    for (int b = b0; b < bend;) {
      const BlockGroup g = b == b0 ? g0 : block_group(P, b, bend);
      const int o0 = g.o0, sb = g.sb, bc = g.bc, nb = g.nb;
      const int tot = nb * sb;
      __syncthreads();  // the previous group's apply has read xs (block 0: wsp is free)
      if (pre && b == b0) {
        if (tid < tot) xs[tid] = (Acc)update_pre();
      } else
      // two slots per thread while there are two, then one
      for (int i0 = tid; i0 < tot; i0 += 2 * kThreads) {
        const int i1 = i0 + kThreads;
        if (i1 < tot) {
          double r0, r1;
          update2(nt_, P.blk_slots[o0 + i0], P.blk_slots[o0 + i1], true, r0, r1);
          xs[i0] = (Acc)r0;
          xs[i1] = (Acc)r1;
        } else {
          xs[i0] = (Acc)update(nt_, P.blk_slots[o0 + i0]);
        }
      }
      __syncthreads();
      const OpT* Mp = minv_op<OpT>(P, transpose != 0) + (b == b0 ? mb0 : P.bcls_off[bc]);
      auto put = [&](int v, int r, Acc val) {
        if (v < nb) zc[P.blk_slots[o0 + v * sb + r]] = (double)val;
      };
      if (nb == 1)
        block_jacobi_apply<1>(Mp, xs, sb, sb, bpart, put);
      else if (nb <= 4)
        block_jacobi_apply<4>(Mp, xs, sb, sb, bpart, put);
      else
        block_jacobi_apply<kGroup>(Mp, xs, sb, sb, bpart, put);
      b += nb;
    }
  };
  if (nt)
    tail(std::true_type{});
  else
    tail(std::false_type{});
}

// Step j's first kernel for NC columns at once, with pre-reduced dot sums (large
// grids, several columns): as k_gm_update, but every block-Jacobi inverse is read
// once for the NC columns.  Same arithmetic per column, so the same bits.
template <typename OpT, int NC, typename VT>
__global__ __launch_bounds__(256) void k_gm_update_n(DevPlan P, GmState S, int par, int use_precond, int transpose) {
  using Acc = typename AccOf<OpT>::type;
  constexpr int kStage = 128;
  // block 0's Givens steps use the front of `area`; after them (behind barriers) it
  // holds the columns' coefficients cst (c and d, m <= kStage) and the staged
  // block-Jacobi inputs xs with their partial sums bpart
  constexpr int kXs = NC * 8 * kMaxN;
  constexpr int kStaged = (2 * kXs * (int)sizeof(Acc) + 7) / 8 + NC * 2 * kStage;
  __shared__ double area[kStaged > kGivensLds ? kStaged : kGivensLds];
  double* gwork = area;
  Acc (*xs)[8 * kMaxN] = reinterpret_cast<Acc (*)[8 * kMaxN]>(area);
  Acc* bpart = reinterpret_cast<Acc*>(area) + kXs;
  double (*cst)[2][kStage] = reinterpret_cast<double (*)[2][kStage]>(area + (2 * kXs * (int)sizeof(Acc) + 7) / 8);
  __shared__ double scal[NC][2];  // rho, e
  __shared__ double hsum[kWaves][64];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int64_t k = P.k;
  const int nrhs = (int)(S.vvs / k);
  const int c0 = blockIdx.y * NC;
  bool on[NC];
  bool any = false;
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    on[c] = c0 + c < nrhs && S.active[c0 + c];
    any = any || on[c];
  }
  if (!any) return;
  const int j = S.jdev[par];
  const bool nt = S.stream > 0 || (S.stream < 0 && stream_basis(j > 1 ? j : 1, S.vvs));
  const int m = j - 1;
  if (m > S.maxit) return;
  if (j > 0) {
    // rho and e per column from the pre-reduced sums: wave w takes columns w, w+4, ...
    for (int c = wave; c < NC; c += kWaves) {
      if (!on[c]) continue;
      const double* cu = S.h2 + (int64_t)(c0 + c) * S.ldv;
      const double* dw = S.dw + (int64_t)(c0 + c) * S.ldv;
      double cc = 0.0, cd = 0.0;
      for (int i = lane; i < m; i += 64) {
        cc = fma(cu[i], cu[i], cc);
        cd = fma(cu[i], dw[i], cd);
      }
      cc = wave_sum(cc);
      cd = wave_sum(cd);
      if (lane == 0) {
        const double rho = sqrt(fmax(cu[m] - cc, 0.0));
        scal[c][0] = rho;
        scal[c][1] = (dw[m] - cd) * (rho > 0.0 ? 1.0 / rho : 0.0);
      }
    }
    __syncthreads();
    if (blockIdx.x == 0) {
      for (int c = 0; c < NC; ++c) {
        if (!on[c]) continue;
        const int col = c0 + c;
        const double rho = scal[c][0], e = scal[c][1];
        const double inv = rho > 0.0 ? 1.0 / rho : 0.0;
        const double* cu = S.h2 + (int64_t)col * S.ldv;
        const double* dw = S.dw + (int64_t)col * S.ldv;
        if (m == 0) {
          if (tid == 0) {
            S.tolb[col] = S.tolv[0] * (S.bref2 ? sqrt(S.bref2[col]) : rho);
            S.g[(int64_t)col * S.ldv] = rho;
            S.res[col] = rho;
            if (!(rho > 0.0)) {
              S.active[col] = 0;
              S.iters[col] = 0;
            }
          }
        } else {
          givens_column<1>(S, col, m, rho, cu, gwork);
        }
        __syncthreads();
        const double* Hu = S.Hu + (int64_t)col * S.ldv * S.maxit;
        double* hp = S.h1 + (int64_t)col * S.ldv;
        for (int l0 = 0; l0 <= m; l0 += 64) {
          const int l = l0 + lane;
          double hc = 0.0;
          if (l <= m) {
            // this wave's columns i = ib, ib + 4, ...: clamped loads issued eight at a time
            const int ib = max(l - 1, 0) + ((wave - max(l - 1, 0)) & 3);
            for (int i0 = ib; i0 < m; i0 += 8 * kWaves) {
              double hv[8];
#pragma unroll
              for (int u = 0; u < 8; ++u) hv[u] = Hu[(int64_t)min(i0 + u * kWaves, m - 1) * S.ldv + l];
#pragma unroll
              for (int u = 0; u < 8; ++u)
                if (i0 + u * kWaves < m) hc = fma(hv[u], cu[i0 + u * kWaves], hc);
            }
          }
          hsum[wave][lane] = hc;
          __syncthreads();
          if (wave == 0 && l <= m)
            hp[l] = ((l < m ? dw[l] : e) - ((hsum[0][lane] + hsum[1][lane]) + (hsum[2][lane] + hsum[3][lane]))) * inv;
          __syncthreads();
        }
      }
    }
    if (m >= S.maxit) return;
  }
  // q_m and u_{m+1} of column c at one slot (step 0: u_0)
  // the columns' coefficients in LDS when they fit (the common case), else read
  // from memory in the loop; the same products in the same order either way
  const bool staged = m >= 0 && m <= kStage;
  if (staged) {
    for (int t = tid; t < NC * m; t += kThreads) {
      const int c = t / max(m, 1), i = t - c * m;
      if (on[c]) {
        cst[c][0][i] = S.h2[(int64_t)(c0 + c) * S.ldv + i];
        cst[c][1][i] = S.dw[(int64_t)(c0 + c) * S.ldv + i];
      }
    }
    __syncthreads();
  }
  auto update = [&](auto nt_, int c, int64_t x) {
    const int col = c0 + c;
    const VT* Vc = basis<VT>(S) + (int64_t)col * k;
    VT* vn = basis<VT>(S) + (int64_t)(m + 1) * S.vvs + (int64_t)col * k;
    if (m < 0) return (double)vn[x];
    VT* vm = basis<VT>(S) + (int64_t)m * S.vvs + (int64_t)col * k;
    const double rho = scal[c][0], e = scal[c][1];
    const double inv = rho > 0.0 ? 1.0 / rho : 0.0;
    double sc = vm[x], sw = S.w[(int64_t)col * k + x];
    if (staged) {
      // clamped loads issued together, then the products in order (same bits as a plain loop)
      for (int i0 = 0; i0 < m; i0 += 16) {
        double v_[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) {
          const int i = min(i0 + u, m - 1);
          v_[u] = ld_basis<kNT<decltype(nt_)>>(&Vc[(int64_t)i * S.vvs + x]);
        }
#pragma unroll
        for (int u = 0; u < 16; ++u) {
          const int i = i0 + u;
          if (i < m) {
            const double v = v_[u];
            sc = fma(-cst[c][0][i], v, sc);
            sw = fma(-cst[c][1][i], v, sw);
          }
        }
      }
    } else {
      const double* cu = S.h2 + (int64_t)col * S.ldv;
      const double* dw = S.dw + (int64_t)col * S.ldv;
      // clamped loads issued together, then the products in order (same bits as a plain loop)
      for (int i0 = 0; i0 < m; i0 += 16) {
        double v_[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) {
          const int i = min(i0 + u, m - 1);
          v_[u] = ld_basis<kNT<decltype(nt_)>>(&Vc[(int64_t)i * S.vvs + x]);
        }
#pragma unroll
        for (int u = 0; u < 16; ++u) {
          const int i = i0 + u;
          if (i < m) {
            const double v = v_[u];
            sc = fma(-cu[i], v, sc);
            sw = fma(-dw[i], v, sw);
          }
        }
      }
    }
    const double q = sc * inv;
    const double un = fma(-e, q, sw) * inv;
    vm[x] = (VT)q;
    vn[x] = (VT)un;
    return un;
  };
  // the same for column ca at slot xa and column cb at slot xb, the loads of both in
  // flight together (both columns active, m >= 0)
  auto update2 = [&](auto nt_, int ca, int64_t xa, int cb, int64_t xb, double& ra, double& rb) {
    const VT* Va = basis<VT>(S) + (int64_t)(c0 + ca) * k;
    const VT* Vb = basis<VT>(S) + (int64_t)(c0 + cb) * k;
    VT* vma = basis<VT>(S) + (int64_t)m * S.vvs + (int64_t)(c0 + ca) * k;
    VT* vmb = basis<VT>(S) + (int64_t)m * S.vvs + (int64_t)(c0 + cb) * k;
    double sca = vma[xa], swa = S.w[(int64_t)(c0 + ca) * k + xa];
    double scb = vmb[xb], swb = S.w[(int64_t)(c0 + cb) * k + xb];
    if (staged) {
      // clamped loads issued together, then the products in order (same bits as a plain loop)
      for (int i0 = 0; i0 < m; i0 += 8) {
        double va_[8];
        double vb_[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int i = min(i0 + u, m - 1);
          va_[u] = ld_basis<kNT<decltype(nt_)>>(&Va[(int64_t)i * S.vvs + xa]);
          vb_[u] = ld_basis<kNT<decltype(nt_)>>(&Vb[(int64_t)i * S.vvs + xb]);
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int i = i0 + u;
          if (i < m) {
            const double va = va_[u];
            const double vb = vb_[u];
            sca = fma(-cst[ca][0][i], va, sca);
            swa = fma(-cst[ca][1][i], va, swa);
            scb = fma(-cst[cb][0][i], vb, scb);
            swb = fma(-cst[cb][1][i], vb, swb);
          }
        }
      }
    } else {
      const double* cua = S.h2 + (int64_t)(c0 + ca) * S.ldv;
      const double* dwa = S.dw + (int64_t)(c0 + ca) * S.ldv;
      const double* cub = S.h2 + (int64_t)(c0 + cb) * S.ldv;
      const double* dwb = S.dw + (int64_t)(c0 + cb) * S.ldv;
      // clamped loads issued together, then the products in order (same bits as a plain loop)
      for (int i0 = 0; i0 < m; i0 += 8) {
        double va_[8];
        double vb_[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int i = min(i0 + u, m - 1);
          va_[u] = ld_basis<kNT<decltype(nt_)>>(&Va[(int64_t)i * S.vvs + xa]);
          vb_[u] = ld_basis<kNT<decltype(nt_)>>(&Vb[(int64_t)i * S.vvs + xb]);
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int i = i0 + u;
          if (i < m) {
            const double va = va_[u];
            const double vb = vb_[u];
            sca = fma(-cua[i], va, sca);
            swa = fma(-dwa[i], va, swa);
            scb = fma(-cub[i], vb, scb);
            swb = fma(-dwb[i], vb, swb);
          }
        }
      }
    }
    const double inva = scal[ca][0] > 0.0 ? 1.0 / scal[ca][0] : 0.0;
    const double invb = scal[cb][0] > 0.0 ? 1.0 / scal[cb][0] : 0.0;
    const double qa = sca * inva, qb = scb * invb;
    ra = fma(-scal[ca][1], qa, swa) * inva;
    rb = fma(-scal[cb][1], qb, swb) * invb;
    vma[xa] = (VT)qa;
    basis<VT>(S)[(int64_t)(m + 1) * S.vvs + (int64_t)(c0 + ca) * k + xa] = (VT)ra;
    vmb[xb] = (VT)qb;
    basis<VT>(S)[(int64_t)(m + 1) * S.vvs + (int64_t)(c0 + cb) * k + xb] = (VT)rb;
  };
  // block 0 takes the Givens steps alone; blocks 1.. share the slots
  if (blockIdx.x == 0 && gridDim.x > 1) return;
  // the rest once per launch, with the basis loads compiled for the streaming choice
  auto tail = [&](auto nt_) {
    int wb = gridDim.x > 1 ? blockIdx.x - 1 : 0;
    const int nwb = gridDim.x > 1 ? gridDim.x - 1 : 1;
    if (!use_precond) {
      for (int64_t x = (int64_t)wb * kThreads + tid; x < k; x += (int64_t)nwb * kThreads)
  #pragma unroll
        for (int c = 0; c < NC; ++c)
          if (on[c]) S.z[(int64_t)(c0 + c) * k + x] = update(nt_, c, x);
      return;
    }
    // a contiguous run of the (class-ordered) blocks per workgroup, runs of one XCD adjacent
    if (nwb % 8 == 0) wb = xcd_block(wb, nwb);
    const int per = (P.nblk + nwb - 1) / nwb;
    for (int b = wb * per; b < min(P.nblk, (wb + 1) * per); ++b) {
      const int o = P.blk_off[b], sb = P.blk_off[b + 1] - o;
      const int bc = P.blk_cls[b];
      __syncthreads();
      // the NC * sb (column, slot) items, two per thread
      const int tot = NC * sb;
      for (int u = tid; u < tot; u += 2 * kThreads) {
        const int ca = u / sb, ia = u - ca * sb;
        const int u1 = u + kThreads;
        const bool in1 = u1 < tot;
        const int cb = in1 ? u1 / sb : ca, ib = in1 ? u1 - cb * sb : ia;
        const bool pa = on[ca], pb = in1 && on[cb];
        if (pa && pb && m >= 0) {
          double ra, rb;
          update2(nt_, ca, P.blk_slots[o + ia], cb, P.blk_slots[o + ib], ra, rb);
          xs[ca][ia] = (Acc)ra;
          xs[cb][ib] = (Acc)rb;
        } else {
          xs[ca][ia] = pa ? (Acc)update(nt_, ca, P.blk_slots[o + ia]) : Acc(0);
          if (in1) xs[cb][ib] = pb ? (Acc)update(nt_, cb, P.blk_slots[o + ib]) : Acc(0);
        }
      }
      __syncthreads();
      const OpT* Mp = minv_op<OpT>(P, transpose != 0) + P.bcls_off[bc];
      block_jacobi_apply<NC>(Mp, &xs[0][0], 8 * kMaxN, sb, bpart, [&](int c, int r, Acc v) {
        if (on[c]) S.z[(int64_t)(c0 + c) * k + P.blk_slots[o + r]] = (double)v;
      });
    }
  };
  if (nt)
    tail(std::true_type{});
  else
    tail(std::false_type{});
}

// Step j's last kernel: w = t - (Z c2 + {S Z c2 | S^T Z c2}) on this block's rows (or
// w = t), then the partial dots of V_0..V_j with w and with u_j = V_j; the next
// step's index.
template <typename VT>
__global__ __launch_bounds__(256) void k_gm_dots(DevPlan P, GmState S, int par, int defl, int transpose) {
  __shared__ double wv[kRowsMax];
  __shared__ double uv[kRowsMax];
  const int col = blockIdx.y, chunk = blockIdx.x, tid = threadIdx.x;
  const int64_t k = P.k, x0 = (int64_t)chunk * S.rows;
  const int rows = (int)min((int64_t)S.rows, k - x0);
  // with one row per thread, the row's t and its deflation table entry need nothing
  // of this step's counters: their loads go out first
  const int64_t xt = x0 + min(tid, rows - 1);
  const double tv0 = S.t[(int64_t)col * k + xt];
  int4 ta = {0, 0, 0, 0}, tb = {0, 0, 0, 0};
  if (defl && rows <= kThreads) deflation_table(P, xt, transpose != 0, ta, tb);
  const int j = S.jdev[par];
  // the step's last kernel sets the next step's index in the other slot (whatever the
  // columns' activity, so steps keep counting)
  if (blockIdx.x == 0 && blockIdx.y == 0 && tid == 0) S.jdev[par ^ 1] = j + 1;
  // the step that completes a chunk reports the columns' progress to the host (the
  // flags were set by this step's first kernel)
  if (S.pub_every > 0 && blockIdx.x == 0 && blockIdx.y == 0 && (j + 1) % S.pub_every == 0) {
    const int done = (j + 1) / S.pub_every, slot = (done - 1) & 1;
    for (int i = tid; i < (int)gridDim.y; i += kThreads) {
      S.hflag[slot * S.pub_stride + i] = S.active[i];
      S.hratio[slot * S.pub_stride + i] = S.tolb[i] > 0.0 ? S.res[i] / S.tolb[i] : 0.0;
    }
    __threadfence_system();
    __syncthreads();
    if (tid == 0) S.hseq[0] = done;
  }
  if (!S.active[col] || j > S.maxit) return;
  const double* tc = S.t + (int64_t)col * k;
  double* wc = S.w + (int64_t)col * k;
  const VT* Vc = basis<VT>(S) + (int64_t)col * k;
  const VT* uj = Vc + (int64_t)j * S.vvs;
  const double* cc = S.c2 + (int64_t)col * P.d;
  const bool nt = S.stream > 0 || (S.stream < 0 && stream_basis(j + 1, S.vvs));
  double* p1 = S.part1 + (int64_t)col * S.ldv * S.nch;
  double* p2 = S.part2 + (int64_t)col * S.ldv * S.nch;
  // At most 32 basis vectors and 256 rows (one group of kDotUnroll vectors per wave,
  // four rows per lane): the wave's basis entries are loaded before w is formed (they
  // need no w), so their round trip overlaps the deflation's; the products then run
  // in chunk_dots2's order.
  const int nvec = j + 1, wave = tid >> 6, lane = tid & 63;
  if (nvec <= kDotUnroll * kWaves && rows <= 4 * 64) {
    const int i0 = wave * kDotUnroll;
    double vv[4][kDotUnroll];
    if (i0 < nvec) {
      auto load = [&](auto nt_) {
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
          for (int u = 0; u < kDotUnroll; ++u)
            vv[r][u] = ld_basis<kNT<decltype(nt_)>>(
                &Vc[(int64_t)min(i0 + u, nvec - 1) * S.vvs + x0 + min(lane + 64 * r, rows - 1)]);
      };
      if (nt)
        load(std::true_type{});
      else
        load(std::false_type{});
    }
    if (tid < rows) {
      double v = tv0;
      if (defl) v -= deflation_tb(P, cc, xt, transpose != 0, ta, tb);
      wc[xt] = v;
      wv[tid] = v;
      uv[tid] = uj[xt];
    }
    __syncthreads();
    if (i0 >= nvec) return;
    double aw[kDotUnroll], au[kDotUnroll];
#pragma unroll
    for (int u = 0; u < kDotUnroll; ++u) aw[u] = au[u] = 0.0;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int x = lane + 64 * r;
      if (x < rows) {
        const double wx = wv[x], ux = uv[x];
#pragma unroll
        for (int u = 0; u < kDotUnroll; ++u) {
          aw[u] = fma(vv[r][u], wx, aw[u]);
          au[u] = fma(vv[r][u], ux, au[u]);
        }
      }
    }
#pragma unroll
    for (int u = 0; u < kDotUnroll; ++u) {
      const double sw = wave_sum(aw[u]);
      const double su = wave_sum(au[u]);
      if (lane == 0 && i0 + u < nvec) {
        p1[(int64_t)chunk * S.ldv + i0 + u] = sw;
        p2[(int64_t)chunk * S.ldv + i0 + u] = su;
      }
    }
    return;
  }
  for (int q = tid; q < rows; q += kThreads) {
    const int64_t slot = x0 + q;
    double v = tc[slot];
    if (defl) v -= deflation(P, cc, slot, transpose != 0);
    wc[slot] = v;
    wv[q] = v;
    uv[q] = uj[slot];
  }
  __syncthreads();
  if (nt)
    chunk_dots2<true>(Vc, S.vvs, x0, rows, wv, uv, nvec, p1, p2, S.ldv, chunk);
  else
    chunk_dots2<false>(Vc, S.vvs, x0, rows, wv, uv, nvec, p1, p2, S.ldv, chunk);
}

// Pre-reduction after gm_dots: the dots with w into dw and with u_j into h2, summed
// exactly as gm_update sums them itself (chunk class c mod 16, each class in
// increasing c, then the same tree).  A block takes 16 vectors: its lanes are
// 16 vectors x 4 classes and its 4 waves the class quarters, so every wave load reads
// four 128-byte rows and the blocks of a column share the work.
constexpr int kReduceVecs = 16;
__global__ __launch_bounds__(256) void k_gm_reduce(GmState S, int par) {
  __shared__ double cs[2][16][kReduceVecs];
  const int col = blockIdx.y;
  const int j = S.jdev[par];
  if (!S.active[col] || j > S.maxit) return;
  const int nvec = j + 1, v0 = blockIdx.x * kReduceVecs;
  if (v0 >= nvec) return;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int vl = lane & 15, q = wave * 4 + (lane >> 4);  // vector v0 + vl, class q
  const int v = min(v0 + vl, nvec - 1);
  const int nch = S.nch, ld = S.ldv;
  const double* pa = S.part1 + (int64_t)col * ld * nch;
  const double* pb = S.part2 + (int64_t)col * ld * nch;
  double sa = 0.0, sb = 0.0;
  for (int c0 = q; c0 < nch; c0 += 16 * 16) {
    // sixteen chunks of the class per batch (past nch: the last chunk, not added)
    double la[16], lb[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int64_t at = (int64_t)min(c0 + 16 * u, nch - 1) * ld + v;
      la[u] = pa[at];
      lb[u] = pb[at];
    }
#pragma unroll
    for (int u = 0; u < 16; ++u)
      if (c0 + 16 * u < nch) {
        sa += la[u];
        sb += lb[u];
      }
  }
  cs[0][q][vl] = sa;
  cs[1][q][vl] = sb;
  __syncthreads();
  if (threadIdx.x < 2 * kReduceVecs) {
    const int a = threadIdx.x / kReduceVecs, vv = threadIdx.x - a * kReduceVecs;
    if (v0 + vv < nvec) {
      double tr[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) tr[r] = (cs[a][r][vv] + cs[a][r + 4][vv]) + (cs[a][r + 8][vv] + cs[a][r + 12][vv]);
      (a == 0 ? S.dw : S.h2)[(int64_t)col * ld + v0 + vv] = (tr[0] + tr[1]) + (tr[2] + tr[3]);
    }
  }
}

// Start of a solve: u_0 = w (the initial residual) into V_0; all columns active;
// j = 0 and the tolerance.
template <typename VT>
__global__ __launch_bounds__(256) void k_gm_start(DevPlan P, GmState S, double tol) {
  const int col = blockIdx.y, chunk = blockIdx.x, tid = threadIdx.x;
  const int64_t k = P.k, x0 = (int64_t)chunk * S.rows;
  const int rows = (int)min((int64_t)S.rows, k - x0);
  const double* wc = S.w + (int64_t)col * k;
  VT* v0 = basis<VT>(S) + (int64_t)col * k;
  for (int q = tid; q < rows; q += kThreads) v0[x0 + q] = (VT)wc[x0 + q];
  if (chunk == 0 && tid == 0) {
    S.active[col] = 1;
    S.iters[col] = 0;
    if (col == 0) {
      S.jdev[0] = 0;
      S.tolv[0] = tol;
    }
  }
}

// Start of a deflated solve from b: r_0 = b - (Z c2 + {S, S^T} Z c2) into w and V_0,
// all columns active, j = 0 and the tolerance (the values of k_prolong followed by
// k_gm_start, in one launch).
template <typename VT>
__global__ __launch_bounds__(256) void k_gm_start_defl(DevPlan P, GmState S, const double* __restrict__ b,
                                                       const double* __restrict__ c2, int transpose, double tol) {
  const int col = blockIdx.y, tid = threadIdx.x;
  if (blockIdx.x == 0 && tid == 0) {
    S.active[col] = 1;
    S.iters[col] = 0;
    if (col == 0) {
      S.jdev[0] = 0;
      S.tolv[0] = tol;
    }
  }
  const int64_t slot = (int64_t)blockIdx.x * kThreads + tid;
  if (slot >= P.k) return;
  const double acc = deflation(P, c2 + (int64_t)col * P.d, slot, transpose != 0);
  const int64_t o = (int64_t)col * P.k + slot;
  const double v = b[o] + -1.0 * acc;
  S.w[o] = v;
  basis<VT>(S)[o] = (VT)v;
}

// y = R^{-1} g for the first iters[col] columns (R = rotated Hessenberg), one
// block per column, column-oriented back substitution.
constexpr int kLsqStage = 64;  // Krylov dimensions whose triangle is staged in LDS
__global__ __launch_bounds__(256) void k_gm_lsq(GmState S) {
  __shared__ double gs[kMaxIt + 1];
  __shared__ double rs[kLsqStage * kLsqStage];
  const int col = blockIdx.x, tid = threadIdx.x;
  const int J = S.iters[col];
  const double* gc = S.g + (int64_t)col * S.ldv;
  const double* Hc = S.H + (int64_t)col * S.ldv * S.maxit;
  double* yc = S.y + (int64_t)col * S.ldv;
  for (int i = tid; i < J; i += kThreads) gs[i] = gc[i];
  for (int i = J + tid; i < S.ldv; i += kThreads) yc[i] = 0.0;
  if (J <= kLsqStage) {
    // the triangle staged in LDS with every load in flight, then the same steps
    // from LDS (one memory round trip instead of two per column)
    for (int t = tid; t < J * J; t += kThreads) {
      const int i = t / J, m = t - i * J;
      if (m <= i) rs[i * kLsqStage + m] = Hc[(int64_t)i * S.ldv + m];
    }
    __syncthreads();
    // one wave: lane m keeps g_m in a register; the steps need no barrier
    if (tid >= 64) return;
    double g = tid < J ? gs[tid] : 0.0;
    for (int i = J - 1; i >= 0; --i) {
      const double yi = __shfl(g, i) / rs[i * kLsqStage + i];
      if (tid < i) g = fma(-rs[i * kLsqStage + tid], yi, g);
      if (tid == 0) yc[i] = yi;
    }
    return;
  }
  __syncthreads();
  for (int i = J - 1; i >= 0; --i) {
    const double yi = gs[i] / Hc[(int64_t)i * S.ldv + i];
    __syncthreads();
    for (int m = tid; m < i; m += kThreads) gs[m] = fma(-Hc[(int64_t)i * S.ldv + m], yi, gs[m]);
    if (tid == 0) yc[i] = yi;
    __syncthreads();
  }
}

// x = sum_{i < iters[col]} y_i V_i
template <typename VT>
__global__ __launch_bounds__(256) void k_gm_combine(DevPlan P, GmState S, double* __restrict__ x) {
  const int col = blockIdx.y;
  const int64_t k = P.k;
  const int J = S.iters[col];
  const double* yc = S.y + (int64_t)col * S.ldv;
  const VT* Vc = basis<VT>(S) + (int64_t)col * k;
  for (int64_t q = (int64_t)blockIdx.x * kThreads + threadIdx.x; q < k; q += (int64_t)gridDim.x * kThreads) {
    double acc = 0.0;
    for (int i0 = 0; i0 < J; i0 += 8) {
      double v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = Vc[(int64_t)min(i0 + u, J - 1) * S.vvs + q];
#pragma unroll
      for (int u = 0; u < 8; ++u)
        if (i0 + u < J) acc = fma(yc[i0 + u], v[u], acc);
    }
    x[(int64_t)col * k + q] = acc;
  }
}

// ------------------------------------------------------------------ launchers

void gm_start_deflated(const DevPlan& P, const GmState& S, int nrhs, const double* b, const double* c2, bool tr,
                       double tol, hipStream_t s) {
  const dim3 g((unsigned)((P.k + kThreads - 1) / kThreads), nrhs);
  if (S.basis32)
    hipLaunchKernelGGL(k_gm_start_defl<float>, g, dim3(kThreads), 0, s, P, S, b, c2, tr ? 1 : 0, tol);
  else
    hipLaunchKernelGGL(k_gm_start_defl<double>, g, dim3(kThreads), 0, s, P, S, b, c2, tr ? 1 : 0, tol);
}

void gm_start(const DevPlan& P, const GmState& S, int nrhs, double tol, hipStream_t s) {
  if (S.basis32)
    hipLaunchKernelGGL(k_gm_start<float>, dim3(S.nch, nrhs), dim3(kThreads), 0, s, P, S, tol);
  else
    hipLaunchKernelGGL(k_gm_start<double>, dim3(S.nch, nrhs), dim3(kThreads), 0, s, P, S, tol);
}

// block 0 of gm_update takes the Givens step; the others share the slots
static int precond_grid(const DevPlan& P, const GmState& S, int kind) {
  return 1 + (kind == 1 ? S.nch : std::max(1, std::min(P.nblk, 1024)));
}

void gm_step(const DevPlan& P, const GmState& S, int nrhs, int par, int kind, bool tr, hipStream_t s, int sprec,
             int mprec) {
  const dim3 pg(precond_grid(P, S, kind), nrhs);
  const int up = kind == 1 ? 0 : 1, trn = tr ? 1 : 0;
  if (S.prereduce && nrhs >= 2 && up) {
    // several columns per workgroup: each block-Jacobi inverse is read once for them
    const int nc = nrhs >= 4 ? 4 : 2;
    const dim3 pn(pg.x, (nrhs + nc - 1) / nc);
#define SMPM_UPDATE_NV(T, VT)                                                                        \
  if (nc == 4)                                                                                       \
    hipLaunchKernelGGL((k_gm_update_n<T, 4, VT>), pn, dim3(kThreads), 0, s, P, S, par, up, trn);      \
  else                                                                                               \
    hipLaunchKernelGGL((k_gm_update_n<T, 2, VT>), pn, dim3(kThreads), 0, s, P, S, par, up, trn);
#define SMPM_UPDATE_N(T)      \
  if (S.basis32) {            \
    SMPM_UPDATE_NV(T, float)  \
  } else {                    \
    SMPM_UPDATE_NV(T, double) \
  }
    if (mprec == PREC_F32) {
      SMPM_UPDATE_N(float)
    } else if (mprec == PREC_BF16) {
      SMPM_UPDATE_N(bf16s)
    } else {
      SMPM_UPDATE_N(double)
    }
#undef SMPM_UPDATE_N
#undef SMPM_UPDATE_NV
  } else {
#define SMPM_UPDATE_1V(T, VT)                                                                               \
  if (S.prereduce)                                                                                          \
    hipLaunchKernelGGL((k_gm_update<T, true, VT>), pg, dim3(kThreads), 0, s, P, S, par, up, trn);           \
  else                                                                                                      \
    hipLaunchKernelGGL((k_gm_update<T, false, VT>), pg, dim3(kThreads), 0, s, P, S, par, up, trn);
#define SMPM_UPDATE_1(T)      \
  if (S.basis32) {            \
    SMPM_UPDATE_1V(T, float)  \
  } else {                    \
    SMPM_UPDATE_1V(T, double) \
  }
    if (mprec == PREC_F32) {
      SMPM_UPDATE_1(float)
    } else if (mprec == PREC_BF16) {
      SMPM_UPDATE_1(bf16s)
    } else {
      SMPM_UPDATE_1(double)
    }
#undef SMPM_UPDATE_1
#undef SMPM_UPDATE_1V
  }
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
  if (S.basis32)
    hipLaunchKernelGGL(k_gm_dots<float>, dim3(S.nch, nrhs), dim3(kThreads), 0, s, P, S, par, kind == 3 ? 1 : 0,
                       tr ? 1 : 0);
  else
    hipLaunchKernelGGL(k_gm_dots<double>, dim3(S.nch, nrhs), dim3(kThreads), 0, s, P, S, par, kind == 3 ? 1 : 0,
                       tr ? 1 : 0);
  if (S.prereduce)
    hipLaunchKernelGGL(k_gm_reduce, dim3((S.maxit + kReduceVecs) / kReduceVecs, nrhs), dim3(256), 0, s, S, par);
}

void gm_finish(const DevPlan& P, const GmState& S, int nrhs, double* x, hipStream_t s) {
  hipLaunchKernelGGL(k_gm_lsq, dim3(nrhs), dim3(kThreads), 0, s, S);
  const int64_t blocks = std::min<int64_t>((P.k + kThreads - 1) / kThreads, 2048);
  if (S.basis32)
    hipLaunchKernelGGL(k_gm_combine<float>, dim3((unsigned)blocks, nrhs), dim3(kThreads), 0, s, P, S, x);
  else
    hipLaunchKernelGGL(k_gm_combine<double>, dim3((unsigned)blocks, nrhs), dim3(kThreads), 0, s, P, S, x);
}

int gm_rows_per_chunk(int64_t k) {
  // chunks of 256..kRowsMax rows, at most ~256 chunks
  int64_t rows = 256;
  while (rows < kRowsMax && (k + rows - 1) / rows > 256) rows *= 2;
  return (int)rows;
}

}  // namespace smpm
