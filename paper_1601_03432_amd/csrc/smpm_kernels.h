// Device-side view of the plan and the launchers of the gfx950 kernels.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace smpm {

constexpr int kMaxN = 32;

// Plain-old-data view of the device copy of a Plan; passed to kernels by value.
struct DevPlan {
  int n, n2, nel, d, nblk, ncls, mx, my;
  int has_coarse;          // 1 if the coarse solve is built (deflation available)
  int coarse_mode;         // 1: dense G, 2: substructured
  int64_t r, k, nsides, nbdry;
  const int* nbr;          // nel*4
  const int* cls;          // nel
  const int* slot_off;     // nel+1
  const int* side_slot;    // nel*4
  const int* iface;        // nel*4
  const int* side_elem;    // nsides
  const int* side_dir;     // nsides
  // per side, 8 ints: the deflation's interfaces and coefficient offsets
  //   side_fwd: own interface, the neighbour's 4 interfaces, WZ offset of (neighbour class, facing side)
  //   side_adj: own interface, the element's 4 interfaces, WZc offset of the element class, first slot
  const int* side_fwd;
  const int* side_adj;
  const int* iface_side;   // d*2
  const int* cls_nslots;   // ncls
  const int* cls_sidecol;  // ncls*4
  const int64_t* W_off;    // ncls*4
  const int64_t* H_off;    // ncls*4
  const double* Wc;        // [c][i]
  const double* Wr;        // [i][c]
  const double* Hc;        // [l][i]
  const double* Hr;        // [i][l]
  const double* WZ;        // [cls][s'][t][s'']
  const double* WZc;       // [cls][s'][c]  column sums of W over its rows
  const double* Ainv;      // [cls][l][m]
  const double* AinvT;     // [cls][m][l]
  const int* blk_off;
  const int* blk_slots;
  const int* blk_cls;
  const int64_t* bcls_off;
  const int* bcls_size;
  const double* MinvC;     // [c][r]
  const double* MinvR;     // [r][c]
  const double* G;         // d x d row-major
  const double* GT;        // its transpose
  // substructured coarse solve (patch interiors + separator Schur complement)
  int sub_npatch, sub_nsep, sub_border;
  const int* sub_I_off;    // npatch+1
  const int* sub_I;        // interior interfaces of each patch
  const int* sub_B_off;    // npatch+1
  const int* sub_B;        // separators touching each patch
  const int64_t* sub_K_off;
  const int64_t* sub_FR_off;
  const double* sub_Kc;    // K_pp^{-1} column-major / row-major
  const double* sub_Kr;
  const double* sub_Fc;    // F_p = K_pp^{-1} K_{I,B}  (ni x nbb)
  const double* sub_Fr;
  const double* sub_Rc;    // R_p = K_{B,I} K_pp^{-1}  (nbb x ni)
  const double* sub_Rr;
  const int* sub_sep_iface;  // nsep
  const int* sub_sep_pl;     // nsep*4: (patch, local) of both patches
  const int* sub_B_iface;    // per entry of sub_B: the separator's interface
  const int* sub_sep_woff;   // nsep*2: where the two patches' parts of a separator sit in cws
  const double* sub_Si;    // separator system inverse, row-major, and its transpose
  const double* sub_SiT;
  int sub_lds_max;         // max over patches of max(ni, nbb): LDS doubles of the patch kernels
  double* cws;             // per-column scratch of the substructured solve
  int64_t cws_stride;
  const int* bdry_node;    // nbdry
  const double* bdry_tau;  // nbdry
  // low-precision copies of the Schur side fluxes and block-Jacobi inverses
  const float* WcF;
  const float* WrF;
  const float* MinvCF;
  const float* MinvRF;
  const unsigned short* WcB;     // bf16 bit patterns (upper half of an IEEE float)
  const unsigned short* WrB;
  const unsigned short* MinvCB;
  const unsigned short* MinvRB;
  int ngrp;                // element groups (same class, up to grp_size elements)
  int grp_size;            // 1, 2, 4 or 8
  const int* grp_cls;      // ngrp
  const int* grp_elem;     // ngrp*kGroup, -1 padded
  int ntile;               // matrix-core tiles (same class, up to kTile elements)
  const int* tile_cls;     // ntile
  const int* tile_elem;    // ntile*kTile, -1 padded
  const int* tile_src;     // ntile*kTile: first slot of the element, -1 if none
  const int* tile_dst;     // ntile*kTile*4: first slot facing side s, -1 if none
  int mma_mt;              // 16-row tiles of the matrix-core operator fragments (0: n > 16)
  int schur_nc[4];         // right-hand-side columns per Schur workgroup for 1, 2-3, 4-7 and
                           // >= 8 columns (0: built-in choice); set by the autotuner
  int schur_pers[4];       // persistent Schur apply per column-count class: -1 never, 0 when
                           // items >= 2x resident workgroups, 1 always, 2 the warp-specialized
                           // persistent kernel, 3 the column-pipelined kernel (no side sums)
  int schur_cpw[4];        // columns per workgroup of the column-pipelined kernel (0: 8)
  int num_cu;              // compute units of the device
  const double* Afwd;      // [cls][w][q][lane] fragments of W (forward) and W^T (transpose)
  const double* Aadj;
  const float* AfwdF;
  const float* AadjF;
  const unsigned short* AfwdB;
  const unsigned short* AadjB;
};

constexpr int kGroup = 8;
constexpr int kTile = 16;

// Workgroup b of nb (nb a multiple of 8) mapped so that each of the 8 XCDs (which
// receive workgroup ids round-robin) works on one contiguous range: neighbouring
// work items then share an L2.
__device__ __forceinline__ int xcd_block(int b, int nb) { return (b & 7) * (nb >> 3) + (b >> 3); }

// operator precision of the Schur / block-Jacobi applies
enum OpPrec { PREC_F64 = 0, PREC_F32 = 1, PREC_BF16 = 2 };

struct bf16s {
  unsigned short v;
};

template <typename T>
struct AccOf {
  using type = float;
};
template <>
struct AccOf<double> {
  using type = double;
};

__device__ __forceinline__ double to_acc(double v) { return v; }
__device__ __forceinline__ float to_acc(float v) { return v; }
__device__ __forceinline__ float to_acc(bf16s v) { return __uint_as_float((unsigned)v.v << 16); }

template <typename T>
__device__ __forceinline__ const T* schur_op(const DevPlan& P, bool rows_fast);
template <>
__device__ __forceinline__ const double* schur_op<double>(const DevPlan& P, bool c) { return c ? P.Wc : P.Wr; }
template <>
__device__ __forceinline__ const float* schur_op<float>(const DevPlan& P, bool c) { return c ? P.WcF : P.WrF; }
template <>
__device__ __forceinline__ const bf16s* schur_op<bf16s>(const DevPlan& P, bool c) {
  return reinterpret_cast<const bf16s*>(c ? P.WcB : P.WrB);
}
template <typename T>
__device__ __forceinline__ const T* mma_op(const DevPlan& P, bool adj);
template <>
__device__ __forceinline__ const double* mma_op<double>(const DevPlan& P, bool adj) { return adj ? P.Aadj : P.Afwd; }
template <>
__device__ __forceinline__ const float* mma_op<float>(const DevPlan& P, bool adj) { return adj ? P.AadjF : P.AfwdF; }
template <>
__device__ __forceinline__ const bf16s* mma_op<bf16s>(const DevPlan& P, bool adj) {
  return reinterpret_cast<const bf16s*>(adj ? P.AadjB : P.AfwdB);
}
// One block-Jacobi block applied by a 256-thread workgroup to NV vectors x_v (LDS,
// x_v[c] = xs[v * xstride + c]): y_{v,r} = sum_c M[c*sb + r] x_{v,c} (sb <= 8 kMaxN =
// 256), each entry of M read once for all NV vectors.  The columns of each row are
// split into 256/sb contiguous parts summed by separate threads and then added in a
// fixed order, so every caller (and every NV) gets the same bits per vector.
// Contains a barrier: call from all threads.  part: LDS, NV * 256 Acc.
template <int NV, typename OpT, typename Acc, typename Store>
__device__ __forceinline__ void block_jacobi_apply(const OpT* __restrict__ Mp, const Acc* xs, int xstride, int sb,
                                                   Acc* part, Store store) {
  const int tid = threadIdx.x;
  const int np = max(1, 256 / sb), len = (sb + np - 1) / np;
  if (tid < np * sb) {
    const int r = tid % sb, p = tid / sb;
    const int c0 = p * len, c1 = min(sb, c0 + len);
    Acc acc[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) acc[v] = 0;
#pragma unroll 8
    for (int c = c0; c < c1; ++c) {
      const Acc mv = to_acc(Mp[c * sb + r]);
#pragma unroll
      for (int v = 0; v < NV; ++v) acc[v] = fma(mv, xs[v * xstride + c], acc[v]);
    }
#pragma unroll
    for (int v = 0; v < NV; ++v) part[v * 256 + p * sb + r] = acc[v];
  }
  __syncthreads();
  if (tid < sb) {
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      Acc sum = part[v * 256 + tid];
      for (int p = 1; p < np; ++p) sum += part[v * 256 + p * sb + tid];
      store(v, tid, sum);
    }
  }
}

// (Z c2 + S Z c2)[slot] (forward) or (Z c2 + S^T Z c2)[slot] (transpose): the coarse
// value of the slot's interface plus the coupling of the interfaces the side's
// flux reaches, from the side's table entry (two 16-byte loads), then the values.
// The side's table entry (two int4) of a slot, for deflation_tb.
__device__ __forceinline__ void deflation_table(const DevPlan& P, int64_t slot, bool transpose, int4& a, int4& b) {
  const int4* tb = reinterpret_cast<const int4*>((transpose ? P.side_adj : P.side_fwd) + (slot / P.n) * 8);
  a = tb[0];
  b = tb[1];
}
// deflation() from the slot's table entry, loaded beforehand
__device__ __forceinline__ double deflation_tb(const DevPlan& P, const double* __restrict__ cc, int64_t slot,
                                               bool transpose, int4 a, int4 b) {
  const int n = P.n;
  const int tt = (int)(slot % n);
  const int js[4] = {a.y, a.z, a.w, b.x};
  double acc = cc[a.x];
  if (!transpose) {
    const double* wz = P.WZ + b.y + tt * 4;
#pragma unroll
    for (int s2 = 0; s2 < 4; ++s2)
      if (js[s2] >= 0) acc = fma(wz[s2], cc[js[s2]], acc);
  } else {
    const int cidx = (int)(slot - b.z);
#pragma unroll
    for (int s2 = 0; s2 < 4; ++s2)
      if (js[s2] >= 0) acc = fma(P.WZc[(int64_t)b.y + s2 * 4 * n + cidx], cc[js[s2]], acc);
  }
  return acc;
}
__device__ __forceinline__ double deflation(const DevPlan& P, const double* __restrict__ cc, int64_t slot,
                                            bool transpose) {
  const int n = P.n;
  const int si = (int)(slot / n), tt = (int)(slot - (int64_t)si * n);
  const int4* tb = reinterpret_cast<const int4*>((transpose ? P.side_adj : P.side_fwd) + (int64_t)si * 8);
  const int4 a = tb[0], b = tb[1];
  const int js[4] = {a.y, a.z, a.w, b.x};
  double acc = cc[a.x];
  if (!transpose) {
    const double* wz = P.WZ + b.y + tt * 4;
#pragma unroll
    for (int s2 = 0; s2 < 4; ++s2)
      if (js[s2] >= 0) acc = fma(wz[s2], cc[js[s2]], acc);
  } else {
    const int cidx = (int)(slot - b.z);
#pragma unroll
    for (int s2 = 0; s2 < 4; ++s2)
      if (js[s2] >= 0) acc = fma(P.WZc[(int64_t)b.y + s2 * 4 * n + cidx], cc[js[s2]], acc);
  }
  return acc;
}

template <typename T>
__device__ __forceinline__ const T* minv_op(const DevPlan& P, bool transpose);
template <>
__device__ __forceinline__ const double* minv_op<double>(const DevPlan& P, bool tr) {
  return tr ? P.MinvR : P.MinvC;
}
template <>
__device__ __forceinline__ const float* minv_op<float>(const DevPlan& P, bool tr) {
  return tr ? P.MinvRF : P.MinvCF;
}
template <>
__device__ __forceinline__ const bf16s* minv_op<bf16s>(const DevPlan& P, bool tr) {
  return reinterpret_cast<const bf16s*>(tr ? P.MinvRB : P.MinvCB);
}

// ---- operator applies; nrhs columns, column-blocked with the natural lengths
void launch_schur(const DevPlan& P, const double* y, double* t, int nrhs, bool transpose,
                  const int* active, hipStream_t s);
// as launch_schur; if side_sums != nullptr (forward, n <= 16 only) it also writes the
// sum of t over every inter-element side (nsides per column).  stream_out: t is not
// read again soon (it goes back to the caller), so the FP64 matrix-core kernel writes
// it with non-temporal stores.
void launch_schur_ex(const DevPlan& P, const double* y, double* t, int nrhs, bool transpose,
                     const int* active, double* side_sums, hipStream_t s, int prec = PREC_F64,
                     bool stream_out = false);
bool schur_has_side_sums(const DevPlan& P);
int schur_nc_class(int nrhs);  // index into DevPlan::schur_nc
// persistent, pipelined Schur apply (no side sums); false if the plain launch is used
bool launch_schur_pers(const DevPlan& P, const double* y, double* t, int nrhs, bool transpose, const int* active,
                       hipStream_t s, int prec);

// c2 = G c with c_j = side_sums of interface j's two sides
void launch_coarse_sides(const DevPlan& P, const double* side_sums, double* c2, int nrhs, bool transpose,
                         const int* active, hipStream_t s);
void launch_flux(const DevPlan& P, const double* f, double* b, int nrhs, hipStream_t s);      // b = B A^{-1} f
void launch_flux_adj(const DevPlan& P, const double* x, double* y, int nrhs, hipStream_t s);  // y = A^{-T} B^T x
void launch_backsub(const DevPlan& P, const double* f, const double* x, double* u, int nrhs,
                    hipStream_t s);                                                             // u = A^{-1}(f - E x)
void launch_local_adj(const DevPlan& P, const double* c, double* out, int nrhs, bool to_slots,
                      hipStream_t s);                         // out = A^{-T} c (r) or E^T A^{-T} c (k)
void launch_precond(const DevPlan& P, const double* x, double* y, int nrhs, bool transpose,
                    const int* active, hipStream_t s, int prec = 0);
void launch_iface_sum(const DevPlan& P, const double* t, double* c, int nrhs, const int* active,
                      hipStream_t s);                                                           // c = Z^T t
void launch_coarse(const DevPlan& P, const double* c, double* c2, int nrhs, bool transpose,
                   const int* active, hipStream_t s);                                          // c2 = G c
// w = t + sign * (Z c2 + SZ c2) with sz = 0: no S term, 1: S Z, 2: S^T Z
void launch_prolong(const DevPlan& P, const double* t, const double* c2, double* w, int nrhs, int sz,
                    double sign, const int* active, hipStream_t s);
// rhs = f + T g (g may be NULL); *flag is set to 1 if f or g holds a non-finite entry
void launch_rhs(const DevPlan& P, const double* f, const double* g, double* rhs, int nrhs, int* flag,
                hipStream_t s);
// b = a over len doubles (a kernel, so it can be captured into a graph)
void launch_copy(const double* a, double* b, int64_t len, hipStream_t s);
// *flag = 1 if a[0..len) holds a non-finite entry (flag cleared by the caller)
void launch_check_finite(const double* a, int64_t len, int* flag, hipStream_t s);
void launch_bdry_adj(const DevPlan& P, const double* mu, double* dg, int nrhs, hipStream_t s);  // dg = T^T mu

void launch_fill_pattern(double* b, int64_t len, hipStream_t s);  // values in (-1, 1) for timing runs

// ---- small results into pinned (mapped, coherent) host memory by a kernel
void launch_publish(const double* src, int n, double* host_dst, hipStream_t s);
void launch_publish_i(const int* src, int n, int* host_dst, hipStream_t s);
// up to eight double ranges and one int range in one launch (unused entries: n = 0)
struct PublishSet {
  const double* src[8];
  double* dst[8];
  int n[8];
  const int* isrc;
  int* idst;
  int in;
};
void launch_publish_set(const PublishSet& p, hipStream_t s);

// ---- vector kernels over nrhs columns of length len (column stride ld)
int reduce_chunks(int64_t len);
// out[col*nvec + i] = sum_x A_i(col)[x] * b(col)[x] * (wt ? wt[x] : 1)
// A_i(col) = A + col*a_cs + i*a_vs.  part: scratch of nrhs*nvec*reduce_chunks(len)
void launch_mdot(const double* A, int64_t a_vs, int64_t a_cs, int nvec, const double* b, int64_t b_cs,
                 const double* wt, int64_t len, int nrhs, double* part, double* out, const int* active,
                 hipStream_t s);
// w(col) = w(col) - sum_i coef[col*nvec + i] * A_i(col)     (coef scaled by `scale`)
void launch_mupdate(double* w, int64_t w_cs, const double* A, int64_t a_vs, int64_t a_cs, int nvec,
                    const double* coef, double scale, int64_t len, int nrhs, const int* active, hipStream_t s);
// y(col) = x(col) - (dot[col] * scale) * u   (u shared by all columns); y may alias x
void launch_axpy_shared(const double* x, int64_t x_cs, const double* u, const double* dot, double scale,
                        double* y, int64_t len, int nrhs, hipStream_t s);
// y(col) = x(col) * (1/ nrm[col])  where nrm holds squared norms when sq=true
void launch_scale_inv(const double* x, int64_t x_cs, const double* nrm, bool sq, double* y, int64_t y_cs,
                      int64_t len, int nrhs, const int* active, hipStream_t s);
void launch_add(const double* a, const double* b, double sb, double* y, int64_t len, int nrhs, hipStream_t s);
// Fused pairs (the first three give the bits of the two launches they replace):
//  out[col] = sum_x (a + sb b)[x]^2                         (launch_add, then launch_mdot of the result with itself)
void launch_norm2_diff(const double* a, const double* b, double sb, int64_t len, int nrhs, double* part, double* out,
                       hipStream_t s);
//  y = x - dot[col] * scale * u, out[col] = |y|^2            (launch_axpy_shared, then launch_mdot(y, y));
//  with sides != nullptr also the sums of y over runs of n entries into sides (len / n per column; n a
//  power of two <= 64: the per-side sums of a slot vector)
void launch_axpy_norm2(const double* x, const double* u, const double* dot, double scale, double* y, int64_t len,
                       int nrhs, double* part, double* out, hipStream_t s, double* sides = nullptr, int n = 0);
//  c = Z^T (a + sb t)                                       (launch_add, then launch_iface_sum)
void launch_iface_sum_diff(const DevPlan& P, const double* a, const double* t, double sb, double* c, int nrhs,
                           hipStream_t s);
//  u = A^{-1}(f - E x) and out[col] = wq . u (partials in part, one per tile-block and row
//  group); false (nothing launched) when the element applies do not run on the matrix
//  cores (n > 16)
bool launch_backsub_dot(const DevPlan& P, const double* f, const double* x, double* u, const double* wq, int nrhs,
                        double* part, double* out, hipStream_t s);
//  ft = f - dot[col] * scale * u (r-vector), then b = B A^{-1} ft, and with du != nullptr
//  dout[col] = du . b (partials in part, 4 per tile-block); false (nothing launched) when the
//  element applies do not run on the matrix cores (n > 16)
bool launch_flux_projected(const DevPlan& P, const double* f, const double* u, const double* dot, double scale,
                           double* ft, double* b, int nrhs, hipStream_t s, const double* du = nullptr,
                           double* part = nullptr, double* dout = nullptr);

// ---- GMRES small dense work (one thread per column)
// H(col) (ldh x maxit col-major: H[j*ldh + i]), cs, sn, g of length ldh; hnew: j+1 coefficients,
// nrm2: squared norm of the orthogonalized vector.  Writes res[col] = |g[j+1]|.
void launch_givens(double* H, int ldh, double* cs, double* sn, double* g, const double* hnew,
                   const double* nrm2, int j, int nrhs, double* res, const int* active, hipStream_t s);
void launch_lsq(const double* H, int ldh, const double* g, const int* jcount, double* y, int nrhs,
                hipStream_t s);

}  // namespace smpm
