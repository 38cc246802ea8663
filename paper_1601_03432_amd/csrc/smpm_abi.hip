// C ABI of libsmpm: context lifetime, device upload, operator applies,
// projections and the Algorithm 3 GMRES driver.  Every numerical step runs in
// the kernels of smpm_kernels.hip; the host only sequences launches and reads
// per-column residual estimates to decide convergence.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <mutex>
#include <thread>
#include <functional>
#include <vector>

#include "../../include/smpm.h"
#include "smpm_gmres.h"
#include "smpm_block.h"
#include "smpm_kernels.h"
#include "smpm_plan.h"

using namespace smpm;

namespace {
thread_local std::string g_err;

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

#define HIPCHK(expr)                                                                  \
  do {                                                                                \
    hipError_t e_ = (expr);                                                           \
    if (e_ != hipSuccess) return fail(SMPM_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

// Solver workspace sized for (nrhs, maxit); grown on demand.
struct Workspace {
  int nrhs = 0, maxit = 0;
  double *rhs = nullptr, *ft = nullptr, *bS = nullptr, *bhat = nullptr, *x = nullptr;
  double *z = nullptr, *t = nullptr, *w = nullptr, *c = nullptr, *c2 = nullptr;
  double *V = nullptr, *H = nullptr, *cs = nullptr, *sn = nullptr, *g = nullptr;
  double *h1 = nullptr, *h2 = nullptr, *scal = nullptr, *scal2 = nullptr, *res = nullptr, *y = nullptr;
  double* part = nullptr;
  int *active = nullptr, *jcount = nullptr;
  // device-resident GMRES state
  double *part1 = nullptr, *part2 = nullptr, *sides = nullptr;
  double *Hu = nullptr, *dw = nullptr;  // device GMRES: unrotated Hessenberg, reduced dots
  double *xacc = nullptr, *rho = nullptr;  // iterative refinement: solution and residual
  double* xprev = nullptr;                  // iterate before the last correction
  double* cws = nullptr;                    // substructured coarse solve scratch
  double* ubuf = nullptr;                   // r x nrhs: back-substituted solution before the mean
  double* tolv = nullptr;                   // device GMRES: tolerance and step counter
  int* jdev = nullptr;
  double *tolb = nullptr;
  int* iters = nullptr;
  int* pinned = nullptr;  // pinned host block: flags (2 x nrhs ints), then hres / hout
  double* hres = nullptr;  // 2 x nrhs residual-estimate ratios (per chunk slot)
  double* hout = nullptr;  // 4 x nrhs small results
  int* hiters = nullptr;   // nrhs iteration counts
  // f or g held a non-finite entry: a flag in the pinned (coherent) area, set by the
  // kernels that first read f and g, cleared and read by the host around a solve
  int* nonfinite = nullptr;
  int* hnonfinite = nullptr;  // the same flag (host view)
  double* hhist = nullptr;    // pinned: column 0's rotated right-hand side g (maxit + 1) and tol |ref|
  double* hhist_cs = nullptr;
  double* hhist_tolb = nullptr;
  int hist_len = 0;           // entries of the last GMRES run's history (iterations + 1)
  double hist_tol = 1.0;      // that run's relative tolerance (threshold = tol * reference)
  int* hseq = nullptr;  // pinned: chunks of Arnoldi steps reported by the device (GmState)
  int nch = 0, rows = 0;
  std::vector<void*> mem;
};

// Block GMRES workspace for (s columns, maxit block steps); grown on demand.  The
// basis lives in Workspace::V (s (maxit + 1) vectors fit there).
struct BlockWs {
  int s = 0, maxit = 0, cap = 0, ldH = 0;
  double *H = nullptr, *refl = nullptr, *rbeta = nullptr, *G = nullptr, *res = nullptr;
  double *h = nullptr, *h2 = nullptr, *gram = nullptr, *T1 = nullptr, *T2 = nullptr, *R1 = nullptr, *R2 = nullptr;
  double *Y = nullptr, *part = nullptr, *ht = nullptr;
  int* cnt = nullptr;        // device: kept counts of the two Cholesky QR passes
  int* hcnt = nullptr;       // pinned: the same, published after each step
  double* hres = nullptr;    // pinned: least-squares residual per column
  double* href = nullptr;    // pinned: squared stopping reference per column
  std::vector<void*> mem;
  void* pinned = nullptr;
};

}  // namespace

struct smpm_ctx {
  Plan plan;
  bool device = false;
  int dev_id = -1;
  DevPlan dp{};
  std::vector<void*> mem;                    // setup allocations
  double *uL = nullptr, *uS = nullptr, *v0hat = nullptr, *wq = nullptr, *ones = nullptr;
  double *rhat = nullptr;                    // 1/sqrt(r) vector (left null vector of L^T)
  double* zv0 = nullptr;                     // Z^T v0hat (d), for the deflated null-vector solve
  double *r1_p = nullptr, *r1_q1 = nullptr, *r1_q2 = nullptr;  // its exact coarse correction
  bool r1_defl = false;                      // the deflated null-vector solve is set up
  double wsum = 0;
  bool precond_regular = true;               // false when the single block is all of S
  bool have_null = false;                    // u_L, u_S computed (on first use)
  double null_residual = -1.0;               // ||S^T u_S|| / ||S|| bound (-1: not computed)
  int null_iterations = 0;                   // GMRES iterations the null-vector solve took
  std::vector<double> h_uL, h_uS;
  Workspace ws;
  BlockWs bws;
  // captured chunks of Arnoldi steps, keyed by the solve's shape; they hold workspace
  // pointers, so a workspace reallocation drops them
  struct GraphEntry {
    int nrhs, kind, tr, sprec, mprec, maxit, prereduce, stream, rule;
    int phase;           // 0: a chunk of Arnoldi steps, 1: a solve's pre-phase, 2: its post-phase
    uint64_t tolbits;    // the tolerance the phase bakes in (pre-phase)
    hipGraphExec_t exec;
  };
  std::vector<GraphEntry> graphs;
  hipStream_t cap_stream = nullptr;          // capture-only stream (default priority)
  hipStream_t group_stream = nullptr;        // this problem's stream in smpm_solve_group
  int prereduce_choice[4] = {-1, -1, -1, -1};  // per column-count class: -1 built-in rule, 0/1 tuned
  // inner solves with FP32 / BF16 operators keep their Krylov basis in FP32 (read at
  // setup; the environment SMPM_MIXED_BASIS=64 keeps it FP64, for comparisons)
  int mixed_basis32 = 1;
  void drop_graphs() {
    for (auto& g : graphs) (void)hipGraphExecDestroy(g.exec);
    graphs.clear();
  }
  ~smpm_ctx() {
    if (device) {
      drop_graphs();
      if (cap_stream) (void)hipStreamDestroy(cap_stream);
      if (group_stream) (void)hipStreamDestroy(group_stream);
      for (void* p : ws.mem) (void)hipFree(p);
      if (ws.pinned) (void)hipHostFree(ws.pinned);
      for (void* p : bws.mem) (void)hipFree(p);
      if (bws.pinned) (void)hipHostFree(bws.pinned);
      for (void* p : mem) (void)hipFree(p);
    }
  }
};

namespace {

// float -> bf16 with round-to-nearest-even on the discarded 16 bits
uint16_t to_bf16(float f) {
  uint32_t u;
  std::memcpy(&u, &f, sizeof u);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

std::vector<float> to_f32(const std::vector<double>& v) {
  std::vector<float> o(v.size());
  for (size_t i = 0; i < v.size(); ++i) o[i] = (float)v[i];
  return o;
}

std::vector<uint16_t> to_b16(const std::vector<double>& v) {
  std::vector<uint16_t> o(v.size());
  for (size_t i = 0; i < v.size(); ++i) o[i] = to_bf16((float)v[i]);
  return o;
}

template <class T>
int upload(smpm_ctx* c, const std::vector<T>& v, const T** out, hipStream_t s) {
  if (v.empty()) {
    *out = nullptr;
    return SMPM_OK;
  }
  void* p = nullptr;
  if (hipMalloc(&p, v.size() * sizeof(T)) != hipSuccess) return fail(SMPM_ENOMEM, "hipMalloc failed in setup");
  c->mem.push_back(p);
  HIPCHK(hipMemcpyAsync(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, s));
  *out = static_cast<const T*>(p);
  return SMPM_OK;
}

int dalloc(std::vector<void*>& mem, double** p, size_t count) {
  if (count == 0) count = 1;
  if (hipMalloc((void**)p, count * sizeof(double)) != hipSuccess) return fail(SMPM_ENOMEM, "hipMalloc failed");
  mem.push_back(*p);
  return SMPM_OK;
}

int ialloc(std::vector<void*>& mem, int** p, size_t count) {
  if (count == 0) count = 1;
  if (hipMalloc((void**)p, count * sizeof(int)) != hipSuccess) return fail(SMPM_ENOMEM, "hipMalloc failed");
  mem.push_back(*p);
  return SMPM_OK;
}

int ensure_ws(smpm_ctx* c, int nrhs, int maxit) {
  Workspace& w = c->ws;
  if (w.nrhs >= nrhs && w.maxit >= maxit) return SMPM_OK;
  c->drop_graphs();
  nrhs = std::max(nrhs, w.nrhs);
  maxit = std::max(maxit, w.maxit);
  for (void* p : w.mem) (void)hipFree(p);
  if (w.pinned) (void)hipHostFree(w.pinned);
  w = Workspace();
  const Plan& P = c->plan;
  const size_t r = P.r, k = P.k, d = std::max<int64_t>(P.d, 1), R = nrhs, ldh = maxit + 1;
  int rc = SMPM_OK;
  rc |= dalloc(w.mem, &w.rhs, r * R);
  rc |= dalloc(w.mem, &w.ft, r * R);
  rc |= dalloc(w.mem, &w.bS, k * R);
  rc |= dalloc(w.mem, &w.bhat, k * R);
  rc |= dalloc(w.mem, &w.x, k * R);
  rc |= dalloc(w.mem, &w.z, k * R);
  rc |= dalloc(w.mem, &w.t, k * R);
  rc |= dalloc(w.mem, &w.w, k * R);
  rc |= dalloc(w.mem, &w.c, d * R);
  rc |= dalloc(w.mem, &w.c2, d * R);
  rc |= dalloc(w.mem, &w.V, k * ldh * R);
  rc |= dalloc(w.mem, &w.H, ldh * maxit * R);
  rc |= dalloc(w.mem, &w.cs, ldh * R);
  rc |= dalloc(w.mem, &w.sn, ldh * R);
  rc |= dalloc(w.mem, &w.g, ldh * R);
  rc |= dalloc(w.mem, &w.h1, ldh * R);
  rc |= dalloc(w.mem, &w.h2, ldh * R);
  rc |= dalloc(w.mem, &w.scal, 4 * R);
  rc |= dalloc(w.mem, &w.scal2, 4 * R);
  rc |= dalloc(w.mem, &w.res, R);
  rc |= dalloc(w.mem, &w.y, ldh * R);
  const size_t nch = reduce_chunks(std::max<int64_t>(P.r, P.k));
  // reduction partials: the multi-dots' chunks, or one per back-substitution block
  const size_t ntp = (size_t)((P.ntile + 7) / 8 * 8);  // tile-blocks of the element applies
  const size_t nbk = std::max(ntp * (size_t)((P.n * P.n + 63) / 64), 4 * ntp);
  rc |= dalloc(w.mem, &w.part, std::max(nch * ldh, nbk) * R);
  rc |= ialloc(w.mem, &w.active, R);
  rc |= ialloc(w.mem, &w.jcount, R);
  w.rows = gm_rows_per_chunk(P.k);
  w.nch = (int)((P.k + w.rows - 1) / w.rows);
  rc |= dalloc(w.mem, &w.part1, (size_t)w.nch * ldh * R);
  rc |= dalloc(w.mem, &w.part2, (size_t)w.nch * ldh * R);
  rc |= dalloc(w.mem, &w.Hu, ldh * maxit * R);
  rc |= dalloc(w.mem, &w.dw, ldh * R);
  rc |= dalloc(w.mem, &w.sides, (size_t)P.nsides * R);
  rc |= dalloc(w.mem, &w.xacc, k * R);
  rc |= dalloc(w.mem, &w.ubuf, r * R);
  rc |= dalloc(w.mem, &w.xprev, k * R);
  rc |= dalloc(w.mem, &w.rho, k * R);
  rc |= dalloc(w.mem, &w.tolb, R);
  rc |= ialloc(w.mem, &w.iters, R);
  // scratch of the substructured coarse solve: [patch parts | separator rhs | lambda]
  int64_t cstride = 0;
  if (P.coarse_mode == 2)
    cstride = (int64_t)P.sub.B.size() + (int64_t)P.sub.npatch * P.sub.border + P.sub.nsep + P.sub.border + 1;
  rc |= dalloc(w.mem, &w.cws, (size_t)std::max<int64_t>(cstride, 1) * R);
  rc |= dalloc(w.mem, &w.tolv, 1);
  rc |= ialloc(w.mem, &w.jdev, 2);
  if (rc != SMPM_OK) return SMPM_ENOMEM;
  c->dp.cws = w.cws;
  c->dp.cws_stride = cstride;
  {
    // [flags 2R ints | iters R ints | non-finite flag | chunk count | pad] [hres 2R doubles]
    // [hout 4R doubles] [rotated rhs g: ldh doubles | Givens cosines: ldh doubles | threshold]
    const size_t ibytes = (((3 * R + 2) * sizeof(int) + 63) / 64) * 64;
    const size_t bytes = ibytes + (6 * R + 2 * ldh + 1) * sizeof(double);
    if (hipHostMalloc((void**)&w.pinned, bytes, hipHostMallocCoherent) != hipSuccess)
      return fail(SMPM_ENOMEM, "hipHostMalloc failed");
    w.hiters = w.pinned + 2 * R;
    w.hnonfinite = w.pinned + 3 * R;
    w.nonfinite = w.hnonfinite;
    w.hseq = w.pinned + 3 * R + 1;
    w.hres = reinterpret_cast<double*>(reinterpret_cast<char*>(w.pinned) + ibytes);
    w.hout = w.hres + 2 * R;
    w.hhist = w.hout + 4 * R;
    w.hhist_cs = w.hhist + ldh;
    w.hhist_tolb = w.hhist_cs + ldh;
  }
  if (hipDeviceSynchronize() != hipSuccess) return fail(SMPM_EHIP, "hipDeviceSynchronize failed");
  w.nrhs = nrhs;
  w.maxit = maxit;
  return SMPM_OK;
}

int ensure_bws(smpm_ctx* c, int s, int maxit) {
  BlockWs& b = c->bws;
  if (b.s >= s && b.maxit >= maxit) return SMPM_OK;
  s = std::max(s, b.s);
  maxit = std::max(maxit, b.maxit);
  for (void* p : b.mem) (void)hipFree(p);
  if (b.pinned) (void)hipHostFree(b.pinned);
  b = BlockWs();
  const size_t cap = (size_t)s * (maxit + 1), ldH = cap + kBgMaxCols, S = s, sq = kBgMaxCols * kBgMaxCols;
  int rc = SMPM_OK;
  rc |= dalloc(b.mem, &b.H, ldH * cap);
  rc |= dalloc(b.mem, &b.refl, cap * 64);
  rc |= dalloc(b.mem, &b.rbeta, cap);
  rc |= dalloc(b.mem, &b.G, ldH * S);
  rc |= dalloc(b.mem, &b.res, S);
  rc |= dalloc(b.mem, &b.h, ldH * S);
  rc |= dalloc(b.mem, &b.h2, ldH * S);
  rc |= dalloc(b.mem, &b.ht, ldH * kBgMaxCols);
  rc |= dalloc(b.mem, &b.gram, sq);
  rc |= dalloc(b.mem, &b.T1, sq);
  rc |= dalloc(b.mem, &b.T2, sq);
  rc |= dalloc(b.mem, &b.R1, sq);
  rc |= dalloc(b.mem, &b.R2, sq);
  rc |= dalloc(b.mem, &b.Y, cap * S);
  rc |= dalloc(b.mem, &b.part, (size_t)bg_dot_part_size());
  rc |= ialloc(b.mem, &b.cnt, 2);
  if (rc != SMPM_OK) return SMPM_ENOMEM;
  if (hipHostMalloc(&b.pinned, 64 + 2 * S * sizeof(double), hipHostMallocCoherent) != hipSuccess)
    return fail(SMPM_ENOMEM, "hipHostMalloc failed");
  b.hcnt = static_cast<int*>(b.pinned);
  b.hres = reinterpret_cast<double*>(static_cast<char*>(b.pinned) + 64);
  b.href = b.hres + S;
  b.s = s;
  b.maxit = maxit;
  b.cap = (int)cap;
  b.ldH = (int)ldH;
  return SMPM_OK;
}

int check_device(const smpm_ctx* c) {
  if (!c) return fail(SMPM_EINVAL, "null context");
  if (!c->device) return fail(SMPM_ENODEVICE, "context has no device data (built by smpm_plan)");
  int cur = -1;
  if (hipGetDevice(&cur) != hipSuccess || cur != c->dev_id)
    return fail(SMPM_EINVAL, "current HIP device differs from the context's device");
  return SMPM_OK;
}

// ---------------------------------------------------------------- operator pieces

enum OpKind { OP_S = 1, OP_SM = 2, OP_PSM = 3, OP_RANK1 = 4, OP_RANK1_DEFL = 5 };

// A = S^T + v0hat v0hat^T (nonsingular; its transpose-inverse maps v0hat to a multiple of
// u_S).  Deflated with the coarse space of Algorithm 3: P_A r = r - A Z G^T Z^T r, for
// which A Q_A = P_A A with Q_A = I - Z G^T Z^T A; any fixed coarse map keeps the solve
// exact, and G^T = (C^+)^T approximates (Z^T A Z)^{-1} = (C^T + a a^T)^{-1}, a = Z^T v0hat,
// up to the rank-one term.  w = A Z c2 for the coarse values c2: S^T Z c2 + v0hat (a^T c2).
void rank1_coarse_term(smpm_ctx* c, const double* t, const double* c2, double* w, hipStream_t s) {
  const DevPlan& P = c->dp;
  Workspace& W = c->ws;
  launch_prolong(P, t, c2, w, 1, 2, -1.0, nullptr, s);  // w = t - S^T Z c2
  launch_mdot(c->zv0, 0, 0, 1, c2, P.d, nullptr, P.d, 1, W.part, W.scal2 + 3, nullptr, s);
  launch_axpy_shared(w, P.k, c->v0hat, W.scal2 + 3, 1.0, w, P.k, 1, s);  // w -= v0hat (a^T c2)
}
// c2 = (Z^T A Z)^{-1} cin exactly: Z^T A Z = C^T + a a^T with a = Z^T v0hat.  From the
// coarse solve's G^T = (C^T)^+ (C^T)^{-1} for nonsingular C):
//   singular C (a = gamma tau_hat, tau_hat spanning the right null space of C and u_C
//     the left one): y = G^T c + beta u_C, beta = (tau_hat^T c / (gamma^2 |tau_hat|^2)
//     - tau_hat^T G^T c) / (tau_hat^T u_C);
//   nonsingular C (Sherman-Morrison): y = G^T c - G^T a (a^T G^T c) / (1 + a^T G^T a);
// i.e. c2 = G^T c + p (q1^T c + q2^T G^T c) with the d-vectors p, q1, q2 set up once.
void rank1_coarse(smpm_ctx* c, const double* cin, double* c2, hipStream_t s) {
  const DevPlan& P = c->dp;
  Workspace& W = c->ws;
  launch_coarse(P, cin, c2, 1, true, nullptr, s);
  launch_mdot(c->r1_q1, 0, 0, 1, cin, P.d, nullptr, P.d, 1, W.part, W.scal2 + 1, nullptr, s);
  launch_mdot(c->r1_q2, 0, 0, 1, c2, P.d, nullptr, P.d, 1, W.part, W.scal2 + 2, nullptr, s);
  launch_axpy_shared(c2, P.d, c->r1_p, W.scal2 + 1, -1.0, c2, P.d, 1, s);
  launch_axpy_shared(c2, P.d, c->r1_p, W.scal2 + 2, -1.0, c2, P.d, 1, s);
}

// t = A z
void rank1_apply(smpm_ctx* c, const double* z, double* t, hipStream_t s) {
  const DevPlan& P = c->dp;
  Workspace& W = c->ws;
  launch_schur(P, z, t, 1, true, nullptr, s);
  launch_mdot(c->v0hat, 0, 0, 1, z, P.k, nullptr, P.k, 1, W.part, W.scal2, nullptr, s);
  launch_axpy_shared(t, P.k, c->v0hat, W.scal2, -1.0, t, P.k, 1, s);
}

// w = op(v) for the chosen operator; transpose selects the adjoint pieces.  sprec,
// mprec: precision of the Schur and block-Jacobi operators of OP_S, OP_SM, OP_PSM.
void apply_op(smpm_ctx* c, int kind, bool tr, const double* v, double* w, int nrhs, const int* act,
              hipStream_t s, int sprec = PREC_F64, int mprec = PREC_F64) {
  const DevPlan& P = c->dp;
  Workspace& W = c->ws;
  if (kind == OP_S) {
    launch_schur_ex(P, v, w, nrhs, tr, act, nullptr, s, sprec);
    return;
  }
  if (kind != OP_RANK1 || c->precond_regular) launch_precond(P, v, W.z, nrhs, tr, act, s, mprec);
  if (kind == OP_SM) {
    launch_schur_ex(P, W.z, w, nrhs, tr, act, nullptr, s, sprec);
    return;
  }
  if (kind == OP_RANK1) {
    // (S^T + v0hat v0hat^T) M^{-T} v: nonsingular, its inverse transpose maps v0hat to u_S.
    // On a two-element grid M = S is singular and the operator runs unpreconditioned.
    const double* zin = c->precond_regular ? W.z : v;
    launch_schur(P, zin, w, nrhs, true, act, s);
    launch_mdot(c->v0hat, 0, 0, 1, zin, P.k, nullptr, P.k, nrhs, W.part, W.scal2, act, s);
    launch_axpy_shared(w, P.k, c->v0hat, W.scal2, -1.0, w, P.k, nrhs, s);
    return;
  }
  if (kind == OP_RANK1_DEFL) {
    // P_A A M^{-T} v (one column): t = A z, c2 = G^T Z^T t, w = t - A Z c2
    rank1_apply(c, W.z, W.t, s);
    launch_iface_sum(P, W.t, W.c, 1, nullptr, s);
    rank1_coarse(c, W.c, W.c2, s);
    rank1_coarse_term(c, W.t, W.c2, w, s);
    return;
  }
  launch_schur_ex(P, W.z, W.t, nrhs, tr, act, nullptr, s, sprec);
  launch_iface_sum(P, W.t, W.c, nrhs, act, s);
  launch_coarse(P, W.c, W.c2, nrhs, tr, act, s);
  launch_prolong(P, W.t, W.c2, w, nrhs, tr ? 2 : 1, -1.0, act, s);
}

// Right-preconditioned GMRES from x0 = 0 (Algorithm 3 step 4 and 5-8 for OP_PSM):
// Arnoldi with classical Gram-Schmidt applied twice, Givens rotations, per-column
// stopping |g_{j+1}| <= tol * beta (beta the initial residual, or ref if positive).  b, x: k x nrhs.  Returns iterations (max over
// columns) or a negative status.
int gmres(smpm_ctx* c, int kind, bool tr, const double* b, double* x, int nrhs, double tol, int maxit,
          std::vector<int>& iters, hipStream_t s, double ref = 0.0) {
  const DevPlan& P = c->dp;
  Workspace& W = c->ws;
  const int64_t k = P.k;
  const int ldh = W.maxit + 1;
  // Krylov basis V[j][col][0..k): the j-th vectors of all columns are contiguous so the
  // operator kernels see an ordinary column-blocked block of nrhs k-vectors
  const int64_t vvs = (int64_t)k * nrhs;  // stride between basis vectors
  iters.assign(nrhs, 0);
  std::vector<int> act(nrhs, 1);
  HIPCHK(hipMemcpyAsync(W.active, act.data(), nrhs * sizeof(int), hipMemcpyHostToDevice, s));
  HIPCHK(hipMemsetAsync(W.H, 0, sizeof(double) * (size_t)ldh * W.maxit * nrhs, s));
  HIPCHK(hipMemsetAsync(W.g, 0, sizeof(double) * (size_t)ldh * nrhs, s));
  // r0 = P b (deflated) or b
  double* r0 = W.w;
  if (kind == OP_PSM) {
    launch_iface_sum(P, b, W.c, nrhs, nullptr, s);
    launch_coarse(P, W.c, W.c2, nrhs, tr, nullptr, s);
    launch_prolong(P, b, W.c2, r0, nrhs, tr ? 2 : 1, -1.0, nullptr, s);
  } else if (kind == OP_RANK1_DEFL) {
    launch_iface_sum(P, b, W.c, 1, nullptr, s);
    rank1_coarse(c, W.c, W.c2, s);
    rank1_coarse_term(c, b, W.c2, r0, s);
  } else {
    HIPCHK(hipMemcpyAsync(r0, b, sizeof(double) * k * nrhs, hipMemcpyDeviceToDevice, s));
  }
  launch_mdot(r0, 0, k, 1, r0, k, nullptr, k, nrhs, W.part, W.scal, nullptr, s);
  std::vector<double> beta2(nrhs);
  HIPCHK(hipMemcpyAsync(beta2.data(), W.scal, nrhs * sizeof(double), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  std::vector<double> beta(nrhs), gi(nrhs * (size_t)ldh, 0.0);
  for (int col = 0; col < nrhs; ++col) {
    beta[col] = std::sqrt(beta2[col]);
    if (!(beta[col] > 0.0)) act[col] = 0;
  }
  for (int col = 0; col < nrhs; ++col) gi[(size_t)col * ldh] = beta[col];
  HIPCHK(hipMemcpyAsync(W.g, gi.data(), gi.size() * sizeof(double), hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(W.active, act.data(), nrhs * sizeof(int), hipMemcpyHostToDevice, s));
  launch_scale_inv(r0, k, W.scal, true, W.V, k, k, nrhs, nullptr, s);
  int jmax = 0;
  std::vector<double> res(nrhs);
  int nact = 0;
  for (int col = 0; col < nrhs; ++col) nact += act[col];
  for (int j = 0; j < maxit && nact > 0; ++j) {
    double* vj = W.V + (int64_t)j * vvs;
    apply_op(c, kind, tr, vj, W.w, nrhs, W.active, s);
    // CGS2: h1 = V^T w; w -= V h1; h2 = V^T w; w -= V h2
    launch_mdot(W.V, vvs, k, j + 1, W.w, k, nullptr, k, nrhs, W.part, W.h1, W.active, s);
    launch_mupdate(W.w, k, W.V, vvs, k, j + 1, W.h1, 1.0, k, nrhs, W.active, s);
    launch_mdot(W.V, vvs, k, j + 1, W.w, k, nullptr, k, nrhs, W.part, W.h2, W.active, s);
    launch_mupdate(W.w, k, W.V, vvs, k, j + 1, W.h2, 1.0, k, nrhs, W.active, s);
    launch_add(W.h1, W.h2, 1.0, W.h1, (int64_t)(j + 1) * nrhs, 1, s);
    launch_mdot(W.w, 0, k, 1, W.w, k, nullptr, k, nrhs, W.part, W.scal, W.active, s);
    launch_givens(W.H, ldh, W.cs, W.sn, W.g, W.h1, W.scal, j, nrhs, W.res, W.active, s);
    launch_scale_inv(W.w, k, W.scal, true, W.V + (int64_t)(j + 1) * vvs, k, k, nrhs, W.active, s);
    HIPCHK(hipMemcpyAsync(res.data(), W.res, nrhs * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    bool changed = false;
    for (int col = 0; col < nrhs; ++col) {
      if (!act[col]) continue;
      iters[col] = j + 1;
      if (res[col] <= tol * (ref > 0.0 ? ref : beta[col]) || !std::isfinite(res[col]) || j + 1 == maxit) {
        act[col] = 0;
        --nact;
        changed = true;
      }
    }
    jmax = j + 1;
    if (changed) HIPCHK(hipMemcpyAsync(W.active, act.data(), nrhs * sizeof(int), hipMemcpyHostToDevice, s));
  }
  // y = H^{-1} g, x1 = V y
  HIPCHK(hipMemcpyAsync(W.jcount, iters.data(), nrhs * sizeof(int), hipMemcpyHostToDevice, s));
  launch_lsq(W.H, ldh, W.g, W.jcount, W.y, nrhs, s);
  HIPCHK(hipMemsetAsync(x, 0, sizeof(double) * k * nrhs, s));
  // the coefficient array of column col starts at y + col*maxit; mupdate reads coef + col*nvec
  for (int col = 0; col < nrhs; ++col)
    if (iters[col] > 0)
      launch_mupdate(x + (int64_t)col * k, k, W.V + (int64_t)col * k, vvs, 0, iters[col],
                     W.y + (int64_t)col * W.maxit, -1.0, k, 1, nullptr, s);
  return jmax;
}

// Arnoldi steps per replayed chunk (and per progress report to the host)
constexpr int kChunkIters = 8;

GmState gm_state(smpm_ctx* c, int nrhs, int maxit) {
  Workspace& W = c->ws;
  GmState S;
  S.V = W.V;
  S.vvs = c->plan.k * nrhs;
  S.w = W.w;
  S.z = W.z;
  S.t = W.t;
  S.c = W.c;
  S.sides = W.sides;
  S.c2 = W.c2;
  S.part1 = W.part1;
  S.part2 = W.part2;
  S.h1 = W.h1;
  S.h2 = W.h2;
  S.dw = W.dw;
  S.Hu = W.Hu;
  S.H = W.H;
  S.cs = W.cs;
  S.sn = W.sn;
  S.g = W.g;
  S.y = W.y;
  S.tolb = W.tolb;
  S.res = W.res;
  S.active = W.active;
  S.iters = W.iters;
  S.ldv = W.maxit + 1;
  S.maxit = maxit;
  S.nch = W.nch;
  S.rows = W.rows;
  S.tolv = W.tolv;
  S.jdev = W.jdev;
  // redundant per-block reductions cost (blocks x chunks x vectors) loads; past about
  // a thousand blocks per kernel they are done once per column by small kernels
  S.prereduce = (int64_t)S.nch * nrhs > 1024 ? 1 : 0;
  if (c->prereduce_choice[schur_nc_class(nrhs)] >= 0) S.prereduce = c->prereduce_choice[schur_nc_class(nrhs)];
  if (const char* e = std::getenv("SMPM_PREREDUCE")) S.prereduce = e[0] == '1' ? 1 : e[0] == '0' ? 0 : S.prereduce;
  S.stream = -1;  // test hook: SMPM_STREAM_BASIS=1 / 0 forces one kind of basis load
  if (const char* e = std::getenv("SMPM_STREAM_BASIS")) S.stream = e[0] == '1' ? 1 : e[0] == '0' ? 0 : -1;
  S.bref2 = W.scal2 + 2 * nrhs;
  S.hflag = W.pinned;
  S.hratio = W.hres;
  S.hseq = W.hseq;
  S.pub_stride = W.nrhs;
  S.pub_every = kChunkIters;
  S.basis32 = 0;
  return S;
}

constexpr size_t kMaxGraphs = 32;  // executable graphs kept per context (oldest dropped)
// The executable graph of kChunkIters Arnoldi steps for this solve shape (its last
// step reports the columns' progress to the host; captured on first use on the
// context's capture stream; nothing runs during the capture).

int chunk_graph(smpm_ctx* c, const GmState& S, int nrhs, int kind, bool tr, int sprec, int mprec,
                hipGraphExec_t* out) {
  const int rule = S.bref2 ? 0 : 1;
  for (const auto& g : c->graphs)
    if (g.phase == 0 && g.nrhs == nrhs && g.kind == kind && g.tr == (int)tr && g.sprec == sprec &&
        g.mprec == mprec && g.maxit == S.maxit && g.prereduce == S.prereduce && g.stream == S.stream &&
        g.rule == rule) {
      *out = g.exec;
      return SMPM_OK;
    }
  if (!c->cap_stream) HIPCHK(hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
  hipGraph_t graph = nullptr;
  HIPCHK(hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
  for (int q = 0; q < kChunkIters; ++q) gm_step(c->dp, S, nrhs, q & 1, kind, tr, c->cap_stream, sprec, mprec);
  const hipError_t e1 = hipStreamEndCapture(c->cap_stream, &graph);
  if (e1 != hipSuccess || !graph) return fail(SMPM_EHIP, "hipStreamEndCapture failed");
  hipGraphExec_t exec = nullptr;
  const hipError_t e2 = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (e2 != hipSuccess) return fail(SMPM_EHIP, "hipGraphInstantiate failed");
  if (c->graphs.size() >= kMaxGraphs) {
    (void)hipGraphExecDestroy(c->graphs.front().exec);
    c->graphs.erase(c->graphs.begin());
  }
  c->graphs.push_back({nrhs, kind, (int)tr, sprec, mprec, S.maxit, S.prereduce, S.stream, rule, 0, 0, exec});
  *out = exec;
  return SMPM_OK;
}

// A solve phase (a sequence of kernel launches with no host work in between, on fixed
// workspace pointers) replayed from a graph captured on first use for its key, or run
// directly when graphs are off or the capture fails.
template <typename Body>
int run_phase(smpm_ctx* c, bool use_graph, int phase, const GmState& S, int nrhs, int kind, bool tr, int sprec,
              int mprec, double tol, hipStream_t s, Body&& body) {
  if (!use_graph) {
    body(s);
    HIPCHK(hipGetLastError());
    return SMPM_OK;
  }
  uint64_t tb = 0;
  std::memcpy(&tb, &tol, sizeof tb);
  const int rule = S.bref2 ? 0 : 1;
  for (const auto& g : c->graphs)
    if (g.phase == phase && g.nrhs == nrhs && g.kind == kind && g.tr == (int)tr && g.sprec == sprec &&
        g.mprec == mprec && g.maxit == S.maxit && g.prereduce == S.prereduce && g.stream == S.stream &&
        g.rule == rule && g.tolbits == tb) {
      HIPCHK(hipGraphLaunch(g.exec, s));
      return SMPM_OK;
    }
  if (!c->cap_stream) HIPCHK(hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
  hipGraph_t graph = nullptr;
  HIPCHK(hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
  body(c->cap_stream);
  const hipError_t e1 = hipStreamEndCapture(c->cap_stream, &graph);
  if (e1 != hipSuccess || !graph) return fail(SMPM_EHIP, "hipStreamEndCapture failed (solve phase)");
  hipGraphExec_t exec = nullptr;
  const hipError_t e2 = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (e2 != hipSuccess) return fail(SMPM_EHIP, "hipGraphInstantiate failed (solve phase)");
  if (c->graphs.size() >= kMaxGraphs) {
    (void)hipGraphExecDestroy(c->graphs.front().exec);
    c->graphs.erase(c->graphs.begin());
  }
  c->graphs.push_back({nrhs, kind, (int)tr, sprec, mprec, S.maxit, S.prereduce, S.stream, rule, phase, tb, exec});
  HIPCHK(hipGraphLaunch(exec, s));
  return SMPM_OK;
}

// GMRES prologue for right-hand side b: the stopping reference |b|^2, the initial
// residual r0 = P b (kind 3) or b into W.w, and gm_start (V_0, flags, tolerance).
// (norm_done: the caller already formed |b|^2 there, by the same reduction; sides_done:
// and the per-side sums of b in W.sides, for the dense coarse solve.)
void gm_prologue(smpm_ctx* c, const GmState& S, int kind, bool tr, const double* b, int nrhs, double tol,
                 hipStream_t s, bool norm_done = false, bool sides_done = false) {
  const DevPlan& P = c->dp;
  Workspace& W = c->ws;
  if (!norm_done) launch_mdot(b, 0, P.k, 1, b, P.k, nullptr, P.k, nrhs, W.part, W.scal2 + 2 * nrhs, nullptr, s);
  if (kind == 3) {
    if (sides_done) {
      launch_coarse_sides(P, W.sides, W.c2, nrhs, tr, nullptr, s);  // Z^T b = the interfaces' side sums
    } else {
      launch_iface_sum(P, b, W.c, nrhs, nullptr, s);
      launch_coarse(P, W.c, W.c2, nrhs, tr, nullptr, s);
    }
    gm_start_deflated(P, S, nrhs, b, W.c2, tr, tol, s);  // r0 = P b into w and V_0
  } else {
    launch_copy(b, W.w, P.k * nrhs, s);
    gm_start(P, S, nrhs, tol, s);
  }
}

// GMRES epilogue: the least-squares solution and x1 = V y, and the counts and column 0's
// history (rotated right-hand side, cosines, threshold) into pinned memory, read after
// the caller's synchronization (with defer, the publication is added to *defer for the
// caller to launch with its own).
void gm_epilogue(smpm_ctx* c, const GmState& S, int kind, bool tr, double* x1, int nrhs, hipStream_t s,
                 PublishSet* defer = nullptr) {
  const DevPlan& P = c->dp;
  Workspace& W = c->ws;
  // every column has retired in a Givens step by the time the iterations end (the
  // retirement test includes j >= maxit), so the Hessenberg columns are complete
  gm_finish(P, S, nrhs, x1, s);
  PublishSet ps = {};
  ps.src[0] = W.g;
  ps.dst[0] = W.hhist;
  ps.n[0] = S.maxit + 1;
  ps.src[1] = W.cs;
  ps.dst[1] = W.hhist_cs;
  ps.n[1] = S.maxit + 1;
  ps.src[2] = W.tolb;
  ps.dst[2] = W.hhist_tolb;
  ps.n[2] = 1;
  ps.isrc = W.iters;
  ps.idst = W.hiters;
  ps.in = nrhs;
  if (defer)
    *defer = ps;
  else
    launch_publish_set(ps, s);
}

// Reads what gm_epilogue published (after a synchronization).
int gm_collect(smpm_ctx* c, int nrhs, int maxit, double tol, std::vector<int>& iters) {
  Workspace& W = c->ws;
  iters.assign(W.hiters, W.hiters + nrhs);
  W.hist_len = std::min(iters[0], maxit) + 1;
  W.hist_tol = tol;
  int jmax = 0;
  for (int v : iters) jmax = std::max(jmax, v);
  return jmax;
}

// The Arnoldi iterations after gm_prologue: chunks of kChunkIters steps; the last step
// of each reports the activity flags and residual ratios (estimate / threshold) into
// pinned slot chunk % 2, then the chunk count, which the host polls.  The host keeps
// one chunk queued ahead of the one it waits for (so a slot is never rewritten while
// it is read), except when the observed convergence rate says the queued chunk will
// finish the solve: then it waits for that chunk instead of queueing steps that would
// find every column retired.  Steps past maxit (the last chunk's tail) do nothing.
//
// With post != nullptr the caller's post-processing (which must leave the Arnoldi
// state alone) is queued right behind the chunk predicted to finish, so it runs
// without waiting for the host; *post_done says whether the queued copy followed the
// chunk that did finish.  If the prediction fails, the next chunk is queued after it
// and the caller runs the post-processing again once the loop ends (the early copy
// only wrote outputs the later one rewrites).  Returns once every column has retired
// (queued work may still be running).
int gm_loop(smpm_ctx* c, const GmState& S, int kind, bool tr, int nrhs, int maxit, hipStream_t s, int sprec,
            int mprec, bool use_graph, const std::function<int()>* post = nullptr, bool* post_done = nullptr) {
  const DevPlan& P = c->dp;
  Workspace& W = c->ws;
  if (post_done) *post_done = false;
  hipGraphExec_t exec = nullptr;
  if (use_graph) {
    const int rc = chunk_graph(c, S, nrhs, kind, tr, sprec, mprec, &exec);
    if (rc) return rc;
  }
  // step j finishes Hessenberg column j - 2, so maxit columns take maxit + 2 steps
  const int nchunks = (maxit + 2 + kChunkIters - 1) / kChunkIters;
  bool spec_live = false;  // a speculative post-processing is queued behind the last chunk
  int spec_count = 0;
  auto launch_chunk = [&](int ch) -> int {
    spec_live = false;  // steps queued behind it: it ran too early
    (void)ch;
    if (exec) {
      HIPCHK(hipGraphLaunch(exec, s));
    } else {
      for (int q = 0; q < kChunkIters; ++q) gm_step(P, S, nrhs, q & 1, kind, tr, s, sprec, mprec);
    }
    return SMPM_OK;
  };
  // the device's report of chunk ci (its count in pinned memory, written after the
  // flags with a system-scope fence); the stream is polled now and then so that an
  // error, or work that ended without the report, returns instead of waiting forever
  auto wait_chunk = [&](int ci) -> int {
    volatile int* seq = W.hseq;
    for (long spins = 1; *seq < ci + 1; ++spins) {
      if (spins % 2048 == 0) {
        const hipError_t e = hipStreamQuery(s);
        if (e == hipSuccess && *seq < ci + 1) return fail(SMPM_EHIP, "a chunk of Arnoldi steps ended unreported");
        if (e != hipSuccess && e != hipErrorNotReady) return fail(SMPM_EHIP, hipGetErrorString(e));
      }
    }
    std::atomic_thread_fence(std::memory_order_acquire);
    return SMPM_OK;
  };
  *W.hseq = 0;  // the stream is idle: every caller synchronizes before and after a loop
  std::vector<double> prev_ratio(nrhs, -1.0);
  int launched = 0;
  bool finishing = false;  // the chunk in flight is predicted to complete every column
  int rc0 = launch_chunk(launched++);
  if (rc0) return rc0;
  for (int ci = 0; ci < nchunks; ++ci) {
    if (!finishing && launched == ci + 1 && launched < nchunks) {
      rc0 = launch_chunk(launched++);
      if (rc0) return rc0;
    }
    rc0 = wait_chunk(ci);
    if (rc0) return rc0;
    const int* fl = W.pinned + (ci & 1) * W.nrhs;
    const double* ra = W.hres + (ci & 1) * W.nrhs;
    bool any = false;
    double steps_left = 0.0;
    for (int i = 0; i < nrhs; ++i) {
      if (!fl[i]) continue;
      any = true;
      const double r = ra[i], rp = prev_ratio[i];
      // steps to reach ratio 1 at the rate seen over the last chunk (unknown: far)
      double left = 1e30;
      if (rp > 0.0 && r > 0.0 && r < rp) left = kChunkIters * std::log(r) / std::log(rp / r);
      steps_left = std::max(steps_left, left);
      prev_ratio[i] = r;
    }
    if (!any || ci + 1 >= nchunks) {
      // the queued copy is valid if nothing was queued after this chunk but it
      if (post_done) *post_done = spec_live && launched == ci + 1;
      break;
    }
    // the chunk queued after ci covers the next kChunkIters steps
    finishing = steps_left <= kChunkIters;
    if (launched == ci + 1) {
      rc0 = launch_chunk(launched++);
      if (rc0) return rc0;
    }
    if (post && finishing && !spec_live && spec_count < 2 && launched == ci + 2) {
      rc0 = (*post)();
      if (rc0) return rc0;
      spec_live = true;
      ++spec_count;
    }
  }
  return SMPM_OK;
}

// Device-resident GMRES from x0 = 0 on S (kind 1), S M^{-1} (2) or P S M^{-1} (3):
// prologue, iterations and epilogue, then a synchronization.  Returns the largest
// iteration count over the columns.
int gmres_dev(smpm_ctx* c, int kind, bool tr, const double* b, double* x, int nrhs, double tol, int maxit,
              std::vector<int>& iters, hipStream_t s, int sprec = PREC_F64, int mprec = PREC_F64,
              bool use_graph = true, int rule = 0) {
  Workspace& W = c->ws;
  GmState S = gm_state(c, nrhs, maxit);
  // stopping reference: |b| (the Schur right-hand side, the quantity the FP64 true
  // residual is accepted against), or with rule 1 the initial GMRES residual (the
  // step-0 kernel takes it when bref2 is null)
  S.bref2 = rule == 1 ? nullptr : W.scal2 + 2 * nrhs;
  // an inner solve with low-precision operators only has to reach its loose inner
  // tolerance: its basis is stored in FP32 (half the basis traffic), arithmetic FP64
  S.basis32 = sprec != PREC_F64 && c->mixed_basis32 ? 1 : 0;
  gm_prologue(c, S, kind, tr, b, nrhs, tol, s);
  int rc = gm_loop(c, S, kind, tr, nrhs, maxit, s, sprec, mprec, use_graph);
  if (rc) return rc;
  gm_epilogue(c, S, kind, tr, x, nrhs, s);
  HIPCHK(hipStreamSynchronize(s));
  return gm_collect(c, nrhs, maxit, tol, iters);
}

// x from the GMRES solution x1 of the preconditioned (and deflated) system, with the
// operators (and precisions) of the GMRES operator, so that x = M^{-1} x1 reproduces
// the preconditioned iterate exactly (Algorithm 3 steps 5-8).
void recover_x(smpm_ctx* c, int kind, bool tr, const double* bhat, const double* x1, double* x, int nrhs, int sprec,
               int mprec, hipStream_t s) {
  const DevPlan& P = c->dp;
  Workspace& W = c->ws;
  if (kind == OP_S) {
    launch_copy(x1, x, P.k * nrhs, s);
  } else if (kind == OP_SM) {
    launch_precond(P, x1, x, nrhs, tr, nullptr, s, mprec);
  } else {
    // x = z + Z G Z^T (b_hat - S z), z = M^{-1} x1
    launch_precond(P, x1, W.z, nrhs, tr, nullptr, s, mprec);
    launch_schur_ex(P, W.z, W.t, nrhs, tr, nullptr, nullptr, s, sprec);
    launch_iface_sum_diff(P, bhat, W.t, -1.0, W.c, nrhs, s);  // Z^T (b_hat - S z)
    launch_coarse(P, W.c, W.c2, nrhs, tr, nullptr, s);
    launch_prolong(P, W.z, W.c2, x, nrhs, 0, 1.0, nullptr, s);
  }
}

// |b - S x|^2 and |b|^2 per column into pinned hout[0..nrhs) and hout[nrhs..2 nrhs);
// b2, if given, already holds |b|^2 (the same reduction of the same b); extra, if
// given, nrhs more values published into hout[2 nrhs..3 nrhs); more, if given, the
// caller's other publications, launched together with these.
void true_residual_enqueue(smpm_ctx* c, bool tr, const double* b, const double* x, int nrhs, hipStream_t s,
                           const double* b2 = nullptr, const double* extra = nullptr,
                           const PublishSet* more = nullptr) {
  const DevPlan& P = c->dp;
  Workspace& W = c->ws;
  launch_schur(P, x, W.t, nrhs, tr, nullptr, s);
  launch_norm2_diff(b, W.t, -1.0, P.k, nrhs, W.part, W.scal, s);  // |b - S x|^2
  if (!b2) {
    launch_mdot(b, 0, P.k, 1, b, P.k, nullptr, P.k, nrhs, W.part, W.scal2, nullptr, s);
    b2 = W.scal2;
  }
  PublishSet ps = {};
  if (more) {
    // the caller's entries go after these three
    for (int q = 0; q < 3; ++q) {
      ps.src[4 + q] = more->src[q];
      ps.dst[4 + q] = more->dst[q];
      ps.n[4 + q] = more->n[q];
    }
    ps.isrc = more->isrc;
    ps.idst = more->idst;
    ps.in = more->in;
  }
  ps.src[0] = W.scal;
  ps.dst[0] = W.hout;
  ps.n[0] = nrhs;
  ps.src[1] = b2;
  ps.dst[1] = W.hout + nrhs;
  ps.n[1] = nrhs;
  if (extra) {
    ps.src[2] = extra;
    ps.dst[2] = W.hout + 2 * nrhs;
    ps.n[2] = nrhs;
  }
  launch_publish_set(ps, s);
}

void true_residual_read(smpm_ctx* c, int nrhs, std::vector<double>& out) {
  Workspace& W = c->ws;
  const double* a = W.hout;
  const double* bb = W.hout + nrhs;
  out.resize(nrhs);
  for (int i = 0; i < nrhs; ++i) out[i] = bb[i] > 0 ? std::sqrt(a[i] / bb[i]) : std::sqrt(a[i]);
}

int solve_schur(smpm_ctx* c, int kind, bool tr, const double* bhat, double* x, int nrhs, double tol, int maxit,
                std::vector<int>& iters, hipStream_t s, int sprec = PREC_F64, int mprec = PREC_F64,
                bool use_graph = true, int rule = 0) {
  Workspace& W = c->ws;
  double* x1 = W.x;  // note: x may not alias W.x
  int rc = gmres_dev(c, kind, tr, bhat, x1, nrhs, tol, maxit, iters, s, sprec, mprec, use_graph, rule);
  if (rc < 0) return rc;
  recover_x(c, kind, tr, bhat, x1, x, nrhs, sprec, mprec, s);
  return rc;
}

// ||b - S x|| / ||b|| per column (FP64), returned on the host.
int true_residual(smpm_ctx* c, bool tr, const double* b, const double* x, int nrhs, std::vector<double>& out,
                  hipStream_t s) {
  true_residual_enqueue(c, tr, b, x, nrhs, s);
  HIPCHK(hipStreamSynchronize(s));
  true_residual_read(c, nrhs, out);
  return SMPM_OK;
}

// Rank-deflation threshold of block GMRES: a block column whose part orthogonal to
// the block's earlier columns is at most this fraction of its norm adds no vector
// (the Gram matrix resolves relative parts down to about 1e-7 in FP64).
constexpr double kBlockDrop = 1e-6;

// Cholesky QR applied twice to the m columns at wb (m <= kBgMaxCols), with rank
// deflation in the first pass: the kept vectors go to dst (columns past the kept
// count are zero), the count to B.cnt[1] (B.cnt[0]: the first pass), and R (kept x m,
// ld kBgMaxCols, wb = dst R) to B.R2.  tmp: scratch of m vectors.
template <typename VT>
void block_cholqr(smpm_ctx* c, const double* wb, int m, VT* dst, double* tmp, hipStream_t s) {
  BlockWs& B = c->bws;
  const int64_t k = c->dp.k;
  launch_bg_dot(wb, m, wb, m, k, B.part, B.gram, m, 0.0, s);
  launch_bg_chol(B.gram, m, kBlockDrop, nullptr, nullptr, B.cnt, B.T1, B.R1, s);
  launch_bg_update(wb, m, B.T1, 1, m, 1.0, (const double*)nullptr, 0.0, tmp, m, k, s);
  launch_bg_dot(tmp, m, tmp, m, k, B.part, B.gram, m, 0.0, s);
  launch_bg_chol(B.gram, m, 0.0, B.cnt, B.R1, B.cnt + 1, B.T2, B.R2, s);
  launch_bg_update(tmp, m, B.T2, 1, m, 1.0, (const VT*)nullptr, 0.0, dst, m, k, s);
}

// Block GMRES (FP64) from x1 = 0 for op(x1) = b, all nrhs <= kBgMaxCols columns in one
// block Krylov space, op by kind as in gmres (OP_S, OP_SM, OP_PSM; P b is the start
// for OP_PSM).  Each block step: W = op(V_j); block classical Gram-Schmidt against the
// whole basis, applied twice (the sums and updates on matrix cores); Cholesky QR of
// W twice, with rank deflation, gives V_{j+1} and the block's subdiagonal part; the
// least-squares problem is updated by Householder reflections.  x1 = V Y at the end.
// Stops when every column's least-squares residual is <= tol times its reference
// (ref2: squared references on the device; null: the start block's column norms),
// when a block adds no vector, or after maxit block steps.  res0 (host, optional)
// receives column 0's residual / reference after each step (the start first).
// Returns the block steps taken, or a negative status.
int block_gmres(smpm_ctx* c, int kind, bool tr, const double* b, double* x1, int nrhs, double tol, int maxit,
                const double* ref2, hipStream_t s, std::vector<double>* res0 = nullptr, int sprec = PREC_F64,
                int mprec = PREC_F64) {
  const DevPlan& P = c->dp;
  Workspace& W = c->ws;
  BlockWs& B = c->bws;
  const int64_t k = P.k;
  double* r0 = W.w;
  if (kind == OP_PSM) {
    launch_iface_sum(P, b, W.c, nrhs, nullptr, s);
    launch_coarse(P, W.c, W.c2, nrhs, tr, nullptr, s);
    launch_prolong(P, b, W.c2, r0, nrhs, tr ? 2 : 1, -1.0, nullptr, s);
  } else {
    launch_copy(b, r0, k * nrhs, s);
  }
  if (!ref2) {
    launch_mdot(r0, 0, k, 1, r0, k, nullptr, k, nrhs, W.part, W.scal, nullptr, s);
    ref2 = W.scal;
  }
  HIPCHK(hipMemcpyAsync(B.href, ref2, nrhs * sizeof(double), hipMemcpyDeviceToHost, s));
  BgLsq L{B.H, B.ldH, B.refl, B.rbeta, B.G, nrhs, B.res};
  // an inner solve with low-precision operators stores its basis in FP32 (the
  // products stay FP64), as the batched inner solves do
  const bool b32 = sprec != PREC_F64 && c->mixed_basis32;
  float* V32 = reinterpret_cast<float*>(W.V);
  if (b32)
    block_cholqr(c, r0, nrhs, V32, W.t, s);
  else
    block_cholqr(c, r0, nrhs, W.V, W.t, s);
  launch_bg_lsq_start(L, B.R2, B.cnt + 1, s);
  // |R_0| per column = the start block's column norms (the reflections keep them)
  launch_bg_dot(r0, nrhs, r0, nrhs, k, B.part, B.gram, nrhs, 0.0, s);
  HIPCHK(hipMemcpyAsync(B.hcnt, B.cnt, 2 * sizeof(int), hipMemcpyDeviceToHost, s));
  std::vector<double> g0(nrhs * nrhs);
  HIPCHK(hipMemcpyAsync(g0.data(), B.gram, g0.size() * sizeof(double), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  std::vector<double> ref(nrhs);
  for (int i = 0; i < nrhs; ++i) ref[i] = std::sqrt(std::max(B.href[i], 0.0));
  if (res0) res0->assign(1, ref[0] > 0 ? std::sqrt(std::max(g0[0], 0.0)) / ref[0] : 0.0);
  int nv = B.hcnt[1];
  if (B.hcnt[1] != B.hcnt[0]) return fail(SMPM_EHIP, "block orthonormalization lost a vector in its second pass");
  int n0 = 0, steps = 0;
  const int ldh = B.ldH;
  for (int j = 0; j < maxit && nv > n0; ++j) {
    const int r = nv - n0;
    // the updates read the sums transposed (a row of 32 per basis vector); x1's buffer
    // holds the widened block of an FP32 basis until x1 is formed
    if (b32) {
      launch_bg_widen(V32 + (int64_t)n0 * k, x1, (int64_t)r * k, s);
      apply_op(c, kind, tr, x1, W.w, r, nullptr, s, sprec, mprec);
      launch_bg_dot(V32, nv, W.w, r, k, B.part, B.h, ldh, 0.0, s, B.ht);
      launch_bg_update(V32, nv, B.ht, kBgMaxCols, 1, -1.0, W.w, 1.0, W.w, r, k, s);
      launch_bg_dot(V32, nv, W.w, r, k, B.part, B.h2, ldh, 0.0, s, B.ht);
      launch_bg_update(V32, nv, B.ht, kBgMaxCols, 1, -1.0, W.w, 1.0, W.w, r, k, s);
    } else {
      apply_op(c, kind, tr, W.V + (int64_t)n0 * k, W.w, r, nullptr, s, sprec, mprec);
      launch_bg_dot(W.V, nv, W.w, r, k, B.part, B.h, ldh, 0.0, s, B.ht);
      launch_bg_update(W.V, nv, B.ht, kBgMaxCols, 1, -1.0, W.w, 1.0, W.w, r, k, s);
      launch_bg_dot(W.V, nv, W.w, r, k, B.part, B.h2, ldh, 0.0, s, B.ht);
      launch_bg_update(W.V, nv, B.ht, kBgMaxCols, 1, -1.0, W.w, 1.0, W.w, r, k, s);
    }
    launch_add(B.h, B.h2, 1.0, B.h, (int64_t)ldh * r, 1, s);
    if (b32)
      block_cholqr(c, W.w, r, V32 + (int64_t)nv * k, W.t, s);
    else
      block_cholqr(c, W.w, r, W.V + (int64_t)nv * k, W.t, s);
    launch_bg_lsq(L, n0, r, nv, B.h, ldh, B.R2, B.cnt, B.hres, B.hcnt, s);
    HIPCHK(hipStreamSynchronize(s));
    if (B.hcnt[1] != B.hcnt[0]) return fail(SMPM_EHIP, "block orthonormalization lost a vector in its second pass");
    steps = j + 1;
    n0 = nv;
    nv += B.hcnt[1];
    bool done = true, finite = true;
    for (int i = 0; i < nrhs; ++i) {
      if (!std::isfinite(B.hres[i])) finite = false;
      if (!(B.hres[i] <= tol * ref[i])) done = false;
    }
    if (res0) res0->push_back(ref[0] > 0 ? B.hres[0] / ref[0] : 0.0);
    if (done || !finite) break;
  }
  launch_bg_backsolve(L, n0, B.Y, B.cap, s);
  if (n0 > 0 && b32)
    launch_bg_update(V32, n0, B.Y, 1, B.cap, 1.0, (const double*)nullptr, 0.0, x1, nrhs, k, s);
  else if (n0 > 0)
    launch_bg_update(W.V, n0, B.Y, 1, B.cap, 1.0, (const double*)nullptr, 0.0, x1, nrhs, k, s);
  else
    HIPCHK(hipMemsetAsync(x1, 0, sizeof(double) * k * nrhs, s));
  return steps;
}

// block_gmres, then x from its solution (Algorithm 3 steps 5-8 for OP_PSM), with the
// operators in the given precisions (the refinement cycles of mixed precision).
int block_solve_schur(smpm_ctx* c, int kind, bool tr, const double* bhat, double* x, int nrhs, double tol,
                      int maxit, const double* ref2, hipStream_t s, std::vector<double>* res0,
                      int sprec = PREC_F64, int mprec = PREC_F64) {
  Workspace& W = c->ws;
  const int rc = block_gmres(c, kind, tr, bhat, W.x, nrhs, tol, maxit, ref2, s, res0, sprec, mprec);
  if (rc < 0) return rc;
  recover_x(c, kind, tr, bhat, W.x, x, nrhs, sprec, mprec, s);
  return rc;
}

// Upper bound of ||S||_2: sqrt(||S||_1 ||S||_inf), from the class operators (S = I +
// the side fluxes W; row sums over the neighbour's slots, column sums over the four
// receiving sides).
double schur_norm_bound(const Plan& p) {
  const int n = p.n;
  double rmax = 0.0, cmax = 0.0;
  for (size_t J = 0; J < p.classes.size(); ++J) {
    const int ns = p.classes[J].nslots;
    std::vector<double> col(ns, 0.0);
    for (int so = 0; so < 4; ++so) {
      const int64_t wo = p.W_off[J * 4 + so];
      if (wo < 0) continue;
      for (int t = 0; t < n; ++t) {
        double rs = 0.0;
        for (int cc = 0; cc < ns; ++cc) {
          const double a = std::fabs(p.Wr[wo + (size_t)t * ns + cc]);
          rs += a;
          col[cc] += a;
        }
        rmax = std::max(rmax, rs);
      }
    }
    for (double v : col) cmax = std::max(cmax, v);
  }
  return std::sqrt((1.0 + rmax) * (1.0 + cmax));
}

// u_S: (S + v0hat v0hat^T) is nonsingular and its transpose maps u_S to a multiple of
// v0hat, so u_S = normalize((S + v0hat v0hat^T)^{-T} v0hat).  u_L = normalize(A^{-T} B^T u_S)
// up to sign, since u_L^T L = 0 and E^T u_L is parallel to u_S (Sec. 1.4).
// The solve restarts from its residual (y += GMRES(v0hat - (S^T + v0hat v0hat^T) y))
// until ||S^T u_S|| <= kNullTol ||S|| (the norm bound above); SMPM_ESINGULAR otherwise.
constexpr double kNullTol = 1e-12;
constexpr int kNullCycles = 8, kNullMaxit = 600;
int compute_null_vectors(smpm_ctx* c, hipStream_t s) {
  if (c->have_null) return SMPM_OK;
  const Plan& Pl = c->plan;
  const DevPlan& P = c->dp;
  int rc = ensure_ws(c, 1, kNullMaxit);
  if (rc) return rc;
  Workspace& W = c->ws;
  const int64_t k = Pl.k;
  const double snorm = schur_norm_bound(Pl);
  double* y = W.xacc;   // accumulated solution
  double* rv = W.rho;   // right-hand side of the current cycle
  std::vector<int> it;
  HIPCHK(hipMemsetAsync(y, 0, sizeof(double) * k, s));
  HIPCHK(hipMemcpyAsync(rv, c->v0hat, sizeof(double) * k, hipMemcpyDeviceToDevice, s));
  double null_res = HUGE_VAL;
  int total = 0;
  std::vector<double> hy(k);
  // deflated when the grid has a coarse space and a regular preconditioner
  bool defl = Pl.has_coarse && c->precond_regular;
  if (defl && !c->zv0) {
    // a = Z^T v0hat and the exact coarse correction's vectors p, q1, q2 (see rank1_coarse)
    const int64_t d = Pl.d;
    int r2 = dalloc(c->mem, &c->zv0, d);
    r2 |= dalloc(c->mem, &c->r1_p, d);
    r2 |= dalloc(c->mem, &c->r1_q1, d);
    r2 |= dalloc(c->mem, &c->r1_q2, d);
    if (r2) return SMPM_ENOMEM;
    launch_iface_sum(P, c->v0hat, c->zv0, 1, nullptr, s);
    std::vector<double> a(d), pv(d, 0.0), q1(d, 0.0), q2(d, 0.0);
    HIPCHK(hipMemcpyAsync(a.data(), c->zv0, d * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (Pl.coarse_singular && (int64_t)Pl.tau_hat.size() == d && (int64_t)Pl.uC.size() == d) {
      double tt = 0, ta = 0, tu = 0;
      for (int64_t i = 0; i < d; ++i) {
        tt += Pl.tau_hat[i] * Pl.tau_hat[i];
        ta += Pl.tau_hat[i] * a[i];
        tu += Pl.tau_hat[i] * Pl.uC[i];
      }
      const double gam = ta / tt;
      double off = 0, an = 0;
      for (int64_t i = 0; i < d; ++i) {
        off = std::max(off, std::fabs(a[i] - gam * Pl.tau_hat[i]));
        an = std::max(an, std::fabs(a[i]));
      }
      if (off <= 1e-10 * an && std::fabs(tu) > 1e-14 * std::sqrt(tt) && gam != 0.0) {
        for (int64_t i = 0; i < d; ++i) {
          pv[i] = Pl.uC[i];
          q1[i] = Pl.tau_hat[i] / (gam * gam * tt * tu);
          q2[i] = -Pl.tau_hat[i] / tu;
        }
      } else {
        defl = false;  // not the structure the correction assumes: plain rank-one solve
      }
    } else if (!Pl.coarse_singular) {
      HIPCHK(hipMemcpyAsync(c->r1_q1, c->zv0, d * sizeof(double), hipMemcpyDeviceToDevice, s));
      launch_coarse(P, c->r1_q1, c->r1_p, 1, true, nullptr, s);  // p = G^T a
      HIPCHK(hipMemcpyAsync(pv.data(), c->r1_p, d * sizeof(double), hipMemcpyDeviceToHost, s));
      HIPCHK(hipStreamSynchronize(s));
      double ap = 0;
      for (int64_t i = 0; i < d; ++i) ap += a[i] * pv[i];
      for (int64_t i = 0; i < d; ++i) q2[i] = -a[i] / (1.0 + ap);
    } else {
      defl = false;
    }
    HIPCHK(hipMemcpyAsync(c->r1_p, pv.data(), d * sizeof(double), hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(c->r1_q1, q1.data(), d * sizeof(double), hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(c->r1_q2, q2.data(), d * sizeof(double), hipMemcpyHostToDevice, s));
    HIPCHK(hipStreamSynchronize(s));
    c->r1_defl = defl;
  }
  defl = defl && c->r1_defl;
  for (int cyc = 0; cyc < kNullCycles; ++cyc) {
    if (defl) {
      // GMRES on P_A A M^{-T}, stopped at an absolute 1e-13 = 1e-13 |v0hat|: enough for
      // ||S^T u_S|| / ||S|| <= 1e-12 (|y| >= 1, ||S|| >= 1), and above the rounding floor
      // of the deflated operator (~1e-14); delta = Q_A M^{-T} x + Z G^T Z^T rv
      // = z + Z G^T Z^T (rv - A z),  z = M^{-T} x
      int j = gmres(c, OP_RANK1_DEFL, true, rv, W.x, 1, 1e-13, kNullMaxit, it, s, 1.0);
      if (j < 0) return j;
      total += j;
      launch_precond(P, W.x, W.z, 1, true, nullptr, s);
      rank1_apply(c, W.z, W.t, s);
      launch_add(rv, W.t, -1.0, W.w, k, 1, s);
      launch_iface_sum(P, W.w, W.c, 1, nullptr, s);
      rank1_coarse(c, W.c, W.c2, s);
      launch_prolong(P, W.z, W.c2, W.t, 1, 0, 1.0, nullptr, s);  // t = z + Z c2
    } else {
      // GMRES on (S^T + v0hat v0hat^T) M^{-T}, then delta = M^{-T} x
      int j = gmres(c, OP_RANK1, true, rv, W.x, 1, 1e-14, kNullMaxit, it, s);
      if (j < 0) return j;
      total += j;
      if (c->precond_regular)
        launch_precond(P, W.x, W.t, 1, true, nullptr, s);
      else
        HIPCHK(hipMemcpyAsync(W.t, W.x, sizeof(double) * k, hipMemcpyDeviceToDevice, s));
    }
    launch_add(y, W.t, 1.0, y, k, 1, s);
    // rv = v0hat - S^T y - v0hat (v0hat^T y);  ||S^T y|| and ||y|| for the check
    launch_schur(P, y, W.t, 1, true, nullptr, s);
    launch_mdot(c->v0hat, 0, 0, 1, y, k, nullptr, k, 1, W.part, W.scal2, nullptr, s);
    launch_mdot(W.t, 0, k, 1, W.t, k, nullptr, k, 1, W.part, W.scal2 + 1, nullptr, s);
    launch_mdot(y, 0, k, 1, y, k, nullptr, k, 1, W.part, W.scal2 + 2, nullptr, s);
    launch_add(c->v0hat, W.t, -1.0, rv, k, 1, s);
    launch_axpy_shared(rv, k, c->v0hat, W.scal2, 1.0, rv, k, 1, s);
    launch_publish(W.scal2, 3, W.hout, s);
    HIPCHK(hipStreamSynchronize(s));
    const double sty = std::sqrt(W.hout[1]), yn = std::sqrt(W.hout[2]);
    null_res = yn > 0 ? sty / (yn * snorm) : HUGE_VAL;
    if (!std::isfinite(null_res)) break;
    if (null_res <= kNullTol) break;
  }
  c->null_residual = null_res;
  c->null_iterations = total;
  if (!(null_res <= kNullTol)) {
    char buf[160];
    std::snprintf(buf, sizeof buf,
                  "left null vector of S not resolved: ||S^T u_S|| / ||S|| = %.3g after %d GMRES iterations", null_res,
                  total);
    return fail(SMPM_ESINGULAR, buf);
  }
  HIPCHK(hipMemcpyAsync(hy.data(), y, k * sizeof(double), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  double nn = 0, sum = 0;
  for (double v : hy) {
    nn += v * v;
    sum += v;
  }
  nn = std::sqrt(nn);
  if (!(nn > 0) || !std::isfinite(nn)) return fail(SMPM_ESINGULAR, "null vector computation failed");
  const double sg = sum < 0 ? -1.0 : 1.0;
  for (double& v : hy) v *= sg / nn;
  c->h_uS = hy;
  HIPCHK(hipMemcpyAsync(c->uS, hy.data(), Pl.k * sizeof(double), hipMemcpyHostToDevice, s));
  launch_flux_adj(P, c->uS, W.rhs, 1, s);
  std::vector<double> hl(Pl.r);
  HIPCHK(hipMemcpyAsync(hl.data(), W.rhs, Pl.r * sizeof(double), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  nn = 0;
  sum = 0;
  for (double v : hl) {
    nn += v * v;
    sum += v;
  }
  nn = std::sqrt(nn);
  if (!(nn > 0) || !std::isfinite(nn)) return fail(SMPM_ESINGULAR, "null vector computation failed");
  const double sl = sum < 0 ? -1.0 : 1.0;
  for (double& v : hl) v *= sl / nn;
  c->h_uL = hl;
  HIPCHK(hipMemcpyAsync(c->uL, hl.data(), Pl.r * sizeof(double), hipMemcpyHostToDevice, s));
  HIPCHK(hipStreamSynchronize(s));
  c->have_null = true;
  return SMPM_OK;
}

int do_upload(smpm_ctx* c, hipStream_t s) {
  const Plan& p = c->plan;
  DevPlan& d = c->dp;
  d.n = p.n;
  d.n2 = p.n * p.n;
  d.nel = p.nel;
  d.d = (int)p.d;
  d.nblk = p.nblk;
  d.ncls = (int)p.classes.size();
  d.mx = p.mx;
  d.my = p.my;
  d.r = p.r;
  d.k = p.k;
  d.nsides = p.nsides;
  d.nbdry = 2LL * p.n * (p.mx + p.my);
  std::vector<int> nslots, sidecol;
  for (const auto& cl : p.classes) {
    nslots.push_back(cl.nslots);
    for (int s2 = 0; s2 < 4; ++s2) sidecol.push_back(cl.side_col[s2]);
  }
  // column sums of W for S^T Z
  const int n = p.n;
  std::vector<double> wzc((size_t)d.ncls * 4 * 4 * n, 0.0);
  for (int J = 0; J < d.ncls; ++J)
    for (int s2 = 0; s2 < 4; ++s2) {
      const int64_t o = p.W_off[(size_t)J * 4 + s2];
      if (o < 0) continue;
      const int ns = p.classes[J].nslots;
      for (int cc = 0; cc < ns; ++cc) {
        double acc = 0;
        for (int i = 0; i < n; ++i) acc += p.Wr[o + (size_t)i * ns + cc];
        wzc[((size_t)J * 4 + s2) * 4 * n + cc] = acc;
      }
    }
  std::vector<double> GT(p.G.size());
  if (p.coarse_mode == 1)
    for (int64_t i = 0; i < p.d; ++i)
      for (int64_t j = 0; j < p.d; ++j) GT[(size_t)j * p.d + i] = p.G[(size_t)i * p.d + j];
  d.has_coarse = p.has_coarse ? 1 : 0;
  d.coarse_mode = p.coarse_mode;
  {
    const CoarseSub& q = p.sub;
    d.sub_npatch = q.npatch;
    d.sub_nsep = q.nsep;
    d.sub_border = q.border;
    int lmax = 1;
    for (int pp = 0; pp < q.npatch; ++pp)
      lmax = std::max({lmax, q.I_off[pp + 1] - q.I_off[pp], q.B_off[pp + 1] - q.B_off[pp] + q.border});
    d.sub_lds_max = lmax;
    d.cws = nullptr;
    d.cws_stride = 0;
  }
  // boundary data map: south, north, west, east
  std::vector<int> bnode;
  std::vector<double> btau;
  for (int edge = 0; edge < 4; ++edge) {
    const int cnt = edge < 2 ? p.mx : p.my;
    for (int q = 0; q < cnt; ++q)
      for (int t = 0; t < n; ++t) {
        int e, s2;
        if (edge == 0) { e = q; s2 = SS; }
        else if (edge == 1) { e = (p.my - 1) * p.mx + q; s2 = SN; }
        else if (edge == 2) { e = q * p.mx; s2 = SW; }
        else { e = q * p.mx + p.mx - 1; s2 = SE; }
        int l = s2 == SW ? t * n : s2 == SE ? t * n + n - 1 : s2 == SS ? t : (n - 1) * n + t;
        bnode.push_back(e * n * n + l);
        // coefficient of g: the physical side's tau sigma
        btau.push_back(p.side_tau[(size_t)e * 4 + s2] * p.side_sig[(size_t)e * 4 + s2]);
      }
  }
  // per inter-element side, the interfaces and coefficient offsets that the deflation
  // w = t - Z c2 - {S, S^T} Z c2 reads for the side's slots (two 16-byte loads a side)
  std::vector<int> side_fwd((size_t)p.nsides * 8, -1), side_adj((size_t)p.nsides * 8, -1);
  for (int64_t si = 0; si < p.nsides; ++si) {
    const int e = p.side_elem[si], sd = p.side_dir[si];
    const int J = p.nbr[(size_t)e * 4 + sd];
    int* f = &side_fwd[(size_t)si * 8];
    int* a = &side_adj[(size_t)si * 8];
    f[0] = a[0] = p.iface[(size_t)e * 4 + sd];
    for (int s2 = 0; s2 < 4; ++s2) {
      f[1 + s2] = J >= 0 ? p.iface[(size_t)J * 4 + s2] : -1;
      a[1 + s2] = p.iface[(size_t)e * 4 + s2];
    }
    f[5] = J >= 0 ? (p.cls[J] * 4 + (sd ^ 1)) * n * 4 : 0;
    a[5] = p.cls[e] * 4 * 4 * n;
    a[6] = p.slot_off[e];
  }
  int rc = SMPM_OK;
  rc |= upload(c, side_fwd, &d.side_fwd, s);
  rc |= upload(c, side_adj, &d.side_adj, s);
  rc |= upload(c, p.nbr, &d.nbr, s);
  rc |= upload(c, p.cls, &d.cls, s);
  rc |= upload(c, p.slot_off, &d.slot_off, s);
  rc |= upload(c, p.side_slot, &d.side_slot, s);
  rc |= upload(c, p.iface, &d.iface, s);
  rc |= upload(c, p.side_elem, &d.side_elem, s);
  rc |= upload(c, p.side_dir, &d.side_dir, s);
  rc |= upload(c, p.iface_side, &d.iface_side, s);
  rc |= upload(c, nslots, &d.cls_nslots, s);
  rc |= upload(c, sidecol, &d.cls_sidecol, s);
  rc |= upload(c, p.W_off, &d.W_off, s);
  rc |= upload(c, p.H_off, &d.H_off, s);
  rc |= upload(c, p.Wc, &d.Wc, s);
  rc |= upload(c, p.Wr, &d.Wr, s);
  rc |= upload(c, p.Hc, &d.Hc, s);
  rc |= upload(c, p.Hr, &d.Hr, s);
  rc |= upload(c, p.WZ, &d.WZ, s);
  rc |= upload(c, wzc, &d.WZc, s);
  rc |= upload(c, p.Ainv, &d.Ainv, s);
  rc |= upload(c, p.AinvT, &d.AinvT, s);
  rc |= upload(c, p.blk_off, &d.blk_off, s);
  rc |= upload(c, p.blk_slots, &d.blk_slots, s);
  rc |= upload(c, p.blk_cls, &d.blk_cls, s);
  rc |= upload(c, p.bcls_off, &d.bcls_off, s);
  rc |= upload(c, p.bcls_size, &d.bcls_size, s);
  rc |= upload(c, p.MinvC, &d.MinvC, s);
  rc |= upload(c, p.MinvR, &d.MinvR, s);
  rc |= upload(c, p.G, &d.G, s);
  rc |= upload(c, GT, &d.GT, s);
  rc |= upload(c, p.sub.I_off, &d.sub_I_off, s);
  rc |= upload(c, p.sub.I, &d.sub_I, s);
  rc |= upload(c, p.sub.B_off, &d.sub_B_off, s);
  rc |= upload(c, p.sub.B, &d.sub_B, s);
  rc |= upload(c, p.sub.K_off, &d.sub_K_off, s);
  rc |= upload(c, p.sub.FR_off, &d.sub_FR_off, s);
  rc |= upload(c, p.sub.Kc, &d.sub_Kc, s);
  rc |= upload(c, p.sub.Kr, &d.sub_Kr, s);
  rc |= upload(c, p.sub.Fc, &d.sub_Fc, s);
  rc |= upload(c, p.sub.Fr, &d.sub_Fr, s);
  rc |= upload(c, p.sub.Rc, &d.sub_Rc, s);
  rc |= upload(c, p.sub.Rr, &d.sub_Rr, s);
  rc |= upload(c, p.sub.sep_iface, &d.sub_sep_iface, s);
  rc |= upload(c, p.sub.sep_pl, &d.sub_sep_pl, s);
  // the substructured kernels' two-step index lookups, composed once here
  std::vector<int> sub_B_iface(p.sub.B.size()), sub_sep_woff(p.sub.sep_pl.size() / 2);
  for (size_t i = 0; i < p.sub.B.size(); ++i) sub_B_iface[i] = p.sub.sep_iface[p.sub.B[i]];
  for (size_t b = 0; b * 4 < p.sub.sep_pl.size(); ++b)
    for (int h = 0; h < 2; ++h) {
      const int pp = p.sub.sep_pl[b * 4 + 2 * h], loc = p.sub.sep_pl[b * 4 + 2 * h + 1];
      sub_sep_woff[b * 2 + h] = p.sub.B_off[pp] + pp * p.sub.border + loc;
    }
  rc |= upload(c, sub_B_iface, &d.sub_B_iface, s);
  rc |= upload(c, sub_sep_woff, &d.sub_sep_woff, s);
  rc |= upload(c, p.sub.Si, &d.sub_Si, s);
  rc |= upload(c, p.sub.SiT, &d.sub_SiT, s);
  rc |= upload(c, to_f32(p.Wc), &d.WcF, s);
  rc |= upload(c, to_f32(p.Wr), &d.WrF, s);
  rc |= upload(c, to_f32(p.MinvC), &d.MinvCF, s);
  rc |= upload(c, to_f32(p.MinvR), &d.MinvRF, s);
  rc |= upload(c, to_b16(p.Wc), &d.WcB, s);
  rc |= upload(c, to_b16(p.Wr), &d.WrB, s);
  rc |= upload(c, to_b16(p.MinvC), &d.MinvCB, s);
  rc |= upload(c, to_b16(p.MinvR), &d.MinvRB, s);
  HIPCHK(hipStreamSynchronize(s));  // the converted host copies are temporaries
  d.ngrp = p.ngrp;
  d.grp_size = p.grp_size;
  rc |= upload(c, p.grp_cls, &d.grp_cls, s);
  rc |= upload(c, p.grp_elem, &d.grp_elem, s);
  d.ntile = p.ntile;
  rc |= upload(c, p.tile_cls, &d.tile_cls, s);
  rc |= upload(c, p.tile_elem, &d.tile_elem, s);
  rc |= upload(c, p.tile_src, &d.tile_src, s);
  rc |= upload(c, p.tile_dst, &d.tile_dst, s);
  d.mma_mt = p.mma_mt;
  for (int q = 0; q < 4; ++q) d.schur_nc[q] = 0;
  for (int q = 0; q < 4; ++q) d.schur_pers[q] = 0;
  if (const char* e = std::getenv("SMPM_MIXED_BASIS")) c->mixed_basis32 = std::atoi(e) == 64 ? 0 : 1;
  if (const char* e = std::getenv("SMPM_SCHUR_PERSIST"))  // sweep hook
    for (int q = 0; q < 4; ++q) {
      const int v = std::atoi(e);
      d.schur_pers[q] = v >= 3 ? 3 : v == 2 ? 2 : v > 0 ? 1 : v < 0 ? -1 : 0;
    }
  for (int q = 0; q < 4; ++q) d.schur_cpw[q] = 0;
  if (const char* e = std::getenv("SMPM_SCHUR_CPW"))  // sweep hook: columns per workgroup (column-pipelined)
    for (int q = 0; q < 4; ++q) d.schur_cpw[q] = std::max(0, std::min(64, std::atoi(e)));
  {
    int ncu = 0;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, c->dev_id) != hipSuccess || ncu <= 0)
      ncu = 256;
    d.num_cu = ncu;
  }
  if (const char* e = std::getenv("SMPM_SCHUR_NC")) {  // sweep hook: fixed columns per workgroup
    const int v = std::atoi(e);
    if (v == 1 || v == 2 || v == 4)
      for (int q = 0; q < 4; ++q) d.schur_nc[q] = v;
  }
  rc |= upload(c, p.Afwd, &d.Afwd, s);
  rc |= upload(c, p.Aadj, &d.Aadj, s);
  rc |= upload(c, to_f32(p.Afwd), &d.AfwdF, s);
  rc |= upload(c, to_f32(p.Aadj), &d.AadjF, s);
  rc |= upload(c, to_b16(p.Afwd), &d.AfwdB, s);
  rc |= upload(c, to_b16(p.Aadj), &d.AadjB, s);
  rc |= upload(c, bnode, &d.bdry_node, s);
  rc |= upload(c, btau, &d.bdry_tau, s);
  if (rc != SMPM_OK) return SMPM_ENOMEM;
  // vectors: quadrature weights, ones, unit v0, 1/sqrt(r), null vectors
  std::vector<double> wq(p.r), ones(p.r, 1.0), v0h(p.v0), rh(p.r, 1.0 / std::sqrt((double)p.r));
  double wsum = 0;
  for (int e = 0; e < p.nel; ++e) {
    const int ix = e % p.mx, iy = e / p.mx;
    const double we = p.xb[ix + 1] - p.xb[ix], he = p.yb[iy + 1] - p.yb[iy];
    for (int q = 0; q < n; ++q)
      for (int pp = 0; pp < n; ++pp) {
        const double v = p.omega[pp] * p.omega[q] * we * he / 4.0;
        wq[(size_t)e * n * n + q * n + pp] = v;
        wsum += v;
      }
  }
  double nv = 0;
  for (double v : v0h) nv += v * v;
  nv = std::sqrt(nv);
  for (double& v : v0h) v /= nv;
  c->wsum = wsum;
  c->precond_regular = !(p.nblk == 1 && (int64_t)p.blk_off[1] == p.k);
  const double* tmp = nullptr;
  rc |= upload(c, wq, &tmp, s);
  c->wq = const_cast<double*>(tmp);
  rc |= upload(c, ones, &tmp, s);
  c->ones = const_cast<double*>(tmp);
  rc |= upload(c, v0h, &tmp, s);
  c->v0hat = const_cast<double*>(tmp);
  rc |= upload(c, rh, &tmp, s);
  c->rhat = const_cast<double*>(tmp);
  rc |= dalloc(c->mem, &c->uL, p.r);
  rc |= dalloc(c->mem, &c->uS, p.k);
  if (rc != SMPM_OK) return SMPM_ENOMEM;
  HIPCHK(hipStreamSynchronize(s));
  return SMPM_OK;
}

// ---------------------------------------------------------------- static scratch

// Device scratch of smpm_project_noalloc: a file-scope array, one copy per GPU, held
// until the process ends.  Host code never passes the array's name to a kernel (on
// the host it is only a stand-in for the symbol): its device address is looked up
// once per device with hipGetSymbolAddress (at context setup, with the device
// current) and that pointer is used for every launch.
constexpr size_t kNoAllocScratchDoubles = (size_t)4 << 20;  // 32 MiB
__device__ __align__(256) double scratch[kNoAllocScratchDoubles];
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

// Resolves (once per device) and returns the device address of `scratch` on device
// `dev`, which must be the current device.
int noalloc_scratch(int dev, double** out) {
  if (dev < 0 || dev >= kMaxDevices) return fail(SMPM_EINVAL, "device id out of range for the static scratch");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return fail(SMPM_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_ptr[dev] = static_cast<double*>(ptr);
  }
  *out = g_scratch_ptr[dev];
  return SMPM_OK;
}

// Scratch of a projection: the Schur product t (k x nrhs), the interface sums c and
// the coarse solution c2 (d x nrhs each), the dot partials and the dots.
struct ProjScratch {
  double *t, *c, *c2, *part, *scal;
};

int project_impl(smpm_ctx* c, const DevPlan& P, const ProjScratch& sc, int which, const double* in, double* out,
                 int nrhs, bool tr, hipStream_t s) {
  if ((which == SMPM_PROJ_P || which == SMPM_PROJ_Q) && !c->plan.has_coarse)
    return fail(SMPM_EINVAL, "no coarse space on this grid");
  switch (which) {
    case SMPM_PROJ_L: {
      const double* u = tr ? c->rhat : c->uL;
      launch_mdot(u, 0, 0, 1, in, P.r, nullptr, P.r, nrhs, sc.part, sc.scal, nullptr, s);
      launch_axpy_shared(in, P.r, u, sc.scal, 1.0, out, P.r, nrhs, s);
      break;
    }
    case SMPM_PROJ_S: {
      const double* u = tr ? c->v0hat : c->uS;
      launch_mdot(u, 0, 0, 1, in, P.k, nullptr, P.k, nrhs, sc.part, sc.scal, nullptr, s);
      launch_axpy_shared(in, P.k, u, sc.scal, 1.0, out, P.k, nrhs, s);
      break;
    }
    case SMPM_PROJ_MEAN: {
      // x - 1 (w^T x)/(w^T 1); transposed: x - w (1^T x)/(w^T 1)
      if (!tr) {
        launch_mdot(c->wq, 0, 0, 1, in, P.r, nullptr, P.r, nrhs, sc.part, sc.scal, nullptr, s);
        launch_axpy_shared(in, P.r, c->ones, sc.scal, 1.0 / c->wsum, out, P.r, nrhs, s);
      } else {
        launch_mdot(c->ones, 0, 0, 1, in, P.r, nullptr, P.r, nrhs, sc.part, sc.scal, nullptr, s);
        launch_axpy_shared(in, P.r, c->wq, sc.scal, 1.0 / c->wsum, out, P.r, nrhs, s);
      }
      break;
    }
    case SMPM_PROJ_P: {
      // P x = x - S Z G Z^T x;  P^T x = x - Z G^T Z^T S^T x
      if (!tr) {
        launch_iface_sum(P, in, sc.c, nrhs, nullptr, s);
        launch_coarse(P, sc.c, sc.c2, nrhs, false, nullptr, s);
        launch_prolong(P, in, sc.c2, out, nrhs, 1, -1.0, nullptr, s);
      } else {
        launch_schur(P, in, sc.t, nrhs, true, nullptr, s);
        launch_iface_sum(P, sc.t, sc.c, nrhs, nullptr, s);
        launch_coarse(P, sc.c, sc.c2, nrhs, true, nullptr, s);
        launch_prolong(P, in, sc.c2, out, nrhs, 0, -1.0, nullptr, s);
      }
      break;
    }
    case SMPM_PROJ_Q: {
      // Q x = x - Z G Z^T S x;  Q^T x = x - S^T Z G^T Z^T x
      if (!tr) {
        launch_schur(P, in, sc.t, nrhs, false, nullptr, s);
        launch_iface_sum(P, sc.t, sc.c, nrhs, nullptr, s);
        launch_coarse(P, sc.c, sc.c2, nrhs, false, nullptr, s);
        launch_prolong(P, in, sc.c2, out, nrhs, 0, -1.0, nullptr, s);
      } else {
        launch_iface_sum(P, in, sc.c, nrhs, nullptr, s);
        launch_coarse(P, sc.c, sc.c2, nrhs, true, nullptr, s);
        launch_prolong(P, in, sc.c2, out, nrhs, 2, -1.0, nullptr, s);
      }
      break;
    }
    default:
      return fail(SMPM_EINVAL, "unknown projection");
  }
  HIPCHK(hipGetLastError());
  return SMPM_OK;
}


bool aliases(const void* a, size_t na, const void* b, size_t nb) {
  const char* pa = static_cast<const char*>(a);
  const char* pb = static_cast<const char*>(b);
  return pa < pb + nb && pb < pa + na;
}

}  // namespace

// ======================================================================== ABI

extern "C" {

void smpm_default_opts(smpm_solve_opts* o) {
  if (!o) return;
  o->tol = 1e-10;
  o->maxit = 400;
  o->precision = SMPM_FP64;
  o->transpose = 0;
  o->variant = 3;
  o->inner_tol = 1e-5;
  o->max_refine = 20;
  o->graph = 1;
  o->stop_rule = 0;
  o->profile = 0;
  o->block = 0;
}

const char* smpm_last_error(const smpm_ctx*) { return g_err.c_str(); }

int smpm_plan_robin(int m_y, int m_x, int n, const double* xb, const double* yb, double penalty, int robin,
                    smpm_ctx** out) {
  g_err.clear();
  if (!out) return fail(SMPM_EINVAL, "null output pointer");
  smpm_ctx* c = new (std::nothrow) smpm_ctx();
  if (!c) return fail(SMPM_ENOMEM, "host allocation failed");
  std::string msg;
  try {
    msg = build_plan(c->plan, m_y, m_x, n, xb, yb, penalty, robin);
  } catch (const std::bad_alloc&) {
    delete c;
    return fail(SMPM_ENOMEM, "host allocation failed in setup");
  }
  if (!msg.empty()) {
    delete c;
    const bool sing = msg.find("singular") != std::string::npos;
    return fail(sing ? SMPM_ESINGULAR : SMPM_EINVAL, msg);
  }
  *out = c;
  return SMPM_OK;
}

int smpm_plan(int m_y, int m_x, int n, const double* xb, const double* yb, double penalty, smpm_ctx** out) {
  return smpm_plan_robin(m_y, m_x, n, xb, yb, penalty, SMPM_ROBIN_MIN, out);
}

int smpm_setup_robin(int m_y, int m_x, int n, const double* xb, const double* yb, double penalty, int robin,
                     void* stream, smpm_ctx** out) {
  g_err.clear();
  if (!out) return fail(SMPM_EINVAL, "null output pointer");
  smpm_ctx* c = nullptr;
  int rc = smpm_plan_robin(m_y, m_x, n, xb, yb, penalty, robin, &c);
  if (rc) return rc;
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (hipGetDevice(&c->dev_id) != hipSuccess) {
    delete c;
    return fail(SMPM_EHIP, "no HIP device");
  }
  c->device = true;
  double* scr = nullptr;
  rc = noalloc_scratch(c->dev_id, &scr);  // the static scratch's address on this device
  if (!rc) rc = do_upload(c, s);
  if (rc) {
    std::string keep = g_err;
    delete c;
    g_err = keep;
    return rc;
  }
  *out = c;
  return SMPM_OK;
}

int smpm_setup(int m_y, int m_x, int n, const double* xb, const double* yb, double penalty, void* stream,
               smpm_ctx** out) {
  return smpm_setup_robin(m_y, m_x, n, xb, yb, penalty, SMPM_ROBIN_MIN, stream, out);
}

void smpm_destroy(smpm_ctx* c) { delete c; }

int smpm_sizes(const smpm_ctx* c, int64_t* r, int64_t* k, int64_t* d) {
  if (!c) return fail(SMPM_EINVAL, "null context");
  if (r) *r = c->plan.r;
  if (k) *k = c->plan.k;
  if (d) *d = c->plan.d;
  return SMPM_OK;
}

int smpm_stats(const smpm_ctx* c, smpm_plan_stats* o) {
  if (!c || !o) return fail(SMPM_EINVAL, "null argument");
  const Plan& p = c->plan;
  o->element_classes = (int64_t)p.classes.size();
  o->block_classes = (int64_t)p.bcls_size.size();
  o->schur_operator_bytes = (int64_t)(p.Wc.size() * sizeof(double));
  o->precond_operator_bytes = (int64_t)(p.MinvC.size() * sizeof(double));
  o->flux_operator_bytes = (int64_t)(p.Hc.size() * sizeof(double));
  // bytes one coarse solve reads: the dense G, or the patch matrices and S_B^{-1}
  o->coarse_bytes = p.coarse_mode == 2
                        ? (int64_t)((p.sub.Kc.size() + p.sub.Fc.size() + p.sub.Rc.size() + p.sub.Si.size()) *
                                    sizeof(double))
                        : (int64_t)(p.G.size() * sizeof(double));
  o->coarse_singular = p.coarse_singular ? 1 : 0;
  o->has_coarse = p.has_coarse ? 1 : 0;
  o->null_residual = c->null_residual;
  o->null_iterations = c->null_iterations;
  o->schur_norm_bound = schur_norm_bound(p);
  return SMPM_OK;
}

int smpm_slot_map(const smpm_ctx* c, int64_t* out) {
  if (!c || !out) return fail(SMPM_EINVAL, "null argument");
  const Plan& p = c->plan;
  const int n = p.n;
  for (int64_t si = 0; si < p.nsides; ++si) {
    const int e = p.side_elem[si], s = p.side_dir[si];
    for (int t = 0; t < n; ++t) {
      const int l = s == SW ? t * n : s == SE ? t * n + n - 1 : s == SS ? t : (n - 1) * n + t;
      out[si * n + t] = (int64_t)e * n * n + l;
    }
  }
  return SMPM_OK;
}

int smpm_node_coords(const smpm_ctx* c, double* x, double* y) {
  if (!c || !x || !y) return fail(SMPM_EINVAL, "null argument");
  const Plan& p = c->plan;
  const int n = p.n;
  for (int e = 0; e < p.nel; ++e) {
    const int ix = e % p.mx, iy = e / p.mx;
    const double we = p.xb[ix + 1] - p.xb[ix], he = p.yb[iy + 1] - p.yb[iy];
    for (int q = 0; q < n; ++q)
      for (int pp = 0; pp < n; ++pp) {
        x[(size_t)e * n * n + q * n + pp] = p.xb[ix] + (p.xi[pp] + 1.0) * we / 2.0;
        y[(size_t)e * n * n + q * n + pp] = p.yb[iy] + (p.xi[q] + 1.0) * he / 2.0;
      }
  }
  return SMPM_OK;
}

int smpm_quadrature_weights(const smpm_ctx* c, double* w) {
  if (!c || !w) return fail(SMPM_EINVAL, "null argument");
  const Plan& p = c->plan;
  const int n = p.n;
  for (int e = 0; e < p.nel; ++e) {
    const int ix = e % p.mx, iy = e / p.mx;
    const double we = p.xb[ix + 1] - p.xb[ix], he = p.yb[iy + 1] - p.yb[iy];
    for (int q = 0; q < n; ++q)
      for (int pp = 0; pp < n; ++pp) w[(size_t)e * n * n + q * n + pp] = p.omega[pp] * p.omega[q] * we * he / 4.0;
  }
  return SMPM_OK;
}

int smpm_export(const smpm_ctx* c, int what, int64_t* count, int64_t* rows, int64_t* cols, double* vals) {
  if (!c || !count) return fail(SMPM_EINVAL, "null argument");
  const Plan& p = c->plan;
  if (what == SMPM_EXPORT_COARSE || what == SMPM_EXPORT_COARSE_PINV) {
    if (!p.has_coarse) return fail(SMPM_EINVAL, "no coarse space on this grid");
    *count = p.d * p.d;
    if (!vals) return SMPM_OK;
    if (p.coarse_mode == 1) {
      const std::vector<double>& src = what == SMPM_EXPORT_COARSE ? p.C : p.G;
      std::copy(src.begin(), src.end(), vals);
      return SMPM_OK;
    }
    // substructured mode: dense copies on request (d <= 8192)
    if (p.d > 8192) return fail(SMPM_EINVAL, "dense coarse export limited to d <= 8192");
    const int64_t d = p.d;
    std::fill(vals, vals + d * d, 0.0);
    if (what == SMPM_EXPORT_COARSE) {
      for (int64_t i = 0; i < d; ++i)
        for (int64_t z = p.C_off[i]; z < p.C_off[i + 1]; ++z) vals[i * d + p.C_col[z]] = p.C_val[z];
      return SMPM_OK;
    }
    // G e_j column by column with the host substructured solve
    std::vector<double> e(d, 0.0), col(d, 0.0);
    for (int64_t j = 0; j < d; ++j) {
      e[j] = 1.0;
      sub_solve_host(p, e.data(), 0.0, col.data(), false);
      e[j] = 0.0;
      for (int64_t i = 0; i < d; ++i) vals[i * d + j] = col[i];
    }
    return SMPM_OK;
  }
  std::vector<int64_t> ri, ci;
  std::vector<double> v;
  if (what == SMPM_EXPORT_SCHUR)
    export_schur_coo(p, ri, ci, v);
  else if (what == SMPM_EXPORT_FLUX_SOLVE)
    export_flux_solve_coo(p, ri, ci, v);
  else if (what == SMPM_EXPORT_PRECOND_INV)
    export_precond_inv_coo(p, ri, ci, v);
  else
    return fail(SMPM_EINVAL, "unknown export kind");
  if (rows || cols || vals) {
    if ((int64_t)v.size() > *count) return fail(SMPM_EINVAL, "export buffer too small");
    if (rows) std::copy(ri.begin(), ri.end(), rows);
    if (cols) std::copy(ci.begin(), ci.end(), cols);
    if (vals) std::copy(v.begin(), v.end(), vals);
  }
  *count = (int64_t)v.size();
  return SMPM_OK;
}

int smpm_null_vectors(smpm_ctx* c, double* uL, double* uS) {
  int rc = check_device(c);
  if (rc) return rc;
  rc = compute_null_vectors(c, nullptr);
  if (rc) return rc;
  if (uL) std::copy(c->h_uL.begin(), c->h_uL.end(), uL);
  if (uS) std::copy(c->h_uS.begin(), c->h_uS.end(), uS);
  return SMPM_OK;
}

int smpm_schur_apply(smpm_ctx* c, const double* v, double* Sv, int nrhs, int transpose, void* stream) {
  int rc = check_device(c);
  if (rc) return rc;
  if (!v || !Sv || nrhs < 1) return fail(SMPM_EINVAL, "bad vector arguments");
  const size_t bytes = sizeof(double) * c->plan.k * nrhs;
  if (aliases(v, bytes, Sv, bytes)) return fail(SMPM_EINVAL, "input and output alias");
  // the result goes back to the caller: written past the caches
  launch_schur_ex(c->dp, v, Sv, nrhs, transpose != 0, nullptr, nullptr, static_cast<hipStream_t>(stream), PREC_F64,
                  true);
  HIPCHK(hipGetLastError());
  return SMPM_OK;
}

int smpm_schur_apply_prec(smpm_ctx* c, const double* v, double* Sv, int nrhs, int transpose, int precision,
                          void* stream) {
  int rc = check_device(c);
  if (rc) return rc;
  if (!v || !Sv || nrhs < 1) return fail(SMPM_EINVAL, "bad vector arguments");
  if (precision < SMPM_FP64 || precision > SMPM_MIXED_BF16) return fail(SMPM_EINVAL, "unknown precision");
  const size_t bytes = sizeof(double) * c->plan.k * nrhs;
  if (aliases(v, bytes, Sv, bytes)) return fail(SMPM_EINVAL, "input and output alias");
  const int prec = precision == SMPM_MIXED_FP32 ? PREC_F32 : precision == SMPM_MIXED_BF16 ? PREC_BF16 : PREC_F64;
  launch_schur_ex(c->dp, v, Sv, nrhs, transpose != 0, nullptr, nullptr, static_cast<hipStream_t>(stream), prec);
  HIPCHK(hipGetLastError());
  return SMPM_OK;
}

int smpm_solve_group(smpm_ctx* const* ctxs, int nprob, const double* const* f, const double* const* g,
                     double* const* u, const int* nrhs, const smpm_solve_opts* opts, smpm_solve_info* infos,
                     void* stream) {
  if (!ctxs || nprob < 1 || !f || !u || !nrhs) return fail(SMPM_EINVAL, "bad group arguments");
  smpm_solve_opts o;
  smpm_default_opts(&o);
  if (opts) o = *opts;
  if (o.maxit < 1 || o.maxit > kMaxIt) return fail(SMPM_EINVAL, "bad solve options (1 <= maxit <= 1000)");
  hipStream_t s = static_cast<hipStream_t>(stream);
  for (int i = 0; i < nprob; ++i) {
    int rc = check_device(ctxs[i]);
    if (rc) return fail(rc, "problem " + std::to_string(i) + ": " + g_err);
    if (ctxs[i]->dev_id != ctxs[0]->dev_id) return fail(SMPM_EINVAL, "group problems must share one device");
    if (nrhs[i] < 1 || !f[i] || !u[i]) return fail(SMPM_EINVAL, "problem " + std::to_string(i) + ": bad vectors");
    for (int j = 0; j < i; ++j)
      if (ctxs[j] == ctxs[i]) return fail(SMPM_EINVAL, "a context appears twice in the group");
  }
  // Everything that allocates or synchronizes the device happens here, in order,
  // before the problems run concurrently: null vectors, workspaces, streams.
  for (int i = 0; i < nprob; ++i) {
    smpm_ctx* c = ctxs[i];
    int rc = compute_null_vectors(c, s);
    if (!rc) rc = ensure_ws(c, nrhs[i], o.maxit);
    if (rc) return fail(rc, "problem " + std::to_string(i) + ": " + g_err);
    if (!c->group_stream) HIPCHK(hipStreamCreateWithFlags(&c->group_stream, hipStreamNonBlocking));
  }
  hipEvent_t start;
  HIPCHK(hipEventCreateWithFlags(&start, hipEventDisableTiming));
  hipError_t he = hipEventRecord(start, s);
  for (int i = 0; i < nprob && he == hipSuccess; ++i) he = hipStreamWaitEvent(ctxs[i]->group_stream, start, 0);
  if (he != hipSuccess) {
    (void)hipEventDestroy(start);
    return fail(SMPM_EHIP, std::string("group stream ordering: ") + hipGetErrorString(he));
  }
  // one host thread per problem drives its solve on its own stream; the kernels of
  // the problems overlap on the device
  std::vector<int> rcs(nprob, SMPM_OK);
  std::vector<std::string> msgs(nprob);
  auto run = [&](int i) {
    smpm_ctx* c = ctxs[i];
    if (hipSetDevice(c->dev_id) != hipSuccess) {
      rcs[i] = SMPM_EHIP;
      msgs[i] = "hipSetDevice failed";
      return;
    }
    rcs[i] = smpm_solve(c, f[i], g ? g[i] : nullptr, u[i], nrhs[i], &o, infos ? &infos[i] : nullptr,
                        c->group_stream);
    if (rcs[i] != SMPM_OK) msgs[i] = g_err;
    if (hipStreamSynchronize(c->group_stream) != hipSuccess && rcs[i] == SMPM_OK) {
      rcs[i] = SMPM_EHIP;
      msgs[i] = "stream synchronize failed";
    }
  };
  std::vector<std::thread> workers;
  workers.reserve(nprob - 1);
  for (int i = 1; i < nprob; ++i) workers.emplace_back(run, i);
  run(0);
  for (auto& t : workers) t.join();
  (void)hipEventDestroy(start);
  // a hard error wins over non-convergence
  int worst = -1;
  for (int i = 0; i < nprob; ++i)
    if (rcs[i] != SMPM_OK && (worst < 0 || (rcs[worst] == SMPM_ENOCONV && rcs[i] != SMPM_ENOCONV))) worst = i;
  if (worst >= 0) return fail(rcs[worst], "problem " + std::to_string(worst) + ": " + msgs[worst]);
  return SMPM_OK;
}

int smpm_autotune(smpm_ctx* c, int nrhs, void* stream, smpm_tune_result* out) {
  int rc = check_device(c);
  if (rc) return rc;
  if (nrhs < 1) return fail(SMPM_EINVAL, "nrhs must be positive");
  hipStream_t s = static_cast<hipStream_t>(stream);
  constexpr int kTuneIters = 24;
  rc = ensure_ws(c, nrhs, kTuneIters);
  if (rc) return rc;
  Workspace& W = c->ws;
  DevPlan& P = c->dp;
  const int cls = schur_nc_class(nrhs);
  const int64_t k = c->plan.k;
  launch_fill_pattern(W.xacc, k * nrhs, s);
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return fail(SMPM_EHIP, "hipEventCreate failed");
  }
  auto time_us = [&](auto&& body, int reps) -> float {
    for (int r = 0; r < 2; ++r) body();
    (void)hipEventRecord(e0, s);
    for (int r = 0; r < reps; ++r) body();
    (void)hipEventRecord(e1, s);
    (void)hipEventSynchronize(e1);
    float ms = 0;
    (void)hipEventElapsedTime(&ms, e0, e1);
    return ms * 1e3f / reps;
  };
  // 1. Schur launch shape, timed as the deflated Arnoldi step launches it (with the
  //    fused per-side sums where the dense coarse solve consumes them): the plain
  //    kernel with 1, 2 or 4 columns per workgroup, the persistent kernel, the
  //    warp-specialized persistent kernel (1 or 2 columns per item) or the
  //    column-pipelined kernel (2, 4 or 8 columns per workgroup); the last three have
  //    no side sums
  const bool fused = schur_has_side_sums(P) && P.coarse_mode == 1;
  struct Cand { int pers, nc, cpw; };
  const Cand cands[] = {{-1, 1, 0}, {-1, 2, 0}, {-1, 4, 0}, {1, 0, 0}, {2, 1, 0},
                        {2, 2, 0},  {3, 0, 2},  {3, 0, 4},  {3, 0, 8}};
  float best = 1e30f;
  Cand pick{P.schur_pers[cls], P.schur_nc[cls], P.schur_cpw[cls]};
  if (P.mma_mt > 0) {
    for (const Cand& cd : cands) {
      if (cd.nc > nrhs || (cd.cpw > 1 && cd.cpw / 2 >= nrhs)) continue;
      if (cd.pers > 0 && fused) continue;
      P.schur_pers[cls] = cd.pers;
      P.schur_nc[cls] = cd.nc;
      P.schur_cpw[cls] = cd.cpw;
      const float us =
          time_us([&] { launch_schur_ex(P, W.xacc, W.t, nrhs, false, nullptr, fused ? W.sides : nullptr, s); }, 20);
      if (us < best) {
        best = us;
        pick = cd;
      }
    }
    P.schur_pers[cls] = pick.pers;
    P.schur_nc[cls] = pick.nc;
    P.schur_cpw[cls] = pick.cpw;
  }
  c->drop_graphs();  // captured steps hold the launch shapes they were recorded with
  rc = hipGetLastError() == hipSuccess ? SMPM_OK : fail(SMPM_EHIP, "Schur timing launch failed");
  // 2. reduction of the Gram-Schmidt sums: kTuneIters deflated Arnoldi steps each way
  float best_step = 1e30f;
  int pre_pick = -1;
  if (rc == SMPM_OK && c->plan.has_coarse) {
    for (int pre = 0; pre < 2 && rc == SMPM_OK; ++pre) {
      c->prereduce_choice[cls] = pre;
      std::vector<int> it;
      const float total = time_us(
          [&] {
            const int r = solve_schur(c, OP_PSM, false, W.xacc, W.bS, nrhs, 1e-300, kTuneIters, it, s);
            if (r < 0 && rc == SMPM_OK) rc = r;
          },
          2);
      if (total / kTuneIters < best_step) {
        best_step = total / kTuneIters;
        pre_pick = pre;
      }
    }
    c->prereduce_choice[cls] = rc == SMPM_OK ? pre_pick : -1;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc != SMPM_OK) return rc;
  if (out) {
    out->nrhs = nrhs;
    out->schur_columns_per_workgroup = pick.pers == 3   ? std::min(pick.cpw, nrhs)
                                       : pick.pers == 1 ? (nrhs >= 2 ? 2 : 1)
                                                        : (pick.nc > 0 ? pick.nc : 1);
    out->schur_persistent = pick.pers > 0 ? pick.pers : 0;
    out->prereduce = pre_pick;
    out->schur_us = best < 1e29f ? best : 0.0;
    out->step_us = best_step < 1e29f ? best_step : 0.0;
  }
  return SMPM_OK;
}

int smpm_boundary_transpose(smpm_ctx* c, const double* mu, double* dg, int nrhs, void* stream) {
  int rc = check_device(c);
  if (rc) return rc;
  if (!mu || !dg || nrhs < 1) return fail(SMPM_EINVAL, "bad vector arguments");
  if (aliases(mu, sizeof(double) * c->plan.r * nrhs, dg, sizeof(double) * c->dp.nbdry * nrhs))
    return fail(SMPM_EINVAL, "input and output alias");
  launch_bdry_adj(c->dp, mu, dg, nrhs, static_cast<hipStream_t>(stream));
  HIPCHK(hipGetLastError());
  return SMPM_OK;
}

int smpm_precond_apply(smpm_ctx* c, const double* x, double* y, int nrhs, int transpose, void* stream) {
  int rc = check_device(c);
  if (rc) return rc;
  if (!x || !y || nrhs < 1) return fail(SMPM_EINVAL, "bad vector arguments");
  const size_t bytes = sizeof(double) * c->plan.k * nrhs;
  if (aliases(x, bytes, y, bytes)) return fail(SMPM_EINVAL, "input and output alias");
  launch_precond(c->dp, x, y, nrhs, transpose != 0, nullptr, static_cast<hipStream_t>(stream));
  HIPCHK(hipGetLastError());
  return SMPM_OK;
}

int smpm_project(smpm_ctx* c, int which, const double* in, double* out, int nrhs, int transpose, void* stream) {
  int rc = check_device(c);
  if (rc) return rc;
  if (!in || !out || nrhs < 1) return fail(SMPM_EINVAL, "bad vector arguments");
  hipStream_t s = static_cast<hipStream_t>(stream);
  rc = ensure_ws(c, nrhs, 1);
  if (rc) return rc;
  Workspace& W = c->ws;
  const bool tr = transpose != 0;
  if ((which == SMPM_PROJ_L || which == SMPM_PROJ_S) && !tr) {
    rc = compute_null_vectors(c, s);
    if (rc) return rc;
  }
  ProjScratch sc{W.t, W.c, W.c2, W.part, W.scal};
  return project_impl(c, c->dp, sc, which, in, out, nrhs, tr, s);
}

int smpm_project_noalloc(smpm_ctx* c, int which, const double* in, double* out, int nrhs, int transpose,
                         void* stream) {
  int rc = check_device(c);
  if (rc) return rc;
  if (!in || !out || nrhs < 1) return fail(SMPM_EINVAL, "bad vector arguments");
  if (which < SMPM_PROJ_L || which > SMPM_PROJ_MEAN) return fail(SMPM_EINVAL, "unknown projection");
  const bool tr = transpose != 0;
  if ((which == SMPM_PROJ_L || which == SMPM_PROJ_S) && !tr && !c->have_null)
    return fail(SMPM_EINVAL,
                "the null vectors are not computed yet (computing them allocates): call smpm_null_vectors or "
                "smpm_solve on this context first");
  const Plan& Pl = c->plan;
  // scratch layout per call: [t: k x nrhs][c: d x nrhs][c2: d x nrhs][coarse: cstride x nrhs]
  // [partials: chunks x nrhs][dots: nrhs], each part 32-double aligned
  auto up = [](int64_t v) { return (v + 31) / 32 * 32; };
  const int64_t R = nrhs, d = std::max<int64_t>(Pl.d, 1);
  int64_t cstride = 0;
  if (Pl.coarse_mode == 2)
    cstride = (int64_t)Pl.sub.B.size() + (int64_t)Pl.sub.npatch * Pl.sub.border + Pl.sub.nsep + Pl.sub.border + 1;
  const int64_t nch = reduce_chunks(std::max<int64_t>(Pl.r, Pl.k));
  const int64_t o_t = 0, o_c = o_t + up(Pl.k * R), o_c2 = o_c + up(d * R), o_cws = o_c2 + up(d * R),
                o_part = o_cws + up(std::max<int64_t>(cstride, 1) * R), o_scal = o_part + up(nch * R),
                need = o_scal + up(R);
  if (need > (int64_t)kNoAllocScratchDoubles) {
    char buf[200];
    std::snprintf(buf, sizeof buf,
                  "smpm_project_noalloc: %lld doubles of scratch needed, the static maximum is %lld (%d MiB); "
                  "use fewer columns per call or smpm_project",
                  (long long)need, (long long)kNoAllocScratchDoubles, (int)(kNoAllocScratchDoubles * 8 >> 20));
    return fail(SMPM_EINVAL, buf);
  }
  double* base = nullptr;
  rc = noalloc_scratch(c->dev_id, &base);
  if (rc) return rc;
  DevPlan P = c->dp;  // the substructured coarse solve reads its scratch through the plan view
  P.cws = base + o_cws;
  P.cws_stride = cstride;
  ProjScratch sc{base + o_t, base + o_c, base + o_c2, base + o_part, base + o_scal};
  return project_impl(c, P, sc, which, in, out, nrhs, tr, static_cast<hipStream_t>(stream));
}

int smpm_solve(smpm_ctx* c, const double* f, const double* g, double* u, int nrhs, const smpm_solve_opts* opts_in,
               smpm_solve_info* info, void* stream) {
  int rc = check_device(c);
  if (rc) return rc;
  if (!f || !u || nrhs < 1) return fail(SMPM_EINVAL, "bad vector arguments");
  smpm_solve_opts o;
  smpm_default_opts(&o);
  if (opts_in) o = *opts_in;
  if (o.maxit < 1 || o.maxit > kMaxIt || !(o.tol > 0) || o.variant < 1 || o.variant > 3)
    return fail(SMPM_EINVAL, "bad solve options (1 <= maxit <= 1000, tol > 0, variant 1..3)");
  if (o.precision < SMPM_FP64 || o.precision > SMPM_MIXED_BF16) return fail(SMPM_EINVAL, "unknown precision");
  if (o.precision != SMPM_FP64 && (!(o.inner_tol > 0) || o.inner_tol >= 1 || o.max_refine < 1))
    return fail(SMPM_EINVAL, "mixed precision needs 0 < inner_tol < 1 and max_refine >= 1");
  const bool tr = o.transpose != 0;
  if (tr && g) return fail(SMPM_EINVAL, "the adjoint solve takes no boundary data (g must be NULL)");
  if (o.variant == 3 && !c->plan.has_coarse)
    return fail(SMPM_EINVAL, "no coarse space on this grid: use variant 1 or 2");
  const Plan& Pl = c->plan;
  const DevPlan& P = c->dp;
  const size_t rb = sizeof(double) * Pl.r * nrhs;
  if (aliases(f, rb, u, rb)) return fail(SMPM_EINVAL, "f and u alias");
  if (o.stop_rule != 0 && o.stop_rule != 1) return fail(SMPM_EINVAL, "stop_rule must be 0 or 1");
  if (o.block != 0 && nrhs > kBgMaxCols) return fail(SMPM_EINVAL, "block GMRES takes at most 32 columns");
  hipStream_t s = static_cast<hipStream_t>(stream);
  rc = compute_null_vectors(c, s);
  if (rc) return rc;
  rc = ensure_ws(c, nrhs, o.maxit);
  if (rc) return rc;
  Workspace& W = c->ws;
  W.hist_len = 0;
  // per-phase timing (opts.profile or SMPM_PROFILE=1): events on the solve's stream
  bool profile = o.profile != 0;
  if (const char* e = std::getenv("SMPM_PROFILE")) profile = profile || e[0] == '1';
  hipEvent_t pev[4] = {nullptr, nullptr, nullptr, nullptr};
  if (profile) {
    for (auto& e : pev) HIPCHK(hipEventCreate(&e));
    HIPCHK(hipEventRecord(pev[0], s));
  }
  auto mark = [&](int i) {
    if (profile) (void)hipEventRecord(pev[i], s);
  };
  const int rule = o.stop_rule;
  const bool use_graph = o.graph != 0;
  // non-finite f or g: flagged by the kernel that first reads them, reported as
  // SMPM_EINVAL once the solve has run (a NaN estimate retires its column at once).
  // That kernel copies the user's data into W.rhs (adding T g); every later step works
  // on workspace buffers, so the phases below can be replayed from captured graphs.
  *W.hnonfinite = 0;  // nothing of an earlier solve is in flight (each ends synchronized)
  launch_rhs(P, f, tr ? nullptr : g, W.rhs, nrhs, W.nonfinite, s);
  // u_L^T (f + T g) (adjoint: 1^T c) per column, published with the post-processing
  double* removed = W.scal2 + 3 * nrhs;
  // b_hat's side sums feed the dense coarse solve of the GMRES start (sides of n
  // consecutive slots, summed by n-lane butterflies: n a power of two)
  const bool sides_ok = o.variant == 3 && Pl.has_coarse && P.coarse_mode == 1 && P.d > 0 && Pl.n <= 64 &&
                        (Pl.n & (Pl.n - 1)) == 0;
  auto pre_body = [&](hipStream_t q) {
    if (!tr) {
      // steps 1-3: f~ = (I - u_L u_L^T)(f + T g); b_S = B A^{-1} f~; b_hat = (I - u_S u_S^T) b_S
      launch_mdot(c->uL, 0, 0, 1, W.rhs, Pl.r, nullptr, Pl.r, nrhs, W.part, removed, nullptr, q);
      // f~ while B A^{-1} stages it, with u_S^T b_S from the stored slots
      if (!launch_flux_projected(P, W.rhs, c->uL, removed, 1.0, W.ft, W.bS, nrhs, q, c->uS, W.part, W.scal)) {
        launch_axpy_shared(W.rhs, Pl.r, c->uL, removed, 1.0, W.ft, Pl.r, nrhs, q);
        launch_flux(P, W.ft, W.bS, nrhs, q);
        launch_mdot(c->uS, 0, 0, 1, W.bS, Pl.k, nullptr, Pl.k, nrhs, W.part, W.scal, nullptr, q);
      }
      // b_hat, and |b_hat|^2 (the GMRES stopping reference) and its side sums in the same launch
      launch_axpy_norm2(W.bS, c->uS, W.scal, 1.0, W.bhat, Pl.k, nrhs, W.part, W.scal2 + 2 * nrhs, q,
                        sides_ok ? W.sides : nullptr, P.n);
    } else {
      // adjoint of the solution map: c~ = c - w (1^T c)/(w^T 1); S^T xi = E^T A^{-T} c~
      // (consistent: v0^T E^T A^{-T} c~ = -1^T c~ = 0), projected off v0 against rounding
      launch_mdot(c->ones, 0, 0, 1, W.rhs, Pl.r, nullptr, Pl.r, nrhs, W.part, removed, nullptr, q);
      launch_axpy_shared(W.rhs, Pl.r, c->wq, removed, 1.0 / c->wsum, W.ft, Pl.r, nrhs, q);
      launch_local_adj(P, W.ft, W.bS, nrhs, true, q);
      launch_mdot(c->v0hat, 0, 0, 1, W.bS, Pl.k, nullptr, Pl.k, nrhs, W.part, W.scal, nullptr, q);
      launch_axpy_norm2(W.bS, c->v0hat, W.scal, 1.0, W.bhat, Pl.k, nrhs, W.part, W.scal2 + 2 * nrhs, q,
                        sides_ok ? W.sides : nullptr, P.n);
    }
  };
  // step 9 up to the last store: forward u = A^{-1}(f~ - E x) into W.ubuf and w^T u
  // into W.scal; adjoint mu = A^{-T}(c~ - B^T xi) into W.ubuf and u_L^T mu into W.scal
  auto post_body = [&](const double* xs, hipStream_t q) {
    if (!tr) {
      if (!launch_backsub_dot(P, W.ft, xs, W.ubuf, c->wq, nrhs, W.part, W.scal, q)) {
        launch_backsub(P, W.ft, xs, W.ubuf, nrhs, q);
        launch_mdot(c->wq, 0, 0, 1, W.ubuf, Pl.r, nullptr, Pl.r, nrhs, W.part, W.scal, nullptr, q);
      }
    } else {
      launch_local_adj(P, W.ft, W.ubuf, nrhs, false, q);
      launch_flux_adj(P, xs, W.rhs, nrhs, q);
      launch_add(W.ubuf, W.rhs, -1.0, W.ubuf, Pl.r, nrhs, q);
      launch_mdot(c->uL, 0, 0, 1, W.ubuf, Pl.r, nullptr, Pl.r, nrhs, W.part, W.scal, nullptr, q);
    }
  };
  // the last store into the user's u: the constant (forward: u -= (w^T u / w^T 1) 1) or
  // the u_L component (adjoint, the null space of L^T) removed
  auto store_u = [&](hipStream_t q) {
    if (!tr)
      launch_axpy_shared(W.ubuf, Pl.r, c->ones, W.scal, 1.0 / c->wsum, u, Pl.r, nrhs, q);
    else
      launch_axpy_shared(W.ubuf, Pl.r, c->uL, W.scal, 1.0, u, Pl.r, nrhs, q);
  };
  // steps 4-8
  std::vector<int> iters;
  const int kind = o.variant == 3 ? OP_PSM : o.variant == 2 ? OP_SM : OP_S;
  std::vector<double> tres;
  int cycles = 1;
  int sprec_final = PREC_F64;  // Schur precision of the last inner solve
  double hist[16] = {0};
  int cyc_it[16] = {0};
  int ncyc = 0;
  auto note_cycle = [&](const std::vector<int>& it) {
    int mx = 0;
    for (int v : it) mx = std::max(mx, v);
    if (ncyc < 16) cyc_it[ncyc] = mx;
    ++ncyc;
  };
  bool conv = true;
  if (o.block && o.precision == SMPM_FP64) {
    // Steps 1-3, then step 4 as block GMRES over all columns (FP64, launched as it
    // goes: a block step waits for its kept count), steps 5-9; FP64 correction cycles
    // as below when the true residual misses tol.
    rc = ensure_bws(c, nrhs, o.maxit);
    if (rc) return rc;
    pre_body(s);
    mark(1);
    std::vector<double> res0;
    const int st0 = block_solve_schur(c, kind, tr, W.bhat, W.bS, nrhs, o.tol, o.maxit,
                                      rule == 1 ? nullptr : W.scal2 + 2 * nrhs, s, &res0);
    if (st0 < 0) return st0;
    iters.assign(nrhs, st0);
    note_cycle(iters);
    rc = true_residual(c, tr, W.bhat, W.bS, nrhs, tres, s);
    if (rc) return rc;
    for (int extra = 0; extra < 2; ++extra) {
      double worst = 0.0;
      bool fixable = true, any = false;
      for (int i = 0; i < nrhs; ++i) {
        if (tres[i] <= o.tol) continue;
        any = true;
        if (!std::isfinite(tres[i]) || iters[i] >= o.maxit) fixable = false;
        worst = std::max(worst, tres[i]);
      }
      if (!any || !fixable) break;
      launch_copy(W.bS, W.xacc, Pl.k * nrhs, s);
      launch_schur(P, W.xacc, W.t, nrhs, tr, nullptr, s);
      launch_add(W.bhat, W.t, -1.0, W.rho, Pl.k, nrhs, s);
      const double* nl = tr ? c->v0hat : c->uS;
      launch_mdot(nl, 0, 0, 1, W.rho, Pl.k, nullptr, Pl.k, nrhs, W.part, W.scal, nullptr, s);
      launch_axpy_shared(W.rho, Pl.k, nl, W.scal, 1.0, W.rho, Pl.k, nrhs, s);
      if (rule != 1)
        launch_mdot(W.rho, 0, Pl.k, 1, W.rho, Pl.k, nullptr, Pl.k, nrhs, W.part, W.scal2 + 2 * nrhs, nullptr, s);
      const int st = block_solve_schur(c, kind, tr, W.rho, W.bS, nrhs, std::min(0.5, 0.3 * o.tol / worst), o.maxit,
                                       rule == 1 ? nullptr : W.scal2 + 2 * nrhs, s, &res0);
      if (st < 0) return st;
      std::vector<int> it(nrhs, st);
      note_cycle(it);
      for (int i = 0; i < nrhs; ++i) iters[i] += st;
      launch_add(W.xacc, W.bS, 1.0, W.bS, Pl.k, nrhs, s);
      ++cycles;
      rc = true_residual(c, tr, W.bhat, W.bS, nrhs, tres, s);
      if (rc) return rc;
    }
    for (int i = 0; i < nrhs; ++i)
      if (!(tres[i] <= o.tol)) conv = false;
    mark(2);
    post_body(W.bS, s);
    store_u(s);
    launch_publish(removed, nrhs, W.hout + 2 * nrhs, s);
    // history: column 0's least-squares residual / reference after each block step
    W.hist_len = (int)std::min<size_t>(res0.size(), (size_t)W.maxit + 1);
    for (int i = 0; i < W.hist_len; ++i) {
      W.hhist[i] = res0[i];
      W.hhist_cs[i] = 0.0;
    }
    *W.hhist_tolb = 1.0;
    W.hist_tol = 1.0;
  } else if (o.precision == SMPM_FP64) {
    // One pass with a single synchronization: [steps 1-3, GMRES start] as one phase;
    // the Arnoldi chunks; [closing rotation, least squares, recovery of x into W.bS
    // (steps 5-8), the FP64 true residual, step 9 into W.ubuf] as another; the store
    // into u.  Each phase is a fixed launch sequence on workspace buffers, replayed
    // from a graph captured on first use for its shape.
    GmState S = gm_state(c, nrhs, o.maxit);
    // stopping reference: |b_hat| (the quantity the FP64 true residual is accepted
    // against), or with rule 1 the initial GMRES residual (the step-0 kernel takes it
    // when bref2 is null)
    S.bref2 = rule == 1 ? nullptr : W.scal2 + 2 * nrhs;
    rc = run_phase(c, use_graph, 1, S, nrhs, kind, tr, PREC_F64, PREC_F64, o.tol, s, [&](hipStream_t q) {
      pre_body(q);
      gm_prologue(c, S, kind, tr, W.bhat, nrhs, o.tol, q, true, sides_ok);  // |b_hat|^2 (and sides) with b_hat
    });
    if (rc) return rc;
    mark(1);
    // the post-processing touches no Arnoldi state (it forms its residual terms without
    // a scratch vector), so the loop may queue it behind the chunk it predicts to be
    // the last
    const std::function<int()> post = [&]() -> int {
      mark(2);
      const int r = run_phase(c, use_graph, 2, S, nrhs, kind, tr, PREC_F64, PREC_F64, o.tol, s, [&](hipStream_t q) {
        PublishSet hist = {};
        gm_epilogue(c, S, kind, tr, W.x, nrhs, q, &hist);
        recover_x(c, kind, tr, W.bhat, W.x, W.bS, nrhs, PREC_F64, PREC_F64, q);
        // |b_hat|^2 is the prologue's stopping reference (the same reduction of b_hat)
        true_residual_enqueue(c, tr, W.bhat, W.bS, nrhs, q, W.scal2 + 2 * nrhs, removed, &hist);
        post_body(W.bS, q);
      });
      if (r) return r;
      store_u(s);
      return SMPM_OK;
    };
    bool post_done = false;
    rc = gm_loop(c, S, kind, tr, nrhs, o.maxit, s, PREC_F64, PREC_F64, use_graph, &post, &post_done);
    if (rc) return rc;
    if (!post_done) {
      rc = post();
      if (rc) return rc;
    }
    HIPCHK(hipStreamSynchronize(s));
    gm_collect(c, nrhs, o.maxit, o.tol, iters);
    note_cycle(iters);
    true_residual_read(c, nrhs, tres);
    // The least-squares estimate met tol, but the FP64 true residual decides.  Where it
    // misses tol by rounding (finite, iterations left), FP64 correction cycles
    // x += GMRES(b_hat - S x) bring it down (at most two); u is then formed again.
    bool corrected = false;
    for (int extra = 0; extra < 2; ++extra) {
      double worst = 0.0;
      bool fixable = true, any = false;
      for (int i = 0; i < nrhs; ++i) {
        if (tres[i] <= o.tol) continue;
        any = true;
        if (!std::isfinite(tres[i]) || iters[i] >= o.maxit) fixable = false;
        worst = std::max(worst, tres[i]);
      }
      if (!any || !fixable) break;
      launch_copy(W.bS, W.xacc, Pl.k * nrhs, s);
      launch_schur(P, W.xacc, W.t, nrhs, tr, nullptr, s);
      launch_add(W.bhat, W.t, -1.0, W.rho, Pl.k, nrhs, s);
      const double* nl = tr ? c->v0hat : c->uS;
      launch_mdot(nl, 0, 0, 1, W.rho, Pl.k, nullptr, Pl.k, nrhs, W.part, W.scal, nullptr, s);
      launch_axpy_shared(W.rho, Pl.k, nl, W.scal, 1.0, W.rho, Pl.k, nrhs, s);
      std::vector<int> it;
      rc = solve_schur(c, kind, tr, W.rho, W.bS, nrhs, std::min(0.5, 0.3 * o.tol / worst), o.maxit, it, s,
                       PREC_F64, PREC_F64, use_graph, rule);
      if (rc < 0) return rc;
      note_cycle(it);
      for (int i = 0; i < nrhs; ++i) iters[i] += it[i];
      launch_add(W.xacc, W.bS, 1.0, W.bS, Pl.k, nrhs, s);
      ++cycles;
      corrected = true;
      rc = true_residual(c, tr, W.bhat, W.bS, nrhs, tres, s);
      if (rc) return rc;
    }
    for (int i = 0; i < nrhs; ++i)
      if (!(tres[i] <= o.tol)) conv = false;  // NaN counts as not converged
    if (corrected) {
      post_body(W.bS, s);
      store_u(s);
    }
  } else {
    rc = run_phase(c, use_graph, 1, gm_state(c, nrhs, o.maxit), nrhs, 0, tr, PREC_F64, PREC_F64, 0.0, s,
                   [&](hipStream_t q) { pre_body(q); });
    if (rc) return rc;
    mark(1);
    // Iterative refinement: rho = b_hat - S x in FP64; delta from the deflated GMRES with
    // FP32 (or BF16) Schur and block-Jacobi operators; x += delta.
    //  * Inner tolerance: the reduction that finishes the solve when one cycle can
    //    attain it (see there), else inner_tol; never further than the outer stop needs.
    //  * Basis: with FP32 / BF16 operators the inner solve stores its Krylov basis in
    //    FP32 (its arithmetic stays FP64): half the basis traffic of a step.
    //  * Null space: rho is projected off the left null vector before every inner solve
    //    (see there).
    //  * Precision: the attainable accuracy of a cycle is set by the Schur operator's
    //    rounding times the conditioning of S (the preconditioner's precision only changes
    //    the convergence rate: GMRES minimizes the residual of S M^{-1} with the same
    //    M^{-1} that forms delta).  So a cycle that contracts the FP64 residual too little
    //    raises the Schur precision for the remaining cycles (BF16 -> FP32 below 20x,
    //    FP32 -> FP64 below 2x), and a cycle that makes it grow is undone (x returns to
    //    the previous iterate) before the precision is raised.
    int sprec = o.precision == SMPM_MIXED_FP32 ? PREC_F32 : PREC_BF16;
    const int mprec = sprec;
    HIPCHK(hipMemsetAsync(W.xacc, 0, sizeof(double) * Pl.k * nrhs, s));
    HIPCHK(hipMemcpyAsync(W.rho, W.bhat, sizeof(double) * Pl.k * nrhs, hipMemcpyDeviceToDevice, s));
    iters.assign(nrhs, 0);
    std::vector<double> prev(nrhs, 2.0);
    double cprev = HUGE_VAL;  // largest column residual at the iterate in xprev
    bool reverted = false;
    int stall = 0;
    tres.assign(nrhs, 1.0);
    conv = false;
    for (cycles = 0; cycles <= o.max_refine; ++cycles) {
      if (cycles > 0) {
        launch_schur(P, W.xacc, W.t, nrhs, tr, nullptr, s);
        launch_add(W.bhat, W.t, -1.0, W.rho, Pl.k, nrhs, s);
      }
      launch_mdot(W.rho, 0, Pl.k, 1, W.rho, Pl.k, nullptr, Pl.k, nrhs, W.part, W.scal, nullptr, s);
      launch_mdot(W.bhat, 0, Pl.k, 1, W.bhat, Pl.k, nullptr, Pl.k, nrhs, W.part, W.scal2, nullptr, s);
      launch_publish(W.scal, nrhs, W.hout, s);
      launch_publish(W.scal2, nrhs, W.hout + nrhs, s);
      HIPCHK(hipStreamSynchronize(s));
      const double* a = W.hout;
      const double* bb = W.hout + nrhs;
      bool all = true, finite = true;
      double cmax = 0;
      for (int i = 0; i < nrhs; ++i) {
        tres[i] = bb[i] > 0 ? std::sqrt(a[i] / bb[i]) : std::sqrt(a[i]);
        if (!std::isfinite(tres[i])) finite = false;
        cmax = std::max(cmax, tres[i]);
        if (!(tres[i] <= o.tol)) all = false;
      }
      if (cycles < 16) hist[cycles] = finite ? cmax : NAN;
      if (all) {
        conv = true;
        break;
      }
      if (!finite) break;  // a non-finite residual cannot be refined
      if (cycles > 0 && !reverted && cmax > cprev) {
        // the last correction made the residual grow: undo it, raise the precision
        HIPCHK(hipMemcpyAsync(W.xacc, W.xprev, sizeof(double) * Pl.k * nrhs, hipMemcpyDeviceToDevice, s));
        if (sprec == PREC_F64) break;
        sprec = sprec == PREC_BF16 ? PREC_F32 : PREC_F64;
        reverted = true;
        continue;  // the next pass recomputes the residual of the restored iterate
      }
      bool weak = false, slow = false;
      for (int i = 0; i < nrhs; ++i) {
        if (tres[i] <= o.tol) {
          // converged column: zero residual so the inner solve leaves it alone
          HIPCHK(hipMemsetAsync(W.rho + (size_t)i * Pl.k, 0, sizeof(double) * Pl.k, s));
        } else if (cycles >= 1 && !reverted) {
          if (tres[i] > 0.05 * prev[i]) weak = true;
          if (tres[i] > 0.5 * prev[i]) slow = true;
        }
        prev[i] = tres[i];
      }
      reverted = false;
      // raise the Schur precision after a weak cycle; two cycles without a 2x
      // contraction at FP64 end the loop
      if (weak && sprec == PREC_BF16) {
        sprec = PREC_F32;
        slow = false;
      } else if (slow && sprec == PREC_F32) {
        sprec = PREC_F64;
        slow = false;
      }
      stall = slow ? stall + 1 : 0;
      if (stall >= 2 || cycles == o.max_refine) break;
      cprev = cmax;
      HIPCHK(hipMemcpyAsync(W.xprev, W.xacc, sizeof(double) * Pl.k * nrhs, hipMemcpyDeviceToDevice, s));
      // rho lies in the range of S (of S^T for the adjoint) only up to the rounding of
      // b_hat - S x, a component along the left null vector of about eps |b_hat| that
      // no correction can remove; once |rho| is small it is a sizeable part of rho and
      // the inner GMRES, fitting it, grows a large correction along the right null
      // direction, which the rounding of the low-precision operators turns into residual
      {
        const double* nl = tr ? c->v0hat : c->uS;
        launch_mdot(nl, 0, 0, 1, W.rho, Pl.k, nullptr, Pl.k, nrhs, W.part, W.scal, nullptr, s);
        launch_axpy_shared(W.rho, Pl.k, nl, W.scal, 1.0, W.rho, Pl.k, nrhs, s);
      }
      // inner tolerance: the reduction that finishes the solve (0.3 tol / rho_max) when
      // one cycle at this precision can attain it, else inner_tol (looser than inner_tol
      // near the target, tighter one cycle before it).  Attainable with FP32 operators:
      // 1e-7 for the batched inner solve; 1e-6 for block GMRES, whose FP32 basis holds
      // every column's vectors in one space (an aim of 3e-7 ran its cycle to maxit); with
      // BF16 operators 1e-3.  Aiming lower only lengthens a cycle or stalls it.
      const double need = 0.3 * o.tol / cmax;
      const double reach = sprec == PREC_BF16 ? 1e-3 : sprec == PREC_F32 ? (o.block ? 1e-6 : 1e-7) : 1e-12;
      const double itol = std::min(0.5, need >= reach ? need : std::max(o.inner_tol, need));
      std::vector<int> it;
      if (o.block) {
        // block GMRES as the inner solve: all columns in one block Krylov space
        // (stopping reference |rho| per column, as the batched inner solve takes it)
        rc = ensure_bws(c, nrhs, o.maxit);
        if (rc) return rc;
        if (rule != 1)
          launch_mdot(W.rho, 0, Pl.k, 1, W.rho, Pl.k, nullptr, Pl.k, nrhs, W.part, W.scal2 + 2 * nrhs, nullptr, s);
        const int st = block_solve_schur(c, kind, tr, W.rho, W.bS, nrhs, itol, o.maxit,
                                         rule == 1 ? nullptr : W.scal2 + 2 * nrhs, s, nullptr, sprec, mprec);
        if (st < 0) return st;
        it.assign(nrhs, st);
        rc = st;
      } else {
        rc = solve_schur(c, kind, tr, W.rho, W.bS, nrhs, itol, o.maxit, it, s, sprec, mprec, o.graph != 0, rule);
      }
      if (rc < 0) return rc;
      note_cycle(it);
      sprec_final = sprec;
      for (int i = 0; i < nrhs; ++i) iters[i] += it[i];
      launch_add(W.xacc, W.bS, 1.0, W.xacc, Pl.k, nrhs, s);
    }
    mark(2);
    post_body(W.xacc, s);
    store_u(s);
    launch_publish(removed, nrhs, W.hout + 2 * nrhs, s);
  }
  mark(3);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(s));
  float pms[3] = {0, 0, 0};
  if (profile) {
    for (int i = 0; i < 3; ++i) (void)hipEventElapsedTime(&pms[i], pev[i], pev[i + 1]);
    for (auto& e : pev) (void)hipEventDestroy(e);
  }
  int itmax = 0;
  double resmax = 0;
  for (int i = 0; i < nrhs; ++i) {
    itmax = std::max(itmax, iters[i]);
    resmax = std::isnan(tres[i]) || std::isnan(resmax) ? NAN : std::max(resmax, tres[i]);
  }
  if (info) {
    info->iterations = itmax;
    info->refinements = cycles;
    info->schur_precision = sprec_final;
    for (int q = 0; q < 16; ++q) info->cycle_residual[q] = hist[q];
    if (o.precision == SMPM_FP64) info->cycle_residual[0] = resmax;
    info->rel_residual = resmax;
    // published before the synchronization above; the adjoint removes a multiple of w
    info->removed_component = W.hout[2 * nrhs] / (tr ? c->wsum : 1.0);
    const double ref = *W.hhist_tolb / W.hist_tol;
    // the estimate after i steps was g_i when step i set it; the rotation of step i + 1
    // has since multiplied it by that rotation's cosine (the last entry is unrotated)
    info->history_len = W.hist_len;
    for (int i = 0; i < 1001; ++i) {
      double v = 0.0;
      if (i < W.hist_len && ref > 0) {
        v = std::fabs(W.hhist[i]);
        if (i + 1 < W.hist_len && W.hhist_cs[i] != 0.0) v /= std::fabs(W.hhist_cs[i]);
        v /= ref;
      }
      info->history[i] = v;
    }
    for (int i = 0; i < 16; ++i) info->cycle_iterations[i] = cyc_it[i];
    for (int i = 0; i < 3; ++i) info->phase_ms[i] = pms[i];
    info->phase_ms[3] = pms[0] + pms[1] + pms[2];
  }
  if (*W.hnonfinite)
    return fail(SMPM_EINVAL, tr ? "the cotangent holds a non-finite entry" : "f or g holds a non-finite entry");
  if (!conv)
    return fail(SMPM_ENOCONV, o.precision == SMPM_FP64
                                  ? "the FP64 true residual missed the tolerance (GMRES reached maxit or stalled)"
                                  : "iterative refinement did not reach the tolerance");
  return SMPM_OK;
}

}  // extern "C"
