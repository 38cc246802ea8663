// Host FP64 setup of the SMPM Schur complement solver.
//
// Discretization (Sec. 1.2, Eq. smpm_poisson): on each element the collocated
// Laplacian plus, at the nodes of each side, tau (u + sigma n.grad u) - tau (u_j +
// sigma n.grad u_j) across an inter-element side, or tau sigma n.grad u on a
// physical side (receiving element's values for both u_i and u_j).  Three readings
// of the Robin length sigma and the penalty tau (h_perp = the element's extent
// normal to the side, h_e = its smaller extent, omega_0 the GLL end weight):
//   literal    sigma = 1,          tau = 2 alpha / (omega_0 h_perp)   (R = I + n.grad)
//   reference  sigma = h_perp / 2, tau = 2 alpha / (omega_0 h_perp^2)
//   min        sigma = h_e / 2,    tau = 2 alpha / (omega_0 h_e^2)    (default)
// Split (Sec. 1.3): A = the element-local part, B = the neighbour flux of each
// side slot, E = slot -> node inclusion, S = I + B A^{-1} E.  Each distinct
// element class stores A^{-1} and the outgoing side fluxes W = R A^{-1} E
// (R = -tau_recv (trace - sigma_recv n_own.grad)) used by the Schur apply.
#include "smpm_plan.h"

#include <algorithm>
#include <cmath>
#include <map>
#include <thread>
#include <tuple>

namespace smpm {

// ---------------------------------------------------------------- dense LU

bool lu_factor(std::vector<double>& a, int m, std::vector<int>& piv, double min_pivot) {
  piv.assign(m, 0);
  for (int k = 0; k < m; ++k) {
    int p = k;
    double best = std::fabs(a[(size_t)k * m + k]);
    for (int i = k + 1; i < m; ++i) {
      double v = std::fabs(a[(size_t)i * m + k]);
      if (v > best) { best = v; p = i; }
    }
    piv[k] = p;
    if (!(best > min_pivot) || !std::isfinite(best)) return false;
    if (p != k)
      for (int j = 0; j < m; ++j) std::swap(a[(size_t)k * m + j], a[(size_t)p * m + j]);
    const double inv = 1.0 / a[(size_t)k * m + k];
    const double* rk = &a[(size_t)k * m];
    for (int i = k + 1; i < m; ++i) {
      double* ri = &a[(size_t)i * m];
      const double f = ri[k] * inv;
      ri[k] = f;
      if (f != 0.0)
        for (int j = k + 1; j < m; ++j) ri[j] -= f * rk[j];
    }
  }
  return true;
}

void lu_solve(const std::vector<double>& a, int m, const std::vector<int>& piv, double* b) {
  for (int k = 0; k < m; ++k) std::swap(b[k], b[piv[k]]);
  for (int i = 0; i < m; ++i) {
    double s = b[i];
    const double* ri = &a[(size_t)i * m];
    for (int j = 0; j < i; ++j) s -= ri[j] * b[j];
    b[i] = s;
  }
  for (int i = m - 1; i >= 0; --i) {
    double s = b[i];
    const double* ri = &a[(size_t)i * m];
    for (int j = i + 1; j < m; ++j) s -= ri[j] * b[j];
    b[i] = s / ri[i];
  }
}

bool dense_inverse(const std::vector<double>& a_in, int m, std::vector<double>& inv, double min_rel_pivot) {
  std::vector<double> a = a_in;
  std::vector<int> piv;
  double amax = 0.0;
  for (double v : a) amax = std::max(amax, std::fabs(v));
  if (!lu_factor(a, m, piv, min_rel_pivot * amax)) return false;
  inv.assign((size_t)m * m, 0.0);
  unsigned nth = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  if ((int64_t)m * m * m < (int64_t)1 << 24) nth = 1;
  std::vector<std::thread> pool;
  for (unsigned t = 0; t < nth; ++t) {
    pool.emplace_back([&, t]() {
      std::vector<double> col(m);
      for (int j = (int)t; j < m; j += (int)nth) {
        std::fill(col.begin(), col.end(), 0.0);
        col[j] = 1.0;
        lu_solve(a, m, piv, col.data());
        for (int i = 0; i < m; ++i) inv[(size_t)i * m + j] = col[i];
      }
    });
  }
  for (auto& th : pool) th.join();
  return true;
}

// Generalized inverse of a square matrix with one-dimensional null spaces whose
// right null vector `rn` is known: the left null vector ln solves the bordered
// system [[A^T, rn], [rn^T, 0]] [ln; mu] = [0; 1]; then the top-left block of
// [[A, ln], [rn^T, 0]]^{-1} is the Moore-Penrose inverse (its range is
// orthogonal to rn and it annihilates ln).
static bool bordered_pinv(const std::vector<double>& A, int m, const std::vector<double>& rn,
                          std::vector<double>& ginv, std::vector<double>& ln) {
  const int mb = m + 1;
  std::vector<double> K((size_t)mb * mb, 0.0);
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < m; ++j) K[(size_t)i * mb + j] = A[(size_t)j * m + i];
  for (int i = 0; i < m; ++i) {
    K[(size_t)i * mb + m] = rn[i];
    K[(size_t)m * mb + i] = rn[i];
  }
  std::vector<int> piv;
  if (!lu_factor(K, mb, piv)) return false;
  std::vector<double> rhs(mb, 0.0);
  rhs[m] = 1.0;
  lu_solve(K, mb, piv, rhs.data());
  ln.assign(rhs.begin(), rhs.begin() + m);
  double nn = 0;
  for (double v : ln) nn += v * v;
  nn = std::sqrt(nn);
  double sum = 0;
  for (double v : ln) sum += v;
  const double sg = sum < 0 ? -1.0 : 1.0;
  for (double& v : ln) v *= sg / nn;
  std::fill(K.begin(), K.end(), 0.0);
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < m; ++j) K[(size_t)i * mb + j] = A[(size_t)i * m + j];
  for (int i = 0; i < m; ++i) {
    K[(size_t)i * mb + m] = ln[i];
    K[(size_t)m * mb + i] = rn[i];
  }
  std::vector<double> Kinv;
  if (!dense_inverse(K, mb, Kinv)) return false;
  ginv.assign((size_t)m * m, 0.0);
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < m; ++j) ginv[(size_t)i * m + j] = Kinv[(size_t)i * mb + j];
  return true;
}

// ---------------------------------------------------------------- GLL

// Gauss-Lobatto-Legendre nodes by Newton iteration on the Legendre-Vandermonde
// recurrence started from the Chebyshev-Gauss-Lobatto points (the classical
// "lglnodes" construction); weights 2/(N(N+1) P_N(x)^2); differentiation matrix
// from barycentric weights with the negative-sum diagonal.
static void gll(int n, std::vector<double>& x, std::vector<double>& w, std::vector<double>& D) {
  const int N = n - 1;
  x.assign(n, 0.0);
  for (int i = 0; i < n; ++i) x[i] = -std::cos(M_PI * i / N);
  std::vector<double> P((size_t)n * n, 0.0), xold(n);
  for (int it = 0; it < 200; ++it) {
    xold = x;
    for (int i = 0; i < n; ++i) {
      double* Pi = &P[(size_t)i * n];
      Pi[0] = 1.0;
      Pi[1] = x[i];
      for (int k = 2; k <= N; ++k) Pi[k] = ((2 * k - 1) * x[i] * Pi[k - 1] - (k - 1) * Pi[k - 2]) / k;
    }
    double diff = 0;
    for (int i = 0; i < n; ++i) {
      const double* Pi = &P[(size_t)i * n];
      x[i] = xold[i] - (x[i] * Pi[N] - Pi[N - 1]) / (n * Pi[N]);
      diff = std::max(diff, std::fabs(x[i] - xold[i]));
    }
    if (diff < 1e-16 && it > 2) break;
  }
  for (int i = 0; i < n; ++i) {
    double* Pi = &P[(size_t)i * n];
    Pi[0] = 1.0;
    Pi[1] = x[i];
    for (int k = 2; k <= N; ++k) Pi[k] = ((2 * k - 1) * x[i] * Pi[k - 1] - (k - 1) * Pi[k - 2]) / k;
  }
  x[0] = -1.0;
  x[N] = 1.0;
  w.assign(n, 0.0);
  for (int i = 0; i < n; ++i) w[i] = 2.0 / (N * n * P[(size_t)i * n + N] * P[(size_t)i * n + N]);
  std::vector<double> lam(n, 1.0);
  for (int j = 0; j < n; ++j) {
    double prod = 1.0;
    for (int k = 0; k < n; ++k)
      if (k != j) prod *= (x[j] - x[k]);
    lam[j] = 1.0 / prod;
  }
  D.assign((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) {
    double s = 0;
    for (int j = 0; j < n; ++j) {
      if (j == i) continue;
      const double v = (lam[j] / lam[i]) / (x[i] - x[j]);
      D[(size_t)i * n + j] = v;
      s += v;
    }
    D[(size_t)i * n + i] = -s;
  }
}

// ---------------------------------------------------------------- helpers

static inline int side_node(int n, int s, int t) {
  switch (s) {
    case SW: return t * n;
    case SE: return t * n + (n - 1);
    case SS: return t;
    default: return (n - 1) * n + t;
  }
}

// Row of the outward normal derivative at node t of side s: coefficients and
// the local node they multiply (n entries).
static void outward_derivative(const Plan& p, double w, double h, int s, int t,
                               std::vector<int>& col, std::vector<double>& val) {
  const int n = p.n, N = n - 1;
  col.resize(n);
  val.resize(n);
  for (int a = 0; a < n; ++a) {
    switch (s) {
      case SW: col[a] = t * n + a; val[a] = -(2.0 / w) * p.D[a]; break;
      case SE: col[a] = t * n + a; val[a] = (2.0 / w) * p.D[(size_t)N * n + a]; break;
      case SS: col[a] = a * n + t; val[a] = -(2.0 / h) * p.D[a]; break;
      default: col[a] = a * n + t; val[a] = (2.0 / h) * p.D[(size_t)N * n + a]; break;
    }
  }
}

// A_e of one class (row-major n2 x n2): the element-local part of Eq. smpm_poisson.
static std::vector<double> local_matrix(const Plan& p, const ElementClass& c) {
  const int n = p.n, n2 = n * n;
  std::vector<double> D2((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      double s = 0;
      for (int k = 0; k < n; ++k) s += p.D[(size_t)i * n + k] * p.D[(size_t)k * n + j];
      D2[(size_t)i * n + j] = s;
    }
  std::vector<double> A((size_t)n2 * n2, 0.0);
  const double cx = 4.0 / (c.w * c.w), cy = 4.0 / (c.h * c.h);
  for (int q = 0; q < n; ++q)
    for (int pp = 0; pp < n; ++pp) {
      const int l = q * n + pp;
      for (int a = 0; a < n; ++a) A[(size_t)l * n2 + q * n + a] += cx * D2[(size_t)pp * n + a];
      for (int b = 0; b < n; ++b) A[(size_t)l * n2 + b * n + pp] += cy * D2[(size_t)q * n + b];
    }
  std::vector<int> col;
  std::vector<double> val;
  for (int s = 0; s < 4; ++s) {
    const bool inter = (c.mask >> s) & 1;
    const double tau = c.tau_own[s], tsig = c.tau_own[s] * c.sig_own[s];
    for (int t = 0; t < n; ++t) {
      const int l = side_node(n, s, t);
      outward_derivative(p, c.w, c.h, s, t, col, val);
      for (int a = 0; a < n; ++a) A[(size_t)l * n2 + col[a]] += tsig * val[a];
      if (inter) A[(size_t)l * n2 + l] += tau;
    }
  }
  return A;
}

// ---------------------------------------------------------------- plan

std::string build_plan(Plan& p, int m_y, int m_x, int n, const double* xb, const double* yb,
                       double alpha, int robin) {
  if (m_x < 1 || m_y < 1 || (int64_t)m_x * m_y < 2) return "need at least two elements";
  if (n < 3 || n > 32) return "n must be in [3, 32]";
  if (!xb || !yb) return "null breakpoints";
  if (!std::isfinite(alpha) || alpha == 0.0) return "penalty must be finite and nonzero";
  if (robin != kRobinMin && robin != kRobinLiteral && robin != kRobinReference) return "unknown Robin mode";
  for (int i = 0; i < m_x; ++i)
    if (!(xb[i + 1] > xb[i]) || !std::isfinite(xb[i]) || !std::isfinite(xb[i + 1]))
      return "x breakpoints must be finite and strictly increasing";
  for (int i = 0; i < m_y; ++i)
    if (!(yb[i + 1] > yb[i]) || !std::isfinite(yb[i]) || !std::isfinite(yb[i + 1]))
      return "y breakpoints must be finite and strictly increasing";
  p = Plan();
  p.n = n;
  p.mx = m_x;
  p.my = m_y;
  p.nel = m_x * m_y;
  p.r = (int64_t)n * n * p.nel;
  p.alpha = alpha;
  p.robin = robin;
  p.xb.assign(xb, xb + m_x + 1);
  p.yb.assign(yb, yb + m_y + 1);
  gll(n, p.xi, p.omega, p.D);
  const int N = n - 1, n2 = n * n;
  // element extents; extents that agree to 1e-12 relative share one value so that
  // equal elements share a class and matching interfaces get bitwise-equal penalties
  auto canon = [](const std::vector<double>& br, int m) {
    std::vector<double> out(m), seen;
    for (int i = 0; i < m; ++i) {
      const double v = br[i + 1] - br[i];
      double c = v;
      for (double u : seen)
        if (std::fabs(u - v) <= 1e-12 * std::fabs(u)) { c = u; break; }
      if (c == v) seen.push_back(v);
      out[i] = c;
    }
    return out;
  };
  p.wx = canon(p.xb, m_x);
  p.hy = canon(p.yb, m_y);
  const double omega0 = p.omega[0];

  // elements, sides, slots
  p.mask.assign(p.nel, 0);
  p.nbr.assign((size_t)p.nel * 4, -1);
  p.side_slot.assign((size_t)p.nel * 4, -1);
  p.iface.assign((size_t)p.nel * 4, -1);
  p.slot_off.assign(p.nel + 1, 0);
  for (int iy = 0; iy < m_y; ++iy)
    for (int ix = 0; ix < m_x; ++ix) {
      const int e = iy * m_x + ix;
      const int nb[4] = {ix > 0 ? e - 1 : -1, ix < m_x - 1 ? e + 1 : -1,
                         iy > 0 ? e - m_x : -1, iy < m_y - 1 ? e + m_x : -1};
      for (int s = 0; s < 4; ++s) {
        p.nbr[(size_t)e * 4 + s] = nb[s];
        if (nb[s] >= 0) p.mask[e] |= 1 << s;
      }
    }
  int64_t nsides = 0;
  for (int e = 0; e < p.nel; ++e) {
    p.slot_off[e] = (int)(nsides * n);
    for (int s = 0; s < 4; ++s)
      if ((p.mask[e] >> s) & 1) {
        p.side_slot[(size_t)e * 4 + s] = (int)(nsides * n);
        p.side_elem.push_back(e);
        p.side_dir.push_back(s);
        ++nsides;
      }
  }
  p.slot_off[p.nel] = (int)(nsides * n);
  p.nsides = nsides;
  p.k = nsides * n;
  if (p.k > ((int64_t)1 << 30)) return "grid too large";

  // interfaces
  int64_t d = 0;
  for (int iy = 0; iy < m_y; ++iy)
    for (int ix = 0; ix + 1 < m_x; ++ix) {
      const int a = iy * m_x + ix, b = a + 1;
      p.iface[(size_t)a * 4 + SE] = (int)d;
      p.iface[(size_t)b * 4 + SW] = (int)d;
      p.iface_side.push_back(p.side_slot[(size_t)a * 4 + SE] / n);
      p.iface_side.push_back(p.side_slot[(size_t)b * 4 + SW] / n);
      ++d;
    }
  for (int iy = 0; iy + 1 < m_y; ++iy)
    for (int ix = 0; ix < m_x; ++ix) {
      const int a = iy * m_x + ix, b = a + m_x;
      p.iface[(size_t)a * 4 + SN] = (int)d;
      p.iface[(size_t)b * 4 + SS] = (int)d;
      p.iface_side.push_back(p.side_slot[(size_t)a * 4 + SN] / n);
      p.iface_side.push_back(p.side_slot[(size_t)b * 4 + SS] / n);
      ++d;
    }
  p.d = d;

  // penalty tau and Robin length sigma (R = I + sigma n.grad) of side s of element e
  auto normal_len = [&](int e, int s) { return s == SW || s == SE ? p.wx[e % m_x] : p.hy[e / m_x]; };
  auto elem_len = [&](int e) { return std::min(p.wx[e % m_x], p.hy[e / m_x]); };
  auto tau_of = [&](int e, int s) {
    if (robin == kRobinLiteral) return 2.0 * alpha / (omega0 * normal_len(e, s));
    const double l = robin == kRobinReference ? normal_len(e, s) : elem_len(e);
    return 2.0 * alpha / (omega0 * l * l);
  };
  auto sig_of = [&](int e, int s) {
    if (robin == kRobinLiteral) return 1.0;
    return 0.5 * (robin == kRobinReference ? normal_len(e, s) : elem_len(e));
  };
  p.side_tau.assign((size_t)p.nel * 4, 0.0);
  p.side_sig.assign((size_t)p.nel * 4, 0.0);
  for (int e = 0; e < p.nel; ++e)
    for (int s = 0; s < 4; ++s) {
      p.side_tau[(size_t)e * 4 + s] = tau_of(e, s);
      p.side_sig[(size_t)e * 4 + s] = sig_of(e, s);
    }

  // element classes
  std::map<std::tuple<double, double, int, double, double, double, double, std::tuple<double, double, double, double>>,
           int>
      key2cls;
  p.cls.assign(p.nel, -1);
  for (int e = 0; e < p.nel; ++e) {
    const int ix = e % m_x, iy = e / m_x;
    ElementClass c;
    c.w = p.wx[ix];
    c.h = p.hy[iy];
    c.mask = p.mask[e];
    for (int s = 0; s < 4; ++s) {
      c.tau_own[s] = tau_of(e, s);
      c.sig_own[s] = sig_of(e, s);
      const int j = p.nbr[(size_t)e * 4 + s];
      c.tau_recv[s] = j >= 0 ? tau_of(j, opposite(s)) : 0.0;
      c.sig_recv[s] = j >= 0 ? sig_of(j, opposite(s)) : 0.0;
    }
    auto key = std::make_tuple(c.w, c.h, c.mask, c.tau_recv[0], c.tau_recv[1], c.tau_recv[2], c.tau_recv[3],
                               std::make_tuple(c.sig_recv[0], c.sig_recv[1], c.sig_recv[2], c.sig_recv[3]));
    auto it = key2cls.find(key);
    if (it == key2cls.end()) {
      int col = 0;
      for (int s = 0; s < 4; ++s)
        if ((c.mask >> s) & 1) {
          c.side_col[s] = col;
          col += n;
        }
      c.nslots = col;
      it = key2cls.emplace(key, (int)p.classes.size()).first;
      p.classes.push_back(c);
    }
    p.cls[e] = it->second;
  }

  // element groups: elements sorted by (class, id), cut into runs of one class
  {
    std::vector<int> order(p.nel);
    for (int e = 0; e < p.nel; ++e) order[e] = e;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return p.cls[a] < p.cls[b]; });
    auto cut = [&](int stride, int size, std::vector<int>& gcls, std::vector<int>& gelem) {
      for (int i = 0; i < p.nel;) {
        const int J = p.cls[order[i]];
        int cnt = 0;
        gcls.push_back(J);
        for (; i < p.nel && cnt < size && p.cls[order[i]] == J; ++i, ++cnt) gelem.push_back(order[i]);
        for (int u = cnt; u < stride; ++u) gelem.push_back(-1);
      }
      return (int)gcls.size();
    };
    // vector kernels: enough groups to occupy the chip (about 2048 wavefronts)
    p.grp_size = Plan::kGroup;
    while (p.grp_size > 1 && (p.nel + p.grp_size - 1) / p.grp_size < 2048) p.grp_size /= 2;
    p.ngrp = cut(Plan::kGroup, p.grp_size, p.grp_cls, p.grp_elem);
    // matrix-core tiles: 16 elements form the N side of a 16x16 product.  Narrower tiles
    // would give small grids more workgroups but not a shorter one (the product and
    // the loads per lane do not shrink), and they re-read the class operator per tile.
    p.tile_size = Plan::kTile;
    p.ntile = cut(Plan::kTile, p.tile_size, p.tile_cls, p.tile_elem);
  }

  // class operators
  const int ncls = (int)p.classes.size();
  p.Ainv.assign((size_t)ncls * n2 * n2, 0.0);
  p.AinvT.assign((size_t)ncls * n2 * n2, 0.0);
  p.W_off.assign((size_t)ncls * 4, -1);
  p.H_off.assign((size_t)ncls * 4, -1);
  p.WZ.assign((size_t)ncls * 4 * n * 4, 0.0);
  int64_t wtot = 0, htot = 0;
  for (int J = 0; J < ncls; ++J)
    for (int s = 0; s < 4; ++s)
      if ((p.classes[J].mask >> s) & 1) {
        p.W_off[(size_t)J * 4 + s] = wtot;
        wtot += (int64_t)n * p.classes[J].nslots;
        p.H_off[(size_t)J * 4 + s] = htot;
        htot += (int64_t)n * n2;
      }
  p.Wc.assign(wtot, 0.0);
  p.Wr.assign(wtot, 0.0);
  p.Hc.assign(htot, 0.0);
  p.Hr.assign(htot, 0.0);
  std::vector<int> col;
  std::vector<double> val;
  for (int J = 0; J < ncls; ++J) {
    const ElementClass& c = p.classes[J];
    std::vector<double> A = local_matrix(p, c), Ai;
    if (!dense_inverse(A, n2, Ai)) return "singular element matrix";
    std::copy(Ai.begin(), Ai.end(), p.Ainv.begin() + (size_t)J * n2 * n2);
    for (int l = 0; l < n2; ++l)
      for (int m = 0; m < n2; ++m) p.AinvT[(size_t)J * n2 * n2 + (size_t)m * n2 + l] = Ai[(size_t)l * n2 + m];
    // slot -> local node of this class
    std::vector<int> slot_node(c.nslots);
    std::vector<int> slot_side(c.nslots);
    for (int s = 0; s < 4; ++s)
      if (c.side_col[s] >= 0)
        for (int t = 0; t < n; ++t) {
          slot_node[c.side_col[s] + t] = side_node(n, s, t);
          slot_side[c.side_col[s] + t] = s;
        }
    for (int so = 0; so < 4; ++so) {
      if (!((c.mask >> so) & 1)) continue;
      // R = -tau_recv (trace - sigma_recv n_own.grad) at the nodes of side so; H = R A^{-1}
      std::vector<double> H((size_t)n * n2, 0.0);
      for (int i = 0; i < n; ++i) {
        std::vector<double> row(n2, 0.0);
        row[side_node(n, so, i)] += -c.tau_recv[so];
        outward_derivative(p, c.w, c.h, so, i, col, val);
        for (int a = 0; a < n; ++a) row[col[a]] += c.tau_recv[so] * c.sig_recv[so] * val[a];
        for (int l = 0; l < n2; ++l) {
          double acc = 0;
          for (int m = 0; m < n2; ++m) acc += row[m] * Ai[(size_t)m * n2 + l];
          H[(size_t)i * n2 + l] = acc;
        }
      }
      const int64_t ho = p.H_off[(size_t)J * 4 + so];
      for (int i = 0; i < n; ++i)
        for (int l = 0; l < n2; ++l) {
          p.Hr[ho + (size_t)i * n2 + l] = H[(size_t)i * n2 + l];
          p.Hc[ho + (size_t)l * n + i] = H[(size_t)i * n2 + l];
        }
      const int64_t wo = p.W_off[(size_t)J * 4 + so];
      for (int i = 0; i < n; ++i)
        for (int cc = 0; cc < c.nslots; ++cc) {
          const double v = H[(size_t)i * n2 + slot_node[cc]];
          p.Wr[wo + (size_t)i * c.nslots + cc] = v;
          p.Wc[wo + (size_t)cc * n + i] = v;
          p.WZ[(((size_t)J * 4 + so) * n + i) * 4 + slot_side[cc]] += v;
        }
    }
  }

  // matrix-core fragments of the class operators and the tiles' slot tables
  if (n <= 16) {
    p.mma_mt = (4 * n + 15) / 16;
    p.mma_kt = 4 * p.mma_mt;
    const int mt = p.mma_mt, kt = p.mma_kt;
    p.Afwd.assign((size_t)ncls * mt * kt * 64, 0.0);
    p.Aadj.assign((size_t)ncls * mt * kt * 64, 0.0);
    for (int J = 0; J < ncls; ++J) {
      const int ns = p.classes[J].nslots;
      for (int w = 0; w < mt; ++w)
        for (int q = 0; q < kt; ++q)
          for (int l = 0; l < 64; ++l) {
            const int m = 16 * w + l % 16, kk = 4 * q + l / 16;
            const size_t at = (((size_t)J * mt + w) * kt + q) * 64 + l;
            // forward: row m = node (s, i) of a receiving side, column kk = slot
            if (m < 4 * n && kk < ns) {
              const int64_t wo = p.W_off[(size_t)J * 4 + m / n];
              if (wo >= 0) p.Afwd[at] = p.Wc[wo + (size_t)kk * n + m % n];
            }
            // transpose: row m = slot, column kk = node (s, i)
            if (m < ns && kk < 4 * n) {
              const int64_t wo = p.W_off[(size_t)J * 4 + kk / n];
              if (wo >= 0) p.Aadj[at] = p.Wc[wo + (size_t)m * n + kk % n];
            }
          }
    }
  }
  p.tile_src.assign((size_t)p.ntile * Plan::kTile, -1);
  p.tile_dst.assign((size_t)p.ntile * Plan::kTile * 4, -1);
  for (int t = 0; t < p.ntile; ++t)
    for (int u = 0; u < Plan::kTile; ++u) {
      const int e = p.tile_elem[(size_t)t * Plan::kTile + u];
      if (e < 0) continue;
      p.tile_src[(size_t)t * Plan::kTile + u] = p.slot_off[e];
      for (int s = 0; s < 4; ++s) {
        const int j = p.nbr[(size_t)e * 4 + s];
        if (j >= 0) p.tile_dst[((size_t)t * Plan::kTile + u) * 4 + s] = p.side_slot[(size_t)j * 4 + (s ^ 1)];
      }
    }

  // v0 = B 1: every slot of side s of element e holds -tau_{e,s}
  p.v0.assign(p.k, 0.0);
  for (int64_t si = 0; si < p.nsides; ++si) {
    const double t = tau_of(p.side_elem[si], p.side_dir[si]);
    for (int i = 0; i < n; ++i) p.v0[si * n + i] = -t;
  }

  // block-Jacobi blocks: red element slots, then the facing slots of its neighbours
  std::map<std::tuple<int, int, int, int, int>, int> bkey;
  std::vector<std::vector<double>> bmats;
  p.blk_off.push_back(0);
  for (int e = 0; e < p.nel; ++e) {
    const int ix = e % m_x, iy = e / m_x;
    if ((ix + iy) % 2) continue;
    const ElementClass& ce = p.classes[p.cls[e]];
    const int ns = ce.nslots;
    for (int cc = 0; cc < ns; ++cc) p.blk_slots.push_back(p.slot_off[e] + cc);
    for (int s = 0; s < 4; ++s) {
      const int j = p.nbr[(size_t)e * 4 + s];
      if (j < 0) continue;
      const int base = p.side_slot[(size_t)j * 4 + opposite(s)];
      for (int t = 0; t < n; ++t) p.blk_slots.push_back(base + t);
    }
    p.blk_red.push_back(e);
    p.blk_off.push_back((int)p.blk_slots.size());
    const int* nb = &p.nbr[(size_t)e * 4];
    auto key = std::make_tuple(p.cls[e], nb[0] >= 0 ? p.cls[nb[0]] : -1, nb[1] >= 0 ? p.cls[nb[1]] : -1,
                               nb[2] >= 0 ? p.cls[nb[2]] : -1, nb[3] >= 0 ? p.cls[nb[3]] : -1);
    auto it = bkey.find(key);
    if (it == bkey.end()) {
      const int sb = 2 * ns;
      std::vector<double> M((size_t)sb * sb, 0.0);
      for (int i = 0; i < sb; ++i) M[(size_t)i * sb + i] = 1.0;
      int pos = ns;
      for (int s = 0; s < 4; ++s) {
        const int j = nb[s];
        if (j < 0) continue;
        const ElementClass& cj = p.classes[p.cls[j]];
        const int so = opposite(s);
        // rows of e's side s (receiver) x columns of j's side so
        const int64_t wj = p.W_off[(size_t)p.cls[j] * 4 + so];
        for (int t = 0; t < n; ++t)
          for (int u = 0; u < n; ++u)
            M[(size_t)(ce.side_col[s] + t) * sb + pos + u] = p.Wr[wj + (size_t)t * cj.nslots + cj.side_col[so] + u];
        // rows of j's side so (receiver) x columns of all of e's slots
        const int64_t we = p.W_off[(size_t)p.cls[e] * 4 + s];
        for (int t = 0; t < n; ++t)
          for (int cc = 0; cc < ns; ++cc) M[(size_t)(pos + t) * sb + cc] = p.Wr[we + (size_t)t * ns + cc];
        pos += n;
      }
      std::vector<double> Mi;
      if (sb == p.k) {
        // two-element grid: the block is all of S, which is singular
        std::vector<double> v0b(sb), ln;
        for (int i = 0; i < sb; ++i) v0b[i] = p.v0[p.blk_slots[p.blk_off.back() - sb + i]];
        if (!bordered_pinv(M, sb, v0b, Mi, ln)) return "singular preconditioner block";
      } else if (!dense_inverse(M, sb, Mi)) {
        return "singular preconditioner block";
      }
      it = bkey.emplace(key, (int)bmats.size()).first;
      bmats.push_back(Mi);
      p.bcls_size.push_back(sb);
    }
    p.blk_cls.push_back(it->second);
  }
  p.nblk = (int)p.blk_red.size();
  {
    // order the blocks by class, so that a run of blocks given to one workgroup (and
    // the runs of one XCD) mostly share one block inverse in cache
    std::vector<int> ord(p.nblk);
    for (int b = 0; b < p.nblk; ++b) ord[b] = b;
    std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) { return p.blk_cls[a] < p.blk_cls[b]; });
    std::vector<int> red, off{0}, slots, cls;
    for (int b : ord) {
      red.push_back(p.blk_red[b]);
      cls.push_back(p.blk_cls[b]);
      slots.insert(slots.end(), p.blk_slots.begin() + p.blk_off[b], p.blk_slots.begin() + p.blk_off[b + 1]);
      off.push_back((int)slots.size());
    }
    p.blk_red.swap(red);
    p.blk_off.swap(off);
    p.blk_slots.swap(slots);
    p.blk_cls.swap(cls);
  }
  int64_t mtot = 0;
  for (size_t b = 0; b < bmats.size(); ++b) {
    p.bcls_off.push_back(mtot);
    mtot += (int64_t)p.bcls_size[b] * p.bcls_size[b];
  }
  p.MinvC.assign(mtot, 0.0);
  p.MinvR.assign(mtot, 0.0);
  for (size_t b = 0; b < bmats.size(); ++b) {
    const int sb = p.bcls_size[b];
    for (int i = 0; i < sb; ++i)
      for (int j = 0; j < sb; ++j) {
        p.MinvR[p.bcls_off[b] + (size_t)i * sb + j] = bmats[b][(size_t)i * sb + j];
        p.MinvC[p.bcls_off[b] + (size_t)j * sb + i] = bmats[b][(size_t)i * sb + j];
      }
  }

  // coarse matrix C = Z^T S Z (sparse rows) and its (pseudo-)inverse
  build_coarse_rows(p, p.C_off, p.C_col, p.C_val);
  bool singular = true;
  p.tau_hat.assign(d, 0.0);
  for (int64_t i = 0; i < d; ++i) {
    const int sa = p.iface_side[(size_t)i * 2], sb2 = p.iface_side[(size_t)i * 2 + 1];
    const double ta = tau_of(p.side_elem[sa], p.side_dir[sa]);
    const double tb = tau_of(p.side_elem[sb2], p.side_dir[sb2]);
    if (ta != tb) singular = false;
    p.tau_hat[i] = ta;
  }
  p.coarse_singular = singular;
  p.has_coarse = true;
  if (d <= dense_coarse_limit()) {
    p.coarse_mode = 1;
    p.C.assign((size_t)d * d, 0.0);
    for (int64_t i = 0; i < d; ++i)
      for (int64_t z = p.C_off[i]; z < p.C_off[i + 1]; ++z) p.C[(size_t)i * d + p.C_col[z]] = p.C_val[z];
    if (singular) {
      if (!bordered_pinv(p.C, (int)d, p.tau_hat, p.G, p.uC)) return "coarse bordered system singular";
    } else {
      p.tau_hat.clear();
      if (!dense_inverse(p.C, (int)d, p.G)) return "coarse matrix singular";
    }
  } else {
    p.coarse_mode = 2;
    const std::string err = build_coarse_sub(p, p.C_off, p.C_col, p.C_val);
    if (!err.empty()) return err;
    if (!singular) p.tau_hat.clear();
  }
  (void)N;
  return "";
}

// ---------------------------------------------------------------- exports

void export_schur_coo(const Plan& p, std::vector<int64_t>& ri, std::vector<int64_t>& ci,
                      std::vector<double>& v) {
  const int n = p.n;
  for (int64_t si = 0; si < p.nsides; ++si) {
    const int e = p.side_elem[si], s = p.side_dir[si];
    const int J = p.nbr[(size_t)e * 4 + s], so = opposite(s);
    const ElementClass& c = p.classes[p.cls[J]];
    const int64_t wo = p.W_off[(size_t)p.cls[J] * 4 + so];
    for (int t = 0; t < n; ++t) {
      const int64_t row = si * n + t;
      ri.push_back(row);
      ci.push_back(row);
      v.push_back(1.0);
      for (int cc = 0; cc < c.nslots; ++cc) {
        ri.push_back(row);
        ci.push_back(p.slot_off[J] + cc);
        v.push_back(p.Wr[wo + (size_t)t * c.nslots + cc]);
      }
    }
  }
}

void export_flux_solve_coo(const Plan& p, std::vector<int64_t>& ri, std::vector<int64_t>& ci,
                           std::vector<double>& v) {
  const int n = p.n, n2 = n * n;
  for (int64_t si = 0; si < p.nsides; ++si) {
    const int e = p.side_elem[si], s = p.side_dir[si];
    const int J = p.nbr[(size_t)e * 4 + s], so = opposite(s);
    const int64_t ho = p.H_off[(size_t)p.cls[J] * 4 + so];
    for (int t = 0; t < n; ++t)
      for (int l = 0; l < n2; ++l) {
        ri.push_back(si * n + t);
        ci.push_back((int64_t)J * n2 + l);
        v.push_back(p.Hr[ho + (size_t)t * n2 + l]);
      }
  }
}

void export_precond_inv_coo(const Plan& p, std::vector<int64_t>& ri, std::vector<int64_t>& ci,
                            std::vector<double>& v) {
  for (int b = 0; b < p.nblk; ++b) {
    const int o = p.blk_off[b], sb = p.blk_off[b + 1] - o;
    const int bc = p.blk_cls[b];
    for (int i = 0; i < sb; ++i)
      for (int j = 0; j < sb; ++j) {
        ri.push_back(p.blk_slots[o + i]);
        ci.push_back(p.blk_slots[o + j]);
        v.push_back(p.MinvR[p.bcls_off[bc] + (size_t)i * sb + j]);
      }
  }
}

}  // namespace smpm
