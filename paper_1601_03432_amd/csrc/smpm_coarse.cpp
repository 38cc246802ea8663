// Coarse solve of the deflation (Sec. 2): c2 = G c with G = C^+ for C = Z^T S Z.
//
// Small grids keep G as a dense matrix.  Larger grids solve with C by one level
// of substructuring.  C couples two interfaces only if they share an element, so
// cutting the element grid into P x P patches makes the interfaces interior to
// a patch couple only among themselves and with the separator interfaces (those
// between patches) that touch the patch.  With K the bordered matrix below,
// eliminating each patch's interior leaves a dense Schur complement on the
// separators:
//     S_B = K_BB - sum_p K_{B,I_p} K_pp^{-1} K_{I_p,B}.
// When C is singular (one null vector tau_hat, equal penalties across every
// interface) G = C^+ is the top-left block of the inverse of the nonsingular
// bordered matrix [[C, u_C], [tau_hat^T, 0]] (u_C the left null vector of C);
// its extra unknown lambda joins the separators.  A solve is then
//     y_p = K_pp^{-1} c_p                        (every patch)
//     r   = c_B - sum_p R_p c_p,  R_p = K_{B,I_p} K_pp^{-1}
//     x_B = S_B^{-1} r
//     x_p = y_p - F_p x_B,        F_p = K_pp^{-1} K_{I_p,B}
// and the transposed solve (G^T) runs the same steps with K_pp^{-T}, F_p^T,
// S_B^{-T} and R_p^T.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <map>

#include "smpm_plan.h"

namespace smpm {

namespace {

int env_int(const char* name, int dflt) {
  const char* v = std::getenv(name);
  if (!v || !*v) return dflt;
  return std::atoi(v);
}

// row-major m x n matrix a -> column-major copy
std::vector<double> to_colmajor(const double* a, int m, int n) {
  std::vector<double> o((size_t)m * n);
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < n; ++j) o[(size_t)j * m + i] = a[(size_t)i * n + j];
  return o;
}

}  // namespace

int dense_coarse_limit() { return std::min(env_int("SMPM_DENSE_COARSE_MAX", kDenseCoarseMax), kDenseCoarseMax); }

// Sparse C = Z^T S Z, rows sorted by column.  Row i: 2n on the diagonal (Z^T Z) plus,
// for each side of interface i, the row sums over that side of the outgoing fluxes
// of the element across it, gathered per interface of that element.
void build_coarse_rows(const Plan& p, std::vector<int64_t>& row_off, std::vector<int>& cols,
                       std::vector<double>& vals) {
  const int n = p.n;
  const int64_t d = p.d;
  row_off.assign(d + 1, 0);
  cols.clear();
  vals.clear();
  std::map<int, double> row;
  for (int64_t i = 0; i < d; ++i) {
    row.clear();
    row[(int)i] += 2.0 * n;
    for (int h = 0; h < 2; ++h) {
      const int si = p.iface_side[(size_t)i * 2 + h];
      const int e = p.side_elem[si], s = p.side_dir[si];
      const int J = p.nbr[(size_t)e * 4 + s], so = s ^ 1;
      const int cJ = p.cls[J];
      for (int s2 = 0; s2 < 4; ++s2) {
        const int j2 = p.iface[(size_t)J * 4 + s2];
        if (j2 < 0) continue;
        double sum = 0;
        for (int t = 0; t < n; ++t) sum += p.WZ[(((size_t)cJ * 4 + so) * n + t) * 4 + s2];
        row[j2] += sum;
      }
    }
    for (const auto& kv : row) {
      cols.push_back(kv.first);
      vals.push_back(kv.second);
    }
    row_off[i + 1] = (int64_t)cols.size();
  }
}

// x = K^{-1} [c; c_lambda] (or K^{-T}) with the host copies of the substructured factors;
// returns lambda.  c, x: length d.
double sub_solve_host(const Plan& p, const double* c, double c_lambda, double* x, bool tr) {
  const CoarseSub& q = p.sub;
  const int nS = q.nsep + q.border;
  std::vector<double> r(nS, 0.0);
  for (int b = 0; b < q.nsep; ++b) r[b] = c[q.sep_iface[b]];
  if (q.border) r[q.nsep] = c_lambda;
  std::vector<std::vector<double>> y(q.npatch);
  for (int pp = 0; pp < q.npatch; ++pp) {
    const int ni = q.I_off[pp + 1] - q.I_off[pp];
    const int nb = q.B_off[pp + 1] - q.B_off[pp], nbb = nb + q.border;
    const int* I = &q.I[q.I_off[pp]];
    const double* K = &q.Kr[q.K_off[pp]];   // K_pp^{-1} row-major
    const double* F = &q.Fr[q.FR_off[pp]];  // ni x nbb row-major
    const double* R = &q.Rr[q.FR_off[pp]];  // nbb x ni row-major
    y[pp].assign(ni, 0.0);
    for (int i = 0; i < ni; ++i) {
      double acc = 0;
      for (int j = 0; j < ni; ++j) acc += (tr ? K[(size_t)j * ni + i] : K[(size_t)i * ni + j]) * c[I[j]];
      y[pp][i] = acc;
    }
    for (int l = 0; l < nbb; ++l) {
      double acc = 0;
      for (int j = 0; j < ni; ++j) acc += (tr ? F[(size_t)j * nbb + l] : R[(size_t)l * ni + j]) * c[I[j]];
      const int g = l < nb ? q.B[q.B_off[pp] + l] : q.nsep;
      r[g] -= acc;
    }
  }
  std::vector<double> xb(nS, 0.0);
  const std::vector<double>& Si = tr ? q.SiT : q.Si;
  for (int a = 0; a < nS; ++a) {
    double acc = 0;
    for (int b = 0; b < nS; ++b) acc += Si[(size_t)a * nS + b] * r[b];
    xb[a] = acc;
  }
  for (int b = 0; b < q.nsep; ++b) x[q.sep_iface[b]] = xb[b];
  for (int pp = 0; pp < q.npatch; ++pp) {
    const int ni = q.I_off[pp + 1] - q.I_off[pp];
    const int nb = q.B_off[pp + 1] - q.B_off[pp], nbb = nb + q.border;
    const int* I = &q.I[q.I_off[pp]];
    const double* F = &q.Fr[q.FR_off[pp]];
    const double* R = &q.Rr[q.FR_off[pp]];
    for (int i = 0; i < ni; ++i) {
      double acc = y[pp][i];
      for (int l = 0; l < nbb; ++l) {
        const double xv = l < nb ? xb[q.B[q.B_off[pp] + l]] : xb[q.nsep];
        acc -= (tr ? R[(size_t)l * ni + i] : F[(size_t)i * nbb + l]) * xv;
      }
      x[I[i]] = acc;
    }
  }
  return q.border ? xb[q.nsep] : 0.0;
}

// Builds the substructured factors of K = [[C, a], [b^T, 0]] (border only if C is
// singular; a = b = tau_hat first, then a = u_C).  Returns "" or an error.
std::string build_coarse_sub(Plan& p, const std::vector<int64_t>& row_off, const std::vector<int>& cols,
                             const std::vector<double>& vals) {
  CoarseSub& q = p.sub;
  q = CoarseSub();
  const int64_t d = p.d;
  // patch size: 8 elements a side unless set; doubled while the separator system would
  // exceed 8192 unknowns (its right-hand side is staged in LDS by the device solve)
  int P = std::max(1, env_int("SMPM_COARSE_PATCH", 8));
  auto nsep_of = [&](int Pp) {
    const int ax = (p.mx + Pp - 1) / Pp, ay = (p.my + Pp - 1) / Pp;
    return (int64_t)p.my * (ax - 1) + (int64_t)p.mx * (ay - 1);
  };
  while (nsep_of(P) + 1 > 8192) P *= 2;
  // at least two patches: a patch holding every interface would hold all of C
  while (P > 1 && ((p.mx + P - 1) / P) * ((p.my + P - 1) / P) < 2) P = (P + 1) / 2;
  const int px = (p.mx + P - 1) / P, py = (p.my + P - 1) / P;
  q.P = P;
  q.npatch = px * py;
  q.border = p.coarse_singular ? 1 : 0;
  auto patch_of = [&](int e) { return (e / p.mx / P) * px + (e % p.mx) / P; };
  // roles: interior interfaces of each patch, separators
  std::vector<std::vector<int>> Ilist(q.npatch), Blist(q.npatch);
  q.role.assign(d, 0);
  for (int64_t i = 0; i < d; ++i) {
    const int e1 = p.side_elem[p.iface_side[(size_t)i * 2]];
    const int e2 = p.side_elem[p.iface_side[(size_t)i * 2 + 1]];
    const int p1 = patch_of(e1), p2 = patch_of(e2);
    if (p1 == p2) {
      q.role[i] = (int)Ilist[p1].size();
      Ilist[p1].push_back((int)i);
    } else {
      const int sid = q.nsep++;
      q.role[i] = -(sid + 1);
      q.sep_iface.push_back((int)i);
      q.sep_pl.push_back(p1);
      q.sep_pl.push_back((int)Blist[p1].size());
      Blist[p1].push_back(sid);
      q.sep_pl.push_back(p2);
      q.sep_pl.push_back((int)Blist[p2].size());
      Blist[p2].push_back(sid);
    }
  }
  q.I_off.assign(1, 0);
  q.B_off.assign(1, 0);
  q.K_off.assign(1, 0);
  q.FR_off.assign(1, 0);
  for (int pp = 0; pp < q.npatch; ++pp) {
    q.I.insert(q.I.end(), Ilist[pp].begin(), Ilist[pp].end());
    q.B.insert(q.B.end(), Blist[pp].begin(), Blist[pp].end());
    q.I_off.push_back((int)q.I.size());
    q.B_off.push_back((int)q.B.size());
    const int64_t ni = (int64_t)Ilist[pp].size(), nbb = (int64_t)Blist[pp].size() + q.border;
    q.K_off.push_back(q.K_off.back() + ni * ni);
    q.FR_off.push_back(q.FR_off.back() + ni * nbb);
  }
  const int nS = q.nsep + q.border;
  q.Kr.assign(q.K_off.back(), 0.0);
  q.Fr.assign(q.FR_off.back(), 0.0);
  q.Rr.assign(q.FR_off.back(), 0.0);
  std::vector<double> SB((size_t)nS * nS, 0.0);
  // K_BB: separator rows at separator columns, and the border (tau_hat scaled to unit
  // length: the bordered inverse's top-left block does not depend on the scaling)
  std::vector<double> tau;
  if (q.border) {
    double nt = 0;
    for (double v : p.tau_hat) nt += v * v;
    nt = std::sqrt(nt);
    tau.resize(d);
    for (int64_t i = 0; i < d; ++i) tau[i] = p.tau_hat[i] / nt;
  }
  for (int b = 0; b < q.nsep; ++b) {
    const int i = q.sep_iface[b];
    for (int64_t z = row_off[i]; z < row_off[i + 1]; ++z)
      if (q.role[cols[z]] < 0) SB[(size_t)b * nS + (-q.role[cols[z]] - 1)] += vals[z];
    if (q.border) {
      SB[(size_t)b * nS + q.nsep] = tau[i];
      SB[(size_t)q.nsep * nS + b] = tau[i];
    }
  }
  std::vector<double> Kpp, Kinv, Cib, Cbi;
  for (int pp = 0; pp < q.npatch; ++pp) {
    const std::vector<int>& I = Ilist[pp];
    const std::vector<int>& Bl = Blist[pp];
    const int ni = (int)I.size(), nb = (int)Bl.size(), nbb = nb + q.border;
    if (ni == 0) continue;
    std::map<int, int> bloc;  // separator id -> local index in this patch
    for (int l = 0; l < nb; ++l) bloc[Bl[l]] = l;
    Kpp.assign((size_t)ni * ni, 0.0);
    Cib.assign((size_t)ni * nbb, 0.0);  // [C_{I,B} | a_I]
    Cbi.assign((size_t)nbb * ni, 0.0);  // [C_{B,I} ; b_I^T]
    for (int a = 0; a < ni; ++a) {
      const int i = I[a];
      for (int64_t z = row_off[i]; z < row_off[i + 1]; ++z) {
        const int j = cols[z], rl = q.role[j];
        if (rl >= 0) {
          Kpp[(size_t)a * ni + rl] += vals[z];  // same patch: interior couples only within it
        } else {
          Cib[(size_t)a * nbb + bloc.at(-rl - 1)] += vals[z];
        }
      }
      if (q.border) {
        Cib[(size_t)a * nbb + nb] = tau[i];
        Cbi[(size_t)nb * ni + a] = tau[i];
      }
    }
    for (int l = 0; l < nb; ++l) {
      const int i = q.sep_iface[Bl[l]];
      for (int64_t z = row_off[i]; z < row_off[i + 1]; ++z) {
        const int rl = q.role[cols[z]];
        if (rl >= 0 && patch_of(p.side_elem[p.iface_side[(size_t)cols[z] * 2]]) == pp)
          Cbi[(size_t)l * ni + rl] += vals[z];
      }
    }
    if (!dense_inverse(Kpp, ni, Kinv)) return "singular patch block of the coarse matrix";
    double* Kr = &q.Kr[q.K_off[pp]];
    double* Fr = &q.Fr[q.FR_off[pp]];
    double* Rr = &q.Rr[q.FR_off[pp]];
    std::copy(Kinv.begin(), Kinv.end(), Kr);
    for (int a = 0; a < ni; ++a)
      for (int l = 0; l < nbb; ++l) {
        double acc = 0;
        for (int m = 0; m < ni; ++m) acc += Kinv[(size_t)a * ni + m] * Cib[(size_t)m * nbb + l];
        Fr[(size_t)a * nbb + l] = acc;
      }
    for (int l = 0; l < nbb; ++l)
      for (int a = 0; a < ni; ++a) {
        double acc = 0;
        for (int m = 0; m < ni; ++m) acc += Cbi[(size_t)l * ni + m] * Kinv[(size_t)m * ni + a];
        Rr[(size_t)l * ni + a] = acc;
      }
    // S_B -= [C_BI; b^T] F
    for (int l = 0; l < nbb; ++l) {
      const int gl = l < nb ? Bl[l] : q.nsep;
      for (int l2 = 0; l2 < nbb; ++l2) {
        const int gl2 = l2 < nb ? Bl[l2] : q.nsep;
        double acc = 0;
        for (int m = 0; m < ni; ++m) acc += Cbi[(size_t)l * ni + m] * Fr[(size_t)m * nbb + l2];
        SB[(size_t)gl * nS + gl2] -= acc;
      }
    }
  }
  if (nS > 0 && !dense_inverse(SB, nS, q.Si)) return "singular separator system of the coarse matrix";
  auto transpose_si = [&]() {
    q.SiT.assign((size_t)nS * nS, 0.0);
    for (int a = 0; a < nS; ++a)
      for (int b = 0; b < nS; ++b) q.SiT[(size_t)b * nS + a] = q.Si[(size_t)a * nS + b];
  };
  transpose_si();
  if (q.border) {
    // u_C from the transposed bordered system [[C^T, tau], [tau^T, 0]] [u; mu] = [0; 1]
    std::vector<double> zero(d, 0.0), u(d, 0.0);
    sub_solve_host(p, zero.data(), 1.0, u.data(), true);
    double nn = 0, sum = 0;
    for (double v : u) {
      nn += v * v;
      sum += v;
    }
    nn = std::sqrt(nn);
    const double sg = sum < 0 ? -1.0 : 1.0;
    for (double& v : u) v *= sg / nn;
    p.uC = u;
    // border column a: tau_hat -> u_C.  F's last column and S_B's last column change;
    // S_B^{-1} follows by a rank-one (Sherman-Morrison) update.
    std::vector<double> delta(nS, 0.0);
    for (int b = 0; b < q.nsep; ++b) delta[b] = u[q.sep_iface[b]] - tau[q.sep_iface[b]];
    for (int pp = 0; pp < q.npatch; ++pp) {
      const int ni = q.I_off[pp + 1] - q.I_off[pp];
      const int nb = q.B_off[pp + 1] - q.B_off[pp], nbb = nb + 1;
      if (ni == 0) continue;
      const int* I = &q.I[q.I_off[pp]];
      const double* Kr = &q.Kr[q.K_off[pp]];
      double* Fr = &q.Fr[q.FR_off[pp]];
      const double* Rr = &q.Rr[q.FR_off[pp]];
      std::vector<double> dF(ni, 0.0);
      for (int a = 0; a < ni; ++a) {
        double acc = 0;
        for (int m = 0; m < ni; ++m) acc += Kr[(size_t)a * ni + m] * (u[I[m]] - tau[I[m]]);
        dF[a] = acc;
        Fr[(size_t)a * nbb + nb] += acc;
      }
      // delta of S_B column lambda: -[C_BI; b^T] dF = -(R K_pp)(dF)... computed from C_BI
      // directly: [C_BI; b^T] K_pp^{-1} (du_I) = R_p (du_I)
      for (int l = 0; l < nbb; ++l) {
        double acc = 0;
        for (int m = 0; m < ni; ++m) acc += Rr[(size_t)l * ni + m] * (u[I[m]] - tau[I[m]]);
        const int gl = l < nb ? q.B[q.B_off[pp] + l] : q.nsep;
        delta[gl] -= acc;
      }
    }
    // (S + delta e_lam^T)^{-1} = S^{-1} - (S^{-1} delta)(e_lam^T S^{-1}) / (1 + e_lam^T S^{-1} delta)
    std::vector<double> sd(nS, 0.0);
    for (int a = 0; a < nS; ++a) {
      double acc = 0;
      for (int b = 0; b < nS; ++b) acc += q.Si[(size_t)a * nS + b] * delta[b];
      sd[a] = acc;
    }
    const double den = 1.0 + sd[q.nsep];
    if (!(std::fabs(den) > 1e-300)) return "singular bordered coarse system";
    const double* lastrow = &q.Si[(size_t)q.nsep * nS];
    std::vector<double> lr(lastrow, lastrow + nS);
    for (int a = 0; a < nS; ++a)
      for (int b = 0; b < nS; ++b) q.Si[(size_t)a * nS + b] -= sd[a] * lr[b] / den;
    transpose_si();
  }
  // check: K [x; lambda] = [c; 0] for a fixed pseudo-random c (relative residual)
  {
    std::vector<double> c(d), x(d, 0.0);
    uint64_t st = 0x9E3779B97F4A7C15ull;
    for (int64_t i = 0; i < d; ++i) {
      st = st * 6364136223846793005ull + 1442695040888963407ull;
      c[i] = (double)(st >> 11) * (1.0 / 9007199254740992.0) - 0.5;
    }
    const double lam = sub_solve_host(p, c.data(), 0.0, x.data(), false);
    double rr = 0, cc = 0, bt = 0;
    for (int64_t i = 0; i < d; ++i) {
      double acc = -c[i];
      for (int64_t z = row_off[i]; z < row_off[i + 1]; ++z) acc += vals[z] * x[cols[z]];
      if (q.border) acc += p.uC[i] * lam;
      rr += acc * acc;
      cc += c[i] * c[i];
      if (q.border) bt += tau[i] * x[i];
    }
    if (!(std::sqrt(rr) <= 1e-8 * std::sqrt(cc)) || !(std::fabs(bt) <= 1e-8 * std::sqrt(cc)))
      return "substructured coarse solve failed its setup residual check";
  }
  // column-major copies for the device kernels (lanes over rows, coalesced)
  q.Kc.assign(q.Kr.size(), 0.0);
  q.Fc.assign(q.Fr.size(), 0.0);
  q.Rc.assign(q.Rr.size(), 0.0);
  for (int pp = 0; pp < q.npatch; ++pp) {
    const int ni = q.I_off[pp + 1] - q.I_off[pp];
    const int nbb = q.B_off[pp + 1] - q.B_off[pp] + q.border;
    auto kc = to_colmajor(&q.Kr[q.K_off[pp]], ni, ni);
    auto fc = to_colmajor(&q.Fr[q.FR_off[pp]], ni, nbb);
    auto rc = to_colmajor(&q.Rr[q.FR_off[pp]], nbb, ni);
    std::copy(kc.begin(), kc.end(), q.Kc.begin() + q.K_off[pp]);
    std::copy(fc.begin(), fc.end(), q.Fc.begin() + q.FR_off[pp]);
    std::copy(rc.begin(), rc.end(), q.Rc.begin() + q.FR_off[pp]);
  }
  return "";
}

}  // namespace smpm
