// Host-side plan of the SMPM Schur complement solver: geometry, interface slot
// layout, per-class element operators, block-Jacobi blocks and the coarse
// deflation matrix.  Everything here is FP64 and built once by smpm_setup.
//
// Layouts (all row indices run fastest where a kernel's lanes read them):
//   r-vectors   node (p,q) of element e = iy*m_x + ix at e*n^2 + q*n + p
//   k-vectors   slot = side_index*n + t; side_index enumerates inter-element
//               sides element-major, sides W,E,S,N; t runs along the side
//               (q for W/E, p for S/N)
//   d-vectors   interfaces: vertical (iy, ix|ix+1) row-major, then horizontal
//               (iy|iy+1, ix) row-major
#pragma once
#include <cstdint>
#include <string>
#include <vector>

namespace smpm {

enum Side { SW = 0, SE = 1, SS = 2, SN = 3 };
// readings of the Robin length sigma (values of smpm_robin in smpm.h)
constexpr int kRobinMin = 0, kRobinLiteral = 1, kRobinReference = 2;
inline int opposite(int s) { return s ^ 1; }

struct ElementClass {
  double w = 0, h = 0;
  int mask = 0;            // bit s set: side s is an inter-element side
  double tau_own[4] = {0, 0, 0, 0};   // penalty of this element's sides
  double tau_recv[4] = {0, 0, 0, 0};  // penalty of the neighbour side facing side s
  double sig_own[4] = {0, 0, 0, 0};   // Robin length scale sigma of this element's sides
  double sig_recv[4] = {0, 0, 0, 0};  // ... of the neighbour side facing side s
  int nslots = 0;          // slots owned by an element of this class
  int side_col[4] = {-1, -1, -1, -1};  // first slot column of side s within the element
};

// Substructured coarse solve (grids with many interfaces): patch-interior inverses and
// the dense separator Schur complement.  All matrices FP64; *_r row-major, *_c
// column-major copies of the same matrices.
struct CoarseSub {
  int P = 0;                         // patch size in elements
  int npatch = 0, nsep = 0;
  int border = 0;                    // 1 if C is singular: the bordered unknown lambda
  std::vector<int> role;             // d: local interior index (>= 0) or -(separator + 1)
  std::vector<int> I_off, I;         // interior interfaces of each patch
  std::vector<int> B_off, B;         // separators touching each patch (lambda implied last)
  std::vector<int64_t> K_off;        // offsets of K_pp^{-1} (ni x ni)
  std::vector<int64_t> FR_off;       // offsets of F_p (ni x nbb) and R_p (nbb x ni)
  std::vector<double> Kr, Kc, Fr, Fc, Rr, Rc;
  std::vector<int> sep_iface;        // nsep: interface of each separator
  std::vector<int> sep_pl;           // nsep*4: (patch, local index) for both patches
  std::vector<double> Si, SiT;       // (nsep+border)^2 row-major: S_B^{-1} and its transpose
};

struct Plan {
  int n = 0, mx = 0, my = 0, nel = 0;
  int64_t r = 0, k = 0, d = 0, nsides = 0;
  double alpha = 0;
  int robin = kRobinMin;
  std::vector<double> side_tau, side_sig;  // nel*4: tau and sigma of every side (physical ones too)
  std::vector<double> xb, yb;
  std::vector<double> wx, hy;  // element widths / heights (equal within 1e-12 relative -> identical)
  // GLL
  std::vector<double> xi, omega, D;  // D row-major n x n
  // elements
  std::vector<int> mask, nbr, cls, side_slot, iface;  // nbr/side_slot/iface: nel*4
  std::vector<int> slot_off;                           // nel+1
  std::vector<int> side_elem, side_dir;                // per inter-element side
  std::vector<int> iface_side;                         // d*2: side indices of the two sides
  // classes and their operators
  std::vector<ElementClass> classes;
  std::vector<double> Ainv;     // per class n2 x n2 row-major  [l][m]
  std::vector<double> AinvT;    // per class transposed         [m][l]
  std::vector<int64_t> W_off;   // class*4: offset of side s' operator, -1 if absent
  std::vector<double> Wc;       // outgoing flux of side s': [c][i] (nslots x n)
  std::vector<double> Wr;       //                            [i][c] (n x nslots)
  std::vector<int64_t> H_off;   // class*4
  std::vector<double> Hc;       // flux of A^{-1} f through side s': [l][i] (n2 x n)
  std::vector<double> Hr;       //                                    [i][l] (n x n2)
  std::vector<double> WZ;       // class*4*n*4: [s'][t][s''] row sums of W over side s''
  // groups of up to kGroup elements of one class (element operators shared inside a group)
  static constexpr int kGroup = 8;
  int grp_size = 8;                  // elements per group (1..8): fewer on small grids
  int ngrp = 0;
  std::vector<int> grp_cls;          // class of each group
  std::vector<int> grp_elem;         // ngrp*kGroup element ids, -1 padded
  // tiles of up to kTile elements of one class: the columns of the matrix-core products
  static constexpr int kTile = 16;
  int tile_size = 16;                // 4, 8 or 16
  int ntile = 0;
  std::vector<int> tile_cls;
  std::vector<int> tile_elem;        // ntile*kTile element ids, -1 padded
  std::vector<int> tile_src;         // ntile*kTile: first slot of the element, -1 if none
  std::vector<int> tile_dst;         // ntile*kTile*4: first slot facing side s, -1 if none
  // class operators in matrix-core fragment order (n <= 16): [cls][row tile w][step q][lane],
  // lane l of step q holds A[16w + l%16][4q + l/16]; A = W (forward) or W^T (transpose)
  int mma_mt = 0;                    // 16-row tiles covering 4n rows
  int mma_kt = 0;                    // 4-deep steps covering 4n columns (a multiple of 4)
  std::vector<double> Afwd, Aadj;
  // block-Jacobi
  int nblk = 0;
  std::vector<int> blk_red;          // red element of each block
  std::vector<int> blk_off;          // nblk+1 offsets into blk_slots
  std::vector<int> blk_slots;        // slot list of every block
  std::vector<int> blk_cls;          // block class of each block
  std::vector<int> bcls_size;        // size of each block class
  std::vector<int64_t> bcls_off;     // offset of each block class inverse
  std::vector<double> MinvC;         // [c][r] per block class
  std::vector<double> MinvR;         // [r][c] per block class
  // coarse space
  bool has_coarse = false;           // coarse solve built (deflation available)
  int coarse_mode = 0;               // 1: dense G, 2: substructured
  bool coarse_singular = false;
  std::vector<double> C, G;          // d x d row-major (dense mode)
  std::vector<int64_t> C_off;        // sparse C rows (both modes)
  std::vector<int> C_col;
  std::vector<double> C_val;
  CoarseSub sub;                     // substructured mode
  std::vector<double> tau_hat, uC;   // right / left null vectors of C when singular
  // v0 = B 1, the right null vector of S
  std::vector<double> v0;
};

// Builds the plan.  Returns an empty string on success, else the error text.
std::string build_plan(Plan& p, int m_y, int m_x, int n, const double* x_breaks,
                       const double* y_breaks, double alpha, int robin = kRobinMin);

// Host export helpers used by the CPU tests of the setup.
void export_schur_coo(const Plan& p, std::vector<int64_t>& ri, std::vector<int64_t>& ci,
                      std::vector<double>& v);
void export_flux_solve_coo(const Plan& p, std::vector<int64_t>& ri, std::vector<int64_t>& ci,
                           std::vector<double>& v);
void export_precond_inv_coo(const Plan& p, std::vector<int64_t>& ri, std::vector<int64_t>& ci,
                            std::vector<double>& v);

// Coarse solve helpers (smpm_coarse.cpp).  Grids with more interfaces than
// dense_coarse_limit() (kDenseCoarseMax = 4096, the most the dense coarse kernel
// stages; the environment SMPM_DENSE_COARSE_MAX may lower it) use the substructured
// solve with patches of SMPM_COARSE_PATCH (default 8) elements a side.
constexpr int kDenseCoarseMax = 4096;
int dense_coarse_limit();
void build_coarse_rows(const Plan& p, std::vector<int64_t>& row_off, std::vector<int>& cols,
                       std::vector<double>& vals);
std::string build_coarse_sub(Plan& p, const std::vector<int64_t>& row_off, const std::vector<int>& cols,
                             const std::vector<double>& vals);
double sub_solve_host(const Plan& p, const double* c, double c_lambda, double* x, bool tr);

// Dense LU with partial pivoting (row-major, in place).  Returns false if a pivot is
// not above min_pivot (singular).  dense_inverse rejects pivots at or below
// min_rel_pivot times the largest entry.
bool lu_factor(std::vector<double>& a, int m, std::vector<int>& piv, double min_pivot = 0.0);
void lu_solve(const std::vector<double>& a, int m, const std::vector<int>& piv, double* b);
bool dense_inverse(const std::vector<double>& a, int m, std::vector<double>& inv, double min_rel_pivot = 0.0);

}  // namespace smpm
