"""CPU FP64 oracle for the deflated Schur complement method of Joshi & Diamessis
(arXiv 1601.03432) applied to the SMPM discretization of the 2-D Poisson-Neumann
problem.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU-baseline
leg of the benchmark may import this module.  It shares no code, tables or
helpers with the HIP library and never imports it.

It is plain and slow on purpose: element blocks are built from their definition
with dense numpy arrays, global operators are scipy.sparse matrices, inverses
and null vectors come from numpy/scipy factorizations, and GMRES is a textbook
Arnoldi loop whose least-squares problem is re-solved with numpy.linalg.lstsq
at every step.

Notation follows the paper: n GLL points per direction (polynomial order
N = n - 1), an m_y x m_x Cartesian element grid, r = n^2 m_x m_y nodes, the
interface grid Gamma of size k, the operator split L = A + E B (Sec. 1.3), the
Schur complement S = I + B A^{-1} E (Eq. schur_complement_system), the
block-Jacobi preconditioner M and the deflation quantities Z, C, P, Q (Sec. 2,
Eqs. projection1/projection2, deflated_schur).

Readings where the paper is silent or at odds with itself:

* Interface grid.  Sec. 1.3 puts n nodes on either side of every interface and
  Sec. 2 counts 8n points in an interior preconditioner block; B assigns the
  flux of each element side to the facing side of the neighbour.  Gamma is
  therefore the set of side slots: one entry per (element, inter-element side,
  node along the side).  An element-corner node lying on two inter-element
  sides owns two slots, one per side, each holding that side's flux.  E maps a
  slot to its node (so E^T E = I holds except between the two slots of such a
  corner node).
* Robin operator and penalty.  Sec. 1.2 writes R_ij = I + n_i.grad and leaves
  tau to a heuristic.  The oracle takes R = I + sigma n_i.grad with one of three
  readings of the length sigma and the matching penalty tau (omega_0 = 2/(N(N+1))
  the GLL end weight, h_perp the element's extent normal to the side, h_e its
  smaller extent; the values of the element whose row it is serve u_i and u_j
  alike):
    "literal"    sigma = 1 (R exactly as printed, physical coordinates),
                 tau = 2 alpha / (omega_0 h_perp);
    "reference"  sigma = h_perp/2 (the normal derivative in the element's
                 reference coordinates [-1,1]^2), tau = 2 alpha / (omega_0 h_perp^2);
    "min"        sigma = h_e/2, tau = 2 alpha / (omega_0 h_e^2) (default; equal
                 to "reference" on square elements).
  A physical side carries tau sigma n.grad u and tau sigma g (for "literal" the
  tau_i n.grad u_i and tau_i g_i of Eq. smpm_poisson).  alpha = 8 on all sides by
  default (the oracle accepts any alpha_int / alpha_phys).
* Element-corner nodes receive the penalty terms of both sides containing them.
* Block-Jacobi blocks follow the checkerboard: the block of a "red" element
  ((ix+iy) even) holds that element's slots and the slots of its neighbours'
  sides facing it.  Every slot lies on an interface between a red and a black
  element, so the blocks partition Gamma.
* One deflation vector per interface, 1 on the 2n slots of its two sides.
* The additive constant of u is fixed by w^T u = 0 (w = GLL quadrature weights).
* GMRES is unrestarted, right-preconditioned, from x0 = 0, and stops when the
  least-squares residual is <= tol times its initial value.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla
from numpy.polynomial import legendre as leg

# side numbering and outward normals: W (-x), E (+x), S (-y), N (+y)
W, E, S, N = 0, 1, 2, 3
SIDES = (W, E, S, N)
OPPOSITE = {W: E, E: W, S: N, N: S}
DEFAULT_ALPHA = 8.0
ROBIN_MODES = ("min", "literal", "reference")


# ---------------------------------------------------------------------------
# GLL grid and spectral differentiation (Sec. 1.2)
# ---------------------------------------------------------------------------

def gll(n: int):
    """Gauss-Lobatto-Legendre nodes, weights and differentiation matrix.

    Sec. 1.2: n GLL points per direction, derivatives of the Lagrange
    interpolant through a spectral differentiation matrix.  Textbook formulas:
    nodes are -1, 1 and the roots of P_N'; weights 2/(N(N+1) P_N(x_i)^2);
    D_ij = P_N(x_i)/(P_N(x_j)(x_i - x_j)) for i != j, D_00 = -N(N+1)/4,
    D_NN = N(N+1)/4, other diagonal entries 0.
    """
    if n < 2:
        raise ValueError("need n >= 2")
    Np = n - 1
    cN = np.zeros(Np + 1)
    cN[Np] = 1.0
    dcN = leg.legder(cN)
    if Np >= 2:
        interior = np.sort(np.real(leg.legroots(dcN)))
        d2cN = leg.legder(dcN)
        for _ in range(4):  # Newton polish of the roots of P_N'
            interior = interior - leg.legval(interior, dcN) / leg.legval(interior, d2cN)
    else:
        interior = np.zeros(0)
    x = np.concatenate([[-1.0], interior, [1.0]])
    PN = leg.legval(x, cN)
    w = 2.0 / (Np * (Np + 1) * PN ** 2)
    D = np.zeros((n, n))
    for i in range(n):
        for j in range(n):
            if i != j:
                D[i, j] = PN[i] / (PN[j] * (x[i] - x[j]))
    D[0, 0] = -Np * (Np + 1) / 4.0
    D[Np, Np] = Np * (Np + 1) / 4.0
    return x, w, D


# ---------------------------------------------------------------------------
# grid
# ---------------------------------------------------------------------------

class Grid:
    """An m_y x m_x Cartesian element grid with n GLL points per direction.

    Node (p, q) of element (iy, ix) has global index ((iy*m_x + ix)*n + q)*n + p
    (p runs along x).  Element (iy, ix) covers [x_ix, x_ix+1] x [y_iy, y_iy+1].
    """

    def __init__(self, n, x_breaks, y_breaks, alpha_int=DEFAULT_ALPHA, alpha_phys=None, robin="min"):
        if robin not in ROBIN_MODES:
            raise ValueError(f"robin must be one of {ROBIN_MODES}")
        self.robin = robin
        self.n = int(n)
        self.Np = self.n - 1
        self.xb = np.asarray(x_breaks, np.float64)
        self.yb = np.asarray(y_breaks, np.float64)
        self.m_x = len(self.xb) - 1
        self.m_y = len(self.yb) - 1
        self.nel = self.m_x * self.m_y
        self.n2 = self.n * self.n
        self.r = self.n2 * self.nel
        self.alpha_int = float(alpha_int)
        self.alpha_phys = float(alpha_int if alpha_phys is None else alpha_phys)
        self.xi, self.omega, self.D = gll(self.n)

    def eid(self, iy, ix):
        return iy * self.m_x + ix

    def width(self, ix):
        return self.xb[ix + 1] - self.xb[ix]

    def height(self, iy):
        return self.yb[iy + 1] - self.yb[iy]

    def neighbor(self, iy, ix, side):
        jy, jx = iy, ix
        if side == W:
            jx -= 1
        elif side == E:
            jx += 1
        elif side == S:
            jy -= 1
        else:
            jy += 1
        if 0 <= jx < self.m_x and 0 <= jy < self.m_y:
            return jy, jx
        return None

    def elem_len(self, iy, ix):
        """h_e: the smaller extent of element (iy, ix)."""
        return min(self.width(ix), self.height(iy))

    def normal_len(self, iy, ix, side):
        """h_perp: the extent of element (iy, ix) normal to one of its sides."""
        return self.width(ix) if side in (W, E) else self.height(iy)

    def tau(self, iy, ix, side):
        """Penalty of one side of one element (readings stated in the module header):
        2 alpha / (omega_0 h_perp) for "literal", 2 alpha / (omega_0 l^2) otherwise
        with l = h_perp ("reference") or h_e ("min")."""
        omega0 = 2.0 / (self.Np * (self.Np + 1))
        alpha = self.alpha_int if self.neighbor(iy, ix, side) is not None else self.alpha_phys
        if self.robin == "literal":
            return 2.0 * alpha / (omega0 * self.normal_len(iy, ix, side))
        ell = self.normal_len(iy, ix, side) if self.robin == "reference" else self.elem_len(iy, ix)
        return 2.0 * alpha / (omega0 * ell ** 2)

    def sigma(self, iy, ix, side):
        """Length scale of the Robin operator R = I + sigma n.grad on one side of
        element (iy, ix): 1 ("literal"), h_perp/2 ("reference") or h_e/2 ("min")."""
        if self.robin == "literal":
            return 1.0
        if self.robin == "reference":
            return 0.5 * self.normal_len(iy, ix, side)
        return 0.5 * self.elem_len(iy, ix)

    def side_nodes(self, side):
        """Local indices (q*n + p) of a side's nodes, ordered along the side."""
        n, Np = self.n, self.Np
        t = np.arange(n)
        if side == W:
            return t * n
        if side == E:
            return t * n + Np
        if side == S:
            return t
        return Np * n + t

    def node_coords(self):
        n = self.n
        x = np.zeros(self.r)
        y = np.zeros(self.r)
        for iy in range(self.m_y):
            for ix in range(self.m_x):
                e = self.eid(iy, ix)
                xs = self.xb[ix] + (self.xi + 1.0) * self.width(ix) / 2.0
                ys = self.yb[iy] + (self.xi + 1.0) * self.height(iy) / 2.0
                X, Y = np.meshgrid(xs, ys)  # [q][p]
                x[e * n * n:(e + 1) * n * n] = X.ravel()
                y[e * n * n:(e + 1) * n * n] = Y.ravel()
        return x, y

    def quad_weights(self):
        """GLL quadrature weights of the nodes: omega_p omega_q w h / 4."""
        n = self.n
        wv = np.zeros(self.r)
        base = np.outer(self.omega, self.omega).ravel()  # [q][p]
        for iy in range(self.m_y):
            for ix in range(self.m_x):
                e = self.eid(iy, ix)
                wv[e * n * n:(e + 1) * n * n] = base * self.width(ix) * self.height(iy) / 4.0
        return wv

    def boundary_arc(self):
        """Arc coordinates of the boundary-data layout: south (m_x n, along x),
        north, west (m_y n, along y), east."""
        xs = np.concatenate([self.xb[ix] + (self.xi + 1.0) * self.width(ix) / 2.0 for ix in range(self.m_x)])
        ys = np.concatenate([self.yb[iy] + (self.xi + 1.0) * self.height(iy) / 2.0 for iy in range(self.m_y)])
        return xs, xs.copy(), ys, ys.copy()

    @property
    def nbdry(self):
        return 2 * self.n * (self.m_x + self.m_y)

    def bdry_index(self, iy, ix, side, t):
        n = self.n
        if side == S:
            return ix * n + t
        if side == N:
            return self.m_x * n + ix * n + t
        if side == W:
            return 2 * self.m_x * n + iy * n + t
        return 2 * self.m_x * n + self.m_y * n + iy * n + t

    def sides(self):
        """Inter-element sides (iy, ix, s) in slot order: element-major, then W, E, S, N."""
        out = []
        for iy in range(self.m_y):
            for ix in range(self.m_x):
                for s in SIDES:
                    if self.neighbor(iy, ix, s) is not None:
                        out.append((iy, ix, s))
        return out


# ---------------------------------------------------------------------------
# element operators of Eq. smpm_poisson
# ---------------------------------------------------------------------------

def laplacian_block(grid: Grid, w, h):
    """Collocated Laplacian on one element: (4/w^2) D^2 along p + (4/h^2) D^2 along q."""
    D2 = grid.D @ grid.D
    I = np.eye(grid.n)
    return (4.0 / w ** 2) * np.kron(I, D2) + (4.0 / h ** 2) * np.kron(D2, I)


def trace_rows(grid: Grid, side):
    R = np.zeros((grid.n, grid.n2))
    R[np.arange(grid.n), grid.side_nodes(side)] = 1.0
    return R


def outward_derivative_rows(grid: Grid, side, w, h):
    """Rows giving n_hat . grad u at a side's nodes, n_hat the element's outward normal."""
    n, Np, D = grid.n, grid.Np, grid.D
    R = np.zeros((n, grid.n2))
    for t in range(n):
        for a in range(n):
            if side == W:      # node (p=0, q=t), n_hat = (-1, 0)
                R[t, t * n + a] = -(2.0 / w) * D[0, a]
            elif side == E:    # node (p=N, q=t), n_hat = (+1, 0)
                R[t, t * n + a] = (2.0 / w) * D[Np, a]
            elif side == S:    # node (p=t, q=0), n_hat = (0, -1)
                R[t, a * n + t] = -(2.0 / h) * D[0, a]
            else:              # node (p=t, q=N), n_hat = (0, +1)
                R[t, a * n + t] = (2.0 / h) * D[Np, a]
    return R


def local_block(grid: Grid, iy, ix):
    """A_e: the part of Eq. smpm_poisson local to element (iy, ix) (Sec. 1.3).

    Laplacian + tau (u + sigma n.grad u) on every inter-element side (the R_ii
    term) + tau sigma n.grad u on every physical side; corner nodes get both
    sides' terms.
    """
    w, h = grid.width(ix), grid.height(iy)
    A = laplacian_block(grid, w, h)
    for s in SIDES:
        rows = grid.side_nodes(s)
        tau, sig = grid.tau(iy, ix, s), grid.sigma(iy, ix, s)
        dn = outward_derivative_rows(grid, s, w, h)
        if grid.neighbor(iy, ix, s) is None:
            A[rows, :] += tau * sig * dn
        else:
            A[rows, :] += tau * (trace_rows(grid, s) + sig * dn)
    return A


def flux_rows(grid: Grid, iy, ix, s):
    """The neighbour term of side s of element i=(iy,ix) in Eq. smpm_poisson:
    -tau_{i,s} R_ij u_j = -tau_{i,s} (u_j + sigma_{i,s} n_i.grad u_j) at the nodes
    of the neighbour's facing side, as an n x n^2 matrix over the neighbour's
    nodes (element i's tau and sigma).  n_i = -n_j, so n_i.grad u_j = -(n_j.grad u_j)."""
    jy, jx = grid.neighbor(iy, ix, s)
    so = OPPOSITE[s]
    tau, sig = grid.tau(iy, ix, s), grid.sigma(iy, ix, s)
    dn_nb = outward_derivative_rows(grid, so, grid.width(jx), grid.height(jy))
    return -tau * (trace_rows(grid, so) - sig * dn_nb)


def element_rows(grid: Grid, iy, ix):
    """All rows of L at element (iy,ix): {column element: dense n^2 x n^2 block}."""
    blocks = {(iy, ix): local_block(grid, iy, ix)}
    for s in SIDES:
        nb = grid.neighbor(iy, ix, s)
        if nb is None:
            continue
        blk = blocks.setdefault(nb, np.zeros((grid.n2, grid.n2)))
        blk[grid.side_nodes(s), :] += flux_rows(grid, iy, ix, s)
    return blocks


def boundary_operator(grid: Grid):
    """T (r x nbdry): rhs = f + T g, the tau_i g_i term of Eq. smpm_poisson (its
    coefficient is the physical side's tau sigma, that of n.grad u in the row)."""
    ti, tj, tv = [], [], []
    for iy in range(grid.m_y):
        for ix in range(grid.m_x):
            e = grid.eid(iy, ix)
            for s in SIDES:
                if grid.neighbor(iy, ix, s) is not None:
                    continue
                coef = grid.tau(iy, ix, s) * grid.sigma(iy, ix, s)
                for t, l in enumerate(grid.side_nodes(s)):
                    ti.append(e * grid.n2 + int(l))
                    tj.append(grid.bdry_index(iy, ix, s, t))
                    tv.append(coef)
    return sp.csr_matrix((np.array(tv), (np.array(ti, dtype=np.int64), np.array(tj, dtype=np.int64))),
                         shape=(grid.r, grid.nbdry))


def assemble(grid: Grid):
    """Global L (CSR, r x r), Eq. smpm_poisson, and T with rhs = f + T g."""
    n2 = grid.n2
    ri, ci, vv = [], [], []
    for iy in range(grid.m_y):
        for ix in range(grid.m_x):
            e = grid.eid(iy, ix)
            for (jy, jx), blk in element_rows(grid, iy, ix).items():
                j = grid.eid(jy, jx)
                nz = np.nonzero(blk)
                ri.append(e * n2 + nz[0])
                ci.append(j * n2 + nz[1])
                vv.append(blk[nz])
    L = sp.csr_matrix((np.concatenate(vv), (np.concatenate(ri), np.concatenate(ci))),
                      shape=(grid.r, grid.r))
    return L, boundary_operator(grid)


# ---------------------------------------------------------------------------
# operator split L = A + E B and the Schur complement (Sec. 1.3)
# ---------------------------------------------------------------------------

class Split:
    """A (block diagonal), E (slot -> node inclusion), B (node -> slot fluxes).

    Slot index = (position of the side in Grid.sides()) * n + t.
    """

    def __init__(self, grid: Grid):
        self.grid = grid
        n, n2 = grid.n, grid.n2
        self.L, self.T = assemble(grid)
        self.Ablocks = [local_block(grid, iy, ix) for iy in range(grid.m_y) for ix in range(grid.m_x)]
        self.A = sp.block_diag(self.Ablocks, format="csr")
        self.sides = grid.sides()
        self.k = n * len(self.sides)
        slot_node = np.zeros(self.k, np.int64)
        bi, bj, bv = [], [], []
        for si, (iy, ix, s) in enumerate(self.sides):
            e = grid.eid(iy, ix)
            slot_node[si * n:(si + 1) * n] = e * n2 + grid.side_nodes(s)
            fr = flux_rows(grid, iy, ix, s)
            j = grid.eid(*grid.neighbor(iy, ix, s))
            nz = np.nonzero(fr)
            bi.append(si * n + nz[0])
            bj.append(j * n2 + nz[1])
            bv.append(fr[nz])
        self.slot_node = slot_node
        self.E = sp.csr_matrix((np.ones(self.k), (slot_node, np.arange(self.k))), shape=(grid.r, self.k))
        self.B = sp.csr_matrix((np.concatenate(bv), (np.concatenate(bi), np.concatenate(bj))),
                               shape=(self.k, grid.r))
        self.Ainv_blocks = [np.linalg.inv(b) for b in self.Ablocks]
        self.Ainv = sp.block_diag(self.Ainv_blocks, format="csr")

    def schur(self):
        """S = I + B A^{-1} E (Eq. schur_complement_system), sparse k x k."""
        return (sp.identity(self.k, format="csr") + self.B @ (self.Ainv @ self.E)).tocsr()


# ---------------------------------------------------------------------------
# null vectors (Sec. 1.4)
# ---------------------------------------------------------------------------

def left_null_vector(Mat, right_null, border_row=None):
    """Unit y with y^T Mat = 0 for a square matrix with one-dimensional null spaces.

    Solves the bordered system [[Mat^T, v], [b^T, 0]] [y; mu] = [0; 1] with v the
    right null vector of Mat (not in the range of Mat^T) and b a vector with
    b^T y != 0 (default: all ones).  The sign makes the entry sum positive.
    """
    m = Mat.shape[0]
    b = np.ones(m) if border_row is None else border_row
    K = sp.bmat([[sp.csr_matrix(Mat).T, sp.csr_matrix(right_null.reshape(-1, 1))],
                 [sp.csr_matrix(b.reshape(1, -1)), None]], format="csc")
    rhs = np.zeros(m + 1)
    rhs[-1] = 1.0
    sol = spla.spsolve(K, rhs)
    y = sol[:m]
    y = y / np.linalg.norm(y)
    if y.sum() < 0:
        y = -y
    return y


def project_out(u, x):
    """x - u (u^T x) for unit u (Eqs. regularize_poisson, regularize_schur)."""
    return x - u * (u @ x)


def rhs_vector(split: Split, f, g=None):
    """f + T g: the physical-side terms tau_i g_i of Eq. smpm_poisson moved to the right."""
    rhs = np.array(f, np.float64, copy=True)
    if g is not None:
        rhs = rhs + split.T @ g
    return rhs


def mean_zero(grid: Grid, u):
    """Fix the additive constant: subtract (w^T u)/(w^T 1)."""
    w = grid.quad_weights()
    return u - (w @ u) / w.sum()


def solve_unreduced(split: Split, f, g=None):
    """u* solving L u = f~, w^T u = 0, with f~ = (I - u_L u_L^T)(f + T g).

    Sec. 1.4: the right-hand side is projected out of the left null space of L
    and the solution is fixed up to a constant.  Solved with the nonsingular
    bordered matrix [[L, u_L], [w^T, 0]].  Returns (u, mu, u_L, f~); mu ~ 0
    confirms consistency.
    """
    grid = split.grid
    uL = left_null_vector(split.L, np.ones(grid.r))
    ft = project_out(uL, rhs_vector(split, f, g))
    w = grid.quad_weights()
    K = sp.bmat([[split.L, sp.csr_matrix(uL.reshape(-1, 1))],
                 [sp.csr_matrix(w.reshape(1, -1)), None]], format="csc")
    sol = spla.spsolve(K, np.concatenate([ft, [0.0]]))
    return sol[:-1], sol[-1], uL, ft


def solve_adjoint_unreduced(split: Split, c):
    """mu = K^T c for the linear map u = K (f + T g) that solve_unreduced computes.

    The paper solves only the forward problem; its adjoint is the transpose of that
    map.  Forward: u = Pi_w L^- Pi_L b with Pi_L = I - u_L u_L^T (Sec. 1.4: the
    right-hand side projected onto range L) and Pi_w = I - 1 w^T / (w^T 1) (the
    constant fixed by w^T u = 0).  Transposed: c~ = c - w (1^T c)/(w^T 1) lies in
    range(L^T) = 1-perp, and mu is the solution of L^T mu = c~ orthogonal to u_L,
    the null vector of L^T.  Solved with the nonsingular bordered matrix
    [[L^T, 1], [u_L^T, 0]].  For a loss with dLoss/du = c: dLoss/df = mu and
    dLoss/dg = T^T mu.  Returns (mu, lam, c~); lam ~ 0 confirms consistency.
    """
    grid = split.grid
    uL = left_null_vector(split.L, np.ones(grid.r))
    w = grid.quad_weights()
    c = np.asarray(c, np.float64)
    ct = c - w * (c.sum() / w.sum())
    K = sp.bmat([[split.L.T, sp.csr_matrix(np.ones((grid.r, 1)))],
                 [sp.csr_matrix(uL.reshape(1, -1)), None]], format="csc")
    sol = spla.spsolve(K, np.concatenate([ct, [0.0]]))
    return sol[:-1], sol[-1], ct


def boundary_adjoint(split: Split, mu):
    """T^T mu: the gradient with respect to the Neumann data g given dLoss/d(f + T g) = mu."""
    return split.T.T @ np.asarray(mu, np.float64)


class SchurSystem:
    """Everything the Schur route needs, built from a Split (Secs. 1.3-1.4)."""

    def __init__(self, split: Split):
        self.split = split
        self.grid = split.grid
        self.S = split.schur()
        self.k = split.k
        self.v0 = split.B @ np.ones(self.grid.r)          # right null vector of S (L 1 = 0)
        self.uL = left_null_vector(split.L, np.ones(self.grid.r))
        self.uS = left_null_vector(self.S, self.v0)

    def schur_rhs(self, f, g=None):
        """Steps 1-3 of Algorithms 1-3: f~, b_S = B A^{-1} f~, b_hat."""
        ft = project_out(self.uL, rhs_vector(self.split, f, g))
        bS = self.split.B @ (self.split.Ainv @ ft)
        bhat = project_out(self.uS, bS)
        return ft, bS, bhat

    def back_substitute(self, ft, x):
        """u = A^{-1}(f~ - E x) (Sec. 1.3), then the constant fixed by w^T u = 0."""
        u = self.split.Ainv @ (ft - self.split.E @ x)
        return mean_zero(self.grid, u)

    def solve_direct(self, f, g=None):
        """Schur route with a direct solve of S x = b_hat (bordered by u_S and v0)."""
        ft, bS, bhat = self.schur_rhs(f, g)
        K = sp.bmat([[self.S, sp.csr_matrix(self.uS.reshape(-1, 1))],
                     [sp.csr_matrix(self.v0.reshape(1, -1)), None]], format="csc")
        sol = spla.spsolve(K, np.concatenate([bhat, [0.0]]))
        x = sol[:-1]
        return self.back_substitute(ft, x), x, bhat


# ---------------------------------------------------------------------------
# block-Jacobi preconditioner (Sec. 2)
# ---------------------------------------------------------------------------

def precond_block_ids(grid: Grid, sides):
    """Block index of every slot; blocks numbered by red element in row-major order."""
    red_index = {}
    for iy in range(grid.m_y):
        for ix in range(grid.m_x):
            if (ix + iy) % 2 == 0:
                red_index[(iy, ix)] = len(red_index)
    ids = np.zeros(len(sides) * grid.n, np.int64)
    for si, (iy, ix, s) in enumerate(sides):
        owner = (iy, ix) if (ix + iy) % 2 == 0 else grid.neighbor(iy, ix, s)
        ids[si * grid.n:(si + 1) * grid.n] = red_index[owner]
    return ids, len(red_index)


class BlockJacobi:
    """M = the block diagonal of S on the checkerboard blocks; applies M^{-1}."""

    def __init__(self, sys: SchurSystem):
        self.ids, self.nblocks = precond_block_ids(sys.grid, sys.split.sides)
        self.members = [np.nonzero(self.ids == b)[0] for b in range(self.nblocks)]
        Sd = sys.S.tocsr()
        self.blocks = [Sd[m][:, m].toarray() for m in self.members]
        # A block is singular only when it is all of Gamma (a two-element grid,
        # where M = S); the pseudo-inverse is then the plain generalization.
        self.inv = []
        for b in self.blocks:
            sv = np.linalg.svd(b, compute_uv=False)
            self.inv.append(np.linalg.pinv(b, rcond=1e-11) if sv[-1] <= 1e-11 * sv[0] else np.linalg.inv(b))

    def dense(self, k):
        M = np.zeros((k, k))
        for m, b in zip(self.members, self.blocks):
            M[np.ix_(m, m)] = b
        return M

    def solve(self, x):
        y = np.zeros_like(x)
        for m, bi in zip(self.members, self.inv):
            y[m] = bi @ x[m]
        return y

    def solve_transpose(self, x):
        y = np.zeros_like(x)
        for m, bi in zip(self.members, self.inv):
            y[m] = bi.T @ x[m]
        return y


# ---------------------------------------------------------------------------
# deflation (Sec. 2, Eqs. projection1, projection2, deflated_schur)
# ---------------------------------------------------------------------------

def interfaces(grid: Grid):
    """Interfaces: vertical ones (between (iy,ix) and (iy,ix+1)) first in row-major
    order, then horizontal ones (between (iy,ix) and (iy+1,ix))."""
    out = []
    for iy in range(grid.m_y):
        for ix in range(grid.m_x - 1):
            out.append(((iy, ix), E, (iy, ix + 1), W))
    for iy in range(grid.m_y - 1):
        for ix in range(grid.m_x):
            out.append(((iy, ix), N, (iy + 1, ix), S))
    return out


def deflation_matrix(grid: Grid, sides):
    """Z (k x d): column j is 1 on the 2n slots of the two sides of interface j."""
    where = {side: i for i, side in enumerate(sides)}
    rows, cols = [], []
    for j, (a, sa, b, sb) in enumerate(interfaces(grid)):
        for (iy, ix), s in ((a, sa), (b, sb)):
            si = where[(iy, ix, s)]
            rows.extend(range(si * grid.n, (si + 1) * grid.n))
            cols.extend([j] * grid.n)
    d = len(interfaces(grid))
    return sp.csr_matrix((np.ones(len(rows)), (rows, cols)), shape=(len(sides) * grid.n, d))


class Deflation:
    """Z, C = Z^T S Z, a pseudo-inverse G of C and the projections P, Q.

    C inherits the rank deficiency of S (Sec. 2); C\\ then acts on
    (I - u_C u_C^T) Z^T b (Eq. deflated_schur).  The oracle uses the
    Moore-Penrose pseudo-inverse from numpy's SVD for every application of C^{-1}.
    """

    def __init__(self, sys: SchurSystem, G=None):
        self.sys = sys
        self.Z = deflation_matrix(sys.grid, sys.split.sides)
        self.d = self.Z.shape[1]
        self.C = (self.Z.T @ (sys.S @ self.Z)).toarray() if self.d else np.zeros((0, 0))
        # scale of C: ||Z||^2 ||S||, so that a d = 1 coarse matrix can be recognised as singular
        self.scale = 2 * sys.grid.n * spla.norm(sys.S, 1)
        if self.d:
            U, sv, Vt = np.linalg.svd(self.C)
            self.singvals = sv
            self.singular = bool(sv[-1] <= 1e-11 * self.scale)
            self.uC = U[:, -1].copy() if self.singular else None
        else:
            self.singvals = np.zeros(0)
            self.singular = False
            self.uC = None
        if G is None:
            if self.d:
                keep = sv > 1e-11 * self.scale
                G = (Vt[keep].T / sv[keep]) @ U[:, keep].T
            else:
                G = np.zeros((0, 0))
        self.G = G
        self.SZ = (sys.S @ self.Z).toarray() if self.d else np.zeros((sys.k, 0))

    def P(self, x):
        """P x = x - S Z G Z^T x (Eq. projection1)."""
        return x - self.SZ @ (self.G @ (self.Z.T @ x))

    def Q(self, x):
        """Q x = x - Z G Z^T S x (Eq. projection2)."""
        return x - self.Z @ (self.G @ (self.Z.T @ (self.sys.S @ x)))

    def coarse_part(self, bhat):
        """Z C\\ (Z^T - u_C u_C^T Z^T) b_hat (Algorithm 3, coarse solution)."""
        if self.d == 0:
            return np.zeros_like(bhat)
        c = self.Z.T @ bhat
        if self.uC is not None:
            c = c - self.uC * (self.uC @ c)
        return self.Z @ (self.G @ c)


# ---------------------------------------------------------------------------
# GMRES and Algorithms 1-3
# ---------------------------------------------------------------------------

def gmres(apply_op, b, tol=1e-10, maxit=400):
    """Textbook GMRES from x0 = 0: Arnoldi with modified Gram-Schmidt, the
    least-squares problem min ||beta e1 - H y|| re-solved by lstsq each step.

    Stops when the least-squares residual <= tol * beta.  Returns (x, iters, history).
    """
    beta = np.linalg.norm(b)
    hist = [beta]
    if beta == 0.0:
        return np.zeros_like(b), 0, hist
    m = min(maxit, b.size)
    V = np.zeros((b.size, m + 1))
    H = np.zeros((m + 1, m))
    V[:, 0] = b / beta
    y = np.zeros(0)
    j = 0
    for j in range(m):
        w = apply_op(V[:, j])
        for i in range(j + 1):
            H[i, j] = V[:, i] @ w
            w = w - H[i, j] * V[:, i]
        H[j + 1, j] = np.linalg.norm(w)
        e1 = np.zeros(j + 2)
        e1[0] = beta
        y, *_ = np.linalg.lstsq(H[:j + 2, :j + 1], e1, rcond=None)
        res = np.linalg.norm(e1 - H[:j + 2, :j + 1] @ y)
        hist.append(res)
        if res <= tol * beta or H[j + 1, j] == 0.0:
            break
        V[:, j + 1] = w / H[j + 1, j]
    return V[:, :len(y)] @ y, j + 1, hist


def block_orthonormalize(W, drop):
    """Q (k x r), R (r x s) with W = Q R: the columns of W taken in order, each made
    orthogonal to the kept ones by Gram-Schmidt applied twice; a column whose
    remaining part is <= drop times its own norm adds no vector (rank deflation) and
    keeps only its coefficients on the earlier vectors."""
    k, s = W.shape
    Q = []
    R = np.zeros((s, s))
    for i in range(s):
        w = W[:, i].copy()
        nrm0 = np.linalg.norm(w)
        for _ in range(2):
            for c, q in enumerate(Q):
                h = q @ w
                R[c, i] += h
                w = w - h * q
        nrm = np.linalg.norm(w)
        if nrm0 > 0.0 and nrm > drop * nrm0:
            R[len(Q), i] = nrm
            Q.append(w / nrm)
    r = len(Q)
    return (np.column_stack(Q) if r else np.zeros((k, 0))), R[:r, :]


def block_gmres(apply_op, B, tol=1e-10, maxit=400, ref=None, drop=1e-6):
    """Block GMRES from X0 = 0 for op(X) = B with s columns (not in the paper: its
    step 4 solved for all right-hand sides in one block Krylov space).  The iterate
    after j block steps minimizes every column's residual over the block Krylov space
    span{B, op B, ..., op^{j-1} B}.  Block Arnoldi: the new block op(V_j) is made
    orthogonal to every basis vector by block classical Gram-Schmidt applied twice,
    then orthonormalized within itself by block_orthonormalize (whose dropped columns
    shrink the next block); the least-squares problem min ||E_1 R_0 - H Y|| is
    re-solved by lstsq at every step.  Stops when every column's least-squares
    residual is <= tol * ref[c] (ref: the columns' norms of B by default), when no
    vector is added, or after maxit block steps.  Returns (X, steps, history), history
    the per-column residuals after each step (the first entry those of B)."""
    k, s = B.shape
    ref = np.linalg.norm(B, axis=0) if ref is None else np.asarray(ref, float)
    V0, R0 = block_orthonormalize(B, drop)
    hist = [np.linalg.norm(B, axis=0)]
    if V0.shape[1] == 0:
        return np.zeros_like(B), 0, hist
    V = V0
    blocks = [V0.shape[1]]      # sizes of the blocks V_0, V_1, ...
    Hcols = []                  # block columns of H, each (rows so far) x r_j
    Y = np.zeros((0, s))
    X = np.zeros_like(B)
    steps = 0
    for j in range(maxit):
        n_old = V.shape[1]
        lo = n_old - blocks[-1]
        Vj = V[:, lo:]
        Wb = apply_op(Vj)
        h = V.T @ Wb
        Wb = Wb - V @ h
        h2 = V.T @ Wb
        Wb = Wb - V @ h2
        h = h + h2
        Vn, Rn = block_orthonormalize(Wb, drop)
        Hcols.append(np.vstack([h, Rn]))
        rows = n_old + Vn.shape[1]
        H = np.zeros((rows, n_old))
        c0 = 0
        for hc in Hcols:
            H[:hc.shape[0], c0:c0 + hc.shape[1]] = hc
            c0 += hc.shape[1]
        E = np.zeros((rows, s))
        E[:R0.shape[0], :] = R0
        Y, *_ = np.linalg.lstsq(H, E, rcond=None)
        res = np.linalg.norm(E - H @ Y, axis=0)
        hist.append(res)
        steps = j + 1
        X = V @ Y
        if np.all(res <= tol * ref) or Vn.shape[1] == 0:
            break
        V = np.hstack([V, Vn])
        blocks.append(Vn.shape[1])
    return X, steps, hist


class Method:
    """Algorithms 1, 2 and 3 of the paper on one grid."""

    def __init__(self, grid: Grid, G=None):
        self.grid = grid
        self.split = Split(grid)
        self.sys = SchurSystem(self.split)
        self.M = BlockJacobi(self.sys)
        self.defl = Deflation(self.sys, G)

    def solve(self, f, g=None, variant=3, tol=1e-10, maxit=400):
        """Returns (u, info).  variant 1: GMRES(S, b_S); 2: with M; 3: deflated + M."""
        sys = self.sys
        ft, bS, bhat = sys.schur_rhs(f, g)                  # steps 1-3
        S = sys.S
        if variant == 1:
            x, it, hist = gmres(lambda v: S @ v, bhat, tol, maxit)
        elif variant == 2:
            xp, it, hist = gmres(lambda v: S @ self.M.solve(v), bhat, tol, maxit)
            x = self.M.solve(xp)
        else:
            P = self.defl.P
            x1, it, hist = gmres(lambda v: P(S @ self.M.solve(v)), P(bhat), tol, maxit)  # step 4
            x1 = self.defl.Q(self.M.solve(x1))              # step 5
            x2 = self.defl.coarse_part(bhat)                # steps 6-7
            x = x1 + x2                                     # step 8
        u = sys.back_substitute(ft, x)                      # step 9 (+ constant fixed)
        true_res = np.linalg.norm(bhat - S @ x) / max(np.linalg.norm(bhat), 1e-300)
        return u, {"iters": it, "history": hist, "x": x, "bhat": bhat, "true_rel_res": true_res}

    def solve_block(self, F, variant=3, tol=1e-10, maxit=400, drop=1e-6):
        """Algorithm 3 (or 1, 2) for the columns of F (r x s) with step 4 solved by
        block_gmres over all columns at once, stopping at tol * |b_hat| per column.
        Returns (U, info)."""
        sys = self.sys
        S = sys.S
        cols = [sys.schur_rhs(F[:, c]) for c in range(F.shape[1])]
        Bh = np.column_stack([c[2] for c in cols])
        ref = np.linalg.norm(Bh, axis=0)
        Minv = lambda Z: np.column_stack([self.M.solve(Z[:, c]) for c in range(Z.shape[1])])
        if variant == 1:
            X, it, hist = block_gmres(lambda Z: S @ Z, Bh, tol, maxit, ref, drop)
        elif variant == 2:
            Xp, it, hist = block_gmres(lambda Z: S @ Minv(Z), Bh, tol, maxit, ref, drop)
            X = Minv(Xp)
        else:
            P = self.defl.P
            Pc = lambda Z: np.column_stack([P(Z[:, c]) for c in range(Z.shape[1])])
            X1, it, hist = block_gmres(lambda Z: Pc(S @ Minv(Z)), Pc(Bh), tol, maxit, ref, drop)
            X1 = Minv(X1)
            X = np.column_stack([self.defl.Q(X1[:, c]) + self.defl.coarse_part(Bh[:, c])
                                 for c in range(Bh.shape[1])])
        U = np.column_stack([sys.back_substitute(cols[c][0], X[:, c]) for c in range(Bh.shape[1])])
        true_res = np.linalg.norm(Bh - S @ X, axis=0) / np.maximum(ref, 1e-300)
        return U, {"iters": it, "history": hist, "X": X, "Bhat": Bh, "true_rel_res": true_res}


# ---------------------------------------------------------------------------
# element-local evaluation for sampled checks on large grids
# ---------------------------------------------------------------------------

class LocalOperators:
    """Element-local pieces of A^{-1} and B, built on demand, for grids too large
    for global assembly.  Evaluates single sides of S y from their definition."""

    def __init__(self, grid: Grid):
        self.grid = grid
        self.sides = grid.sides()
        self.where = {side: i for i, side in enumerate(self.sides)}
        self._inv = {}

    def Ainv(self, iy, ix):
        if (iy, ix) not in self._inv:
            self._inv[(iy, ix)] = np.linalg.inv(local_block(self.grid, iy, ix))
        return self._inv[(iy, ix)]

    def element_slots(self, iy, ix):
        """(slot indices, local node indices) of all slots of one element."""
        n = self.grid.n
        sl, nodes = [], []
        for s in SIDES:
            if (iy, ix, s) in self.where:
                si = self.where[(iy, ix, s)]
                sl.extend(range(si * n, (si + 1) * n))
                nodes.extend(self.grid.side_nodes(s))
        return np.array(sl, np.int64), np.array(nodes, np.int64)

    def schur_side(self, iy, ix, s, y):
        """(S y) on the slots of side s of element (iy, ix):
        y there + (flux rows of that side) A_j^{-1} E_j y_j, j the neighbour."""
        grid = self.grid
        n = grid.n
        si = self.where[(iy, ix, s)]
        out = y[si * n:(si + 1) * n].copy()
        jy, jx = grid.neighbor(iy, ix, s)
        sl, nodes = self.element_slots(jy, jx)
        zj = np.zeros(grid.n2)
        np.add.at(zj, nodes, y[sl])
        out += flux_rows(grid, iy, ix, s) @ (self.Ainv(jy, jx) @ zj)
        return out
