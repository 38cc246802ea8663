"""Pins of the oracle's operator, Schur route and Algorithm 3 against facts the
paper and the mathematics fix: polynomial exactness, the constant right null
space, conservation at the special penalty, manufactured solutions, the block
elimination identity, projection algebra and brute-force GMRES."""
import json
import math
import os

import numpy as np
import pytest

import smpm_workloads as wl
from oracle import smpm_oracle as O


def grid(m_x, m_y, n, Lx=1.0, Ly=1.0, **kw):
    return O.Grid(n, wl.uniform_breaks(m_x, Lx), wl.uniform_breaks(m_y, Ly), **kw)


# ---------------------------------------------------------------- operator L

@pytest.mark.parametrize("robin", O.ROBIN_MODES)
@pytest.mark.parametrize("alpha", [8.0, -8.0, -1.0, 3.0])
def test_polynomial_exactness(alpha, robin):
    """For a global polynomial of degree <= N per variable the interface jumps vanish,
    so L p = lap p at every node not on the physical boundary, and
    lap p + tau sigma dp/dn there (Eq. smpm_poisson), for every reading of sigma."""
    g = O.Grid(6, [0.0, 0.3, 1.0, 1.2], [0.0, 0.5, 1.1], alpha_int=alpha, alpha_phys=alpha, robin=robin)
    L, _ = O.assemble(g)
    x, y = g.node_coords()
    a, b = 4, 3
    p = x ** a * y ** b
    lap = a * (a - 1) * x ** (a - 2) * y ** b + b * (b - 1) * x ** a * y ** (b - 2)
    px = a * x ** (a - 1) * y ** b
    py = b * x ** a * y ** (b - 1)
    want = lap.copy()
    for iy in range(g.m_y):
        for ix in range(g.m_x):
            e = g.eid(iy, ix)
            for s in O.SIDES:
                if g.neighbor(iy, ix, s) is not None:
                    continue
                coef = g.tau(iy, ix, s) * g.sigma(iy, ix, s)
                for l in g.side_nodes(s):
                    i = e * g.n2 + l
                    dn = {O.W: -px[i], O.E: px[i], O.S: -py[i], O.N: py[i]}[s]
                    want[i] += coef * dn
    got = L @ p
    assert np.abs(got - want).max() <= 1e-9 * np.abs(want).max()


@pytest.mark.parametrize("dims", [(3, 3, 5), (4, 2, 6), (2, 1, 4)])
def test_constant_right_null_space_and_rank(dims):
    """L 1 = 0 and rank L = r - 1 (Sec. 1.4)."""
    g = grid(*dims)
    L, _ = O.assemble(g)
    Ld = L.toarray()
    assert np.abs(Ld @ np.ones(g.r)).max() <= 1e-12 * np.abs(Ld).max()
    sv = np.linalg.svd(Ld, compute_uv=False)
    assert sv[-1] <= 1e-13 * sv[0]
    assert sv[-2] >= 1e-9 * sv[0]


def test_conservation_at_special_penalty():
    """On a grid of equal square elements (non-square domain), alpha = -1 on
    interfaces and -2 on physical sides make GLL summation by parts cancel the
    Laplacian's boundary fluxes: the weighted column sums vanish, w^T L = 0 (the
    value jumps cancel pairwise because tau is equal on both sides).  This pins the
    tau scaling (omega_0, h_e^2), the Robin length sigma = h_e/2 and the corner
    treatment independently of the default penalty."""
    g = O.Grid(7, wl.uniform_breaks(3, 1.2), wl.uniform_breaks(2, 0.8), alpha_int=-1.0, alpha_phys=-2.0)
    L, T = O.assemble(g)
    w = g.quad_weights()
    Ld = L.toarray()
    assert np.abs(w @ Ld).max() <= 1e-12 * np.abs(Ld).max()
    # discrete compatibility is the quadrature form of int f = oint g
    gb = np.arange(g.nbdry, dtype=float) % 5 - 2.0
    xs, xn, yw, ye = g.boundary_arc()
    # w^T T g = (tau sigma)_phys * (GLL side quadrature) = -oint g
    qx = np.concatenate([g.omega * g.width(ix) / 2 for ix in range(g.m_x)])
    qy = np.concatenate([g.omega * g.height(iy) / 2 for iy in range(g.m_y)])
    oint = qx @ gb[:g.m_x * g.n] + qx @ gb[g.m_x * g.n:2 * g.m_x * g.n] \
        + qy @ gb[2 * g.m_x * g.n:2 * g.m_x * g.n + g.m_y * g.n] + qy @ gb[2 * g.m_x * g.n + g.m_y * g.n:]
    assert abs(w @ (T @ gb) + oint) <= 1e-12 * np.abs(gb).sum()


def _weighted_column_sums(g):
    L, _ = O.assemble(g)
    Ld = L.toarray()
    return np.abs(g.quad_weights() @ Ld).max() / np.abs(Ld).max()


def test_conservation_literal_robin_nonuniform():
    """R = I + n.grad as printed (sigma = 1) with tau = 2 alpha/(omega_0 h_perp): GLL
    summation by parts turns w^T L u into side quadratures of
    (1 + alpha_i + alpha_j)(jump of the normal derivative) + (alpha_i - alpha_j)(value
    jump) on interfaces and (1 + alpha_phys) dn u on the boundary, so alpha = -1/2 on
    interfaces and -1 on physical sides give w^T L = 0 on any Cartesian grid,
    non-uniform and non-square elements included.  Pins tau ~ 1/h_perp, sigma = 1
    and the corner sums of the literal reading."""
    g = O.Grid(6, [0.0, 0.3, 1.0, 1.2], [0.0, 0.5, 1.1, 1.25], alpha_int=-0.5, alpha_phys=-1.0,
               robin="literal")
    assert _weighted_column_sums(g) <= 1e-12
    # the same penalty under the other readings is not conservative on this grid
    for robin in ("min", "reference"):
        g2 = O.Grid(6, [0.0, 0.3, 1.0, 1.2], [0.0, 0.5, 1.1, 1.25], alpha_int=-0.5, alpha_phys=-1.0,
                    robin=robin)
        assert _weighted_column_sums(g2) > 1e-6


def test_conservation_reference_robin_uniform_nonsquare():
    """sigma = h_perp/2, tau = 2 alpha/(omega_0 h_perp^2): the side terms weigh
    (alpha/h_perp)(value jump) + (alpha/2)(derivative jump), so alpha = -1 on
    interfaces and -2 on physical sides conserve whenever h_perp agrees across each
    interface (uniform widths and heights), also on non-square elements.  The
    min(w, h) reading is not conservative there."""
    xb, yb = wl.uniform_breaks(3, 1.5), wl.uniform_breaks(4, 0.8)   # w = 0.5, h = 0.2
    g = O.Grid(7, xb, yb, alpha_int=-1.0, alpha_phys=-2.0, robin="reference")
    assert _weighted_column_sums(g) <= 1e-12
    g2 = O.Grid(7, xb, yb, alpha_int=-1.0, alpha_phys=-2.0, robin="min")
    assert _weighted_column_sums(g2) > 1e-6


@pytest.mark.parametrize("robin", O.ROBIN_MODES)
def test_manufactured_non_square_elements(robin):
    """Spectral convergence in n on 4 x 3 elements of aspect 1.5 ([0,2] x [0,1]) and on
    a stretched grid (aspect up to 4) at the default penalty, for every reading of
    the Robin operator (the discretization is consistent for any sigma: a smooth
    solution has zero jumps of u + sigma n.grad u)."""
    for xb, yb in ((wl.uniform_breaks(4, 2.0), wl.uniform_breaks(3, 1.0)),
                   (np.array([0.0, 0.1, 0.25, 0.5, 1.0]), np.array([0.0, 0.3, 0.6, 1.0]))):
        Lx, Ly = xb[-1], yb[-1]
        errs = []
        for n in (5, 7, 9, 11):
            g = O.Grid(n, xb, yb, robin=robin)
            x, y = g.node_coords()
            u, f = wl.manufactured_cos(x, y, 1, Lx, Ly)
            uh, mu, _, _ = O.solve_unreduced(O.Split(g), f)
            errs.append(np.abs(uh - O.mean_zero(g, u)).max())
        for a, b in zip(errs, errs[1:]):
            assert b < a / 50.0, (robin, errs)
        assert errs[-1] < 1e-9, (robin, errs)


def test_left_null_vector_matches_svd():
    g = grid(3, 2, 5)
    L, _ = O.assemble(g)
    uL = O.left_null_vector(L, np.ones(g.r))
    U, sv, Vt = np.linalg.svd(L.toarray())
    u = U[:, -1] * np.sign(U[:, -1].sum())
    assert np.abs(uL - u).max() < 1e-10
    assert np.abs(uL @ L.toarray()).max() < 1e-10 * sv[0]


def _manufactured_error(n, m, lam=1, Lx=1.0, Ly=1.0):
    g = grid(m, m, n, Lx, Ly)
    split = O.Split(g)
    x, y = g.node_coords()
    u, f = wl.manufactured_cos(x, y, lam, Lx, Ly)
    uh, mu, _, _ = O.solve_unreduced(split, f)
    return np.abs(uh - O.mean_zero(g, u)).max(), mu


def test_manufactured_spectral_convergence():
    """Error decays exponentially in n on a fixed 4x4 grid until it meets the rounding
    plateau of the ill-conditioned spectral operators (Sec. 3.1 notes the same
    non-monotone floor at the largest orders)."""
    errs = [_manufactured_error(n, 4)[0] for n in (4, 6, 8, 10, 12, 14)]
    for a, b in zip(errs[:4], errs[1:4]):
        assert b < a / 100.0, errs
    assert max(errs[3:]) < 1e-10, errs


def test_manufactured_non_square_and_h_convergence():
    e1 = _manufactured_error(6, 2, 1, 2.0, 1.0)[0]
    e2 = _manufactured_error(6, 4, 1, 2.0, 1.0)[0]
    assert e2 < e1 / 10.0   # polynomial in h, order well above 2 at N=5
    assert e2 < 1e-4


def test_nonzero_neumann_data():
    """u = sin(pi x/2) cos(pi y) on [0,1]^2: the west edge carries g = -(pi/2) cos(pi y)."""
    errs = []
    for n in (6, 10):
        g = grid(3, 3, n)
        split = O.Split(g)
        x, y = g.node_coords()
        u = np.sin(math.pi * x / 2) * np.cos(math.pi * y)
        f = -(math.pi ** 2 / 4 + math.pi ** 2) * u
        xs, xn, yw, ye = g.boundary_arc()
        gb = np.concatenate([0 * xs, 0 * xn, -(math.pi / 2) * np.cos(math.pi * yw), 0 * ye])
        uh, mu, _, _ = O.solve_unreduced(split, f, gb)
        errs.append(np.abs(uh - O.mean_zero(g, u)).max())
    assert errs[1] < errs[0] / 100 and errs[1] < 1e-7, errs


# ---------------------------------------------------------------- Schur route

@pytest.fixture(scope="module")
def c1_method():
    w = wl.workload("c1")
    g = O.Grid(w.n, w.x_breaks, w.y_breaks)
    return O.Method(g)


def test_split_identity(c1_method):
    sp_ = c1_method.split
    assert abs(sp_.L - sp_.A - sp_.E @ sp_.B).max() == 0.0
    g = c1_method.grid
    d = len(O.interfaces(g))
    assert sp_.k == 2 * d * g.n


def test_schur_null_spaces(c1_method):
    """S v0 = 0 with v0 = B 1; rank S = k - 1; the left null vector of S is E^T u_L (Sec. 1.4)."""
    sys = c1_method.sys
    S = sys.S.toarray()
    assert np.abs(S @ sys.v0).max() <= 1e-11 * np.abs(sys.v0).max()
    sv = np.linalg.svd(S, compute_uv=False)
    assert sv[-1] <= 1e-13 * sv[0] and sv[-2] >= 1e-8 * sv[0]
    eu = sys.split.E.T @ sys.uL
    eu /= np.linalg.norm(eu)
    # null vectors are fixed only up to sign
    assert min(np.abs(sys.uS - eu).max(), np.abs(sys.uS + eu).max()) < 1e-10


def test_block_elimination_identity(c1_method):
    """[[A, E], [B, -I]] [u; v] = [f; 0] reproduces L u = f and v = B u (Eqs. blocksystem,
    operator_decomp, schur_complement_system)."""
    sys = c1_method.sys
    sp_ = sys.split
    g = sys.grid
    x, y = g.node_coords()
    _, f = wl.manufactured_cos(x, y)
    ft = O.project_out(sys.uL, f)
    u_direct, x_S, bhat = sys.solve_direct(f)
    u_un, mu, _, _ = O.solve_unreduced(sp_, f)
    assert np.linalg.norm(u_direct - u_un) <= 1e-12 * np.linalg.norm(u_un)
    # v = B u for the unnormalized back-substituted u
    u_raw = sp_.Ainv @ (ft - sp_.E @ x_S)
    assert np.linalg.norm(sp_.L @ u_raw - ft) <= 1e-10 * np.linalg.norm(ft)
    assert np.linalg.norm(sp_.B @ u_raw - x_S) <= 1e-10 * np.linalg.norm(x_S)
    # b_S is already orthogonal to u_S when f~ is consistent
    _, bS, _ = sys.schur_rhs(f)
    assert abs(sys.uS @ bS) <= 1e-11 * np.linalg.norm(bS)


def test_block_jacobi_structure(c1_method):
    """Interior blocks hold 8n slots, edge blocks 6n, corner blocks 4n (Fig. 2); the
    sub-blocks coupling slots of one element are identities."""
    M = c1_method.M
    g = c1_method.grid
    n = g.n
    sizes = sorted(len(m) for m in M.members)
    assert set(sizes) <= {4 * n, 6 * n, 8 * n}
    owner = np.concatenate([[O.Grid.eid(g, iy, ix)] * n for (iy, ix, s) in g.sides()])
    for m, blk in zip(M.members, M.blocks):
        own = owner[m]
        for e in np.unique(own):
            sel = own == e
            assert np.abs(blk[np.ix_(sel, sel)] - np.eye(sel.sum())).max() == 0.0


def test_deflation_algebra(c1_method):
    """C tau_hat = 0 (v0 lies in range Z on a uniform grid), P^2 = P, Q^2 = Q,
    P S Z = 0, S Q = P S (Eqs. projection1, projection2)."""
    m = c1_method
    D = m.defl
    S = m.sys.S.toarray()
    k = m.sys.k
    assert D.singular
    rng = np.random.default_rng(1)
    X = rng.standard_normal((k, 3))
    for x in X.T:
        Px = D.P(x)
        Qx = D.Q(x)
        assert np.linalg.norm(D.P(Px) - Px) <= 1e-11 * np.linalg.norm(x)
        assert np.linalg.norm(D.Q(Qx) - Qx) <= 1e-11 * np.linalg.norm(x)
        assert np.linalg.norm(S @ Qx - D.P(S @ x)) <= 1e-11 * np.linalg.norm(x)
    PSZ = np.column_stack([D.P(c) for c in D.SZ.T])
    assert np.abs(PSZ).max() <= 1e-11 * np.abs(D.SZ).max()


@pytest.mark.parametrize("variant", [1, 2, 3])
def test_algorithms_match_direct(c1_method, variant):
    g = c1_method.grid
    x, y = g.node_coords()
    _, f = wl.manufactured_cos(x, y)
    u_ref, *_ = O.solve_unreduced(c1_method.split, f)
    u, info = c1_method.solve(f, variant=variant, tol=1e-13)
    assert np.linalg.norm(u - u_ref) <= 1e-11 * np.linalg.norm(u_ref)
    assert info["true_rel_res"] < 1e-11


def test_correctness_does_not_depend_on_G(c1_method):
    """For any fixed G, S Q_G = P_G S, so Algorithm 3 still returns the solution; only
    the iteration count depends on G being the pseudo-inverse of C."""
    g = c1_method.grid
    x, y = g.node_coords()
    _, f = wl.manufactured_cos(x, y)
    u_ref, *_ = O.solve_unreduced(c1_method.split, f)
    D = c1_method.defl
    G = D.G + 0.05 * np.random.default_rng(7).standard_normal(D.G.shape) * np.abs(D.G).max()
    m2 = O.Method(g, G=G)
    u, info = m2.solve(f, variant=3, tol=1e-13)
    assert np.linalg.norm(u - u_ref) <= 1e-10 * np.linalg.norm(u_ref)


def test_edge_case_two_elements():
    """2x1 grid: one interface, C = 0 (tau_hat spans its null space), so G = 0,
    P = Q = I and Algorithm 3 reduces to Algorithm 2."""
    g = grid(2, 1, 6)
    m = O.Method(g)
    assert m.defl.d == 1
    assert abs(m.defl.C[0, 0]) <= 1e-12 * np.abs(m.sys.S.toarray()).max() * 2 * g.n
    x, y = g.node_coords()
    f = np.cos(math.pi * x) + 0.3 * np.sin(2 * y)
    u2, i2 = m.solve(f, variant=2, tol=1e-13)
    u3, i3 = m.solve(f, variant=3, tol=1e-13)
    u_ref, *_ = O.solve_unreduced(m.split, f)
    assert np.linalg.norm(u3 - u_ref) <= 1e-11 * np.linalg.norm(u_ref)
    assert np.linalg.norm(u2 - u3) <= 1e-11 * np.linalg.norm(u_ref)


def test_brute_force_full_gmres():
    """GMRES run to J = k on a tiny grid reproduces the direct Schur solution."""
    g = grid(2, 2, 4)
    m = O.Method(g)
    x, y = g.node_coords()
    f = np.sin(3 * x) * np.cos(2 * y)
    u_ref, *_ = O.solve_unreduced(m.split, f)
    u, info = m.solve(f, variant=1, tol=1e-15, maxit=m.sys.k)
    assert np.linalg.norm(u - u_ref) <= 1e-10 * np.linalg.norm(u_ref)


def test_local_schur_matches_global(c1_method):
    """The element-local evaluation used for sampled checks equals the global S."""
    g = c1_method.grid
    loc = O.LocalOperators(g)
    y = np.random.default_rng(3).standard_normal(c1_method.sys.k)
    Sy = c1_method.sys.S @ y
    for si, (iy, ix, s) in enumerate(g.sides()):
        got = loc.schur_side(iy, ix, s, y)
        assert np.abs(got - Sy[si * g.n:(si + 1) * g.n]).max() <= 1e-12 * np.abs(Sy).max()


# ---------------------------------------------------------------- paper trends

def test_paper_trends(golden_dir):
    """Sec. 3.3: block-Jacobi preconditioned counts nearly independent of p; Sec. 3.2:
    deflation does not lose to the unpreconditioned method as h shrinks."""
    crit = json.load(open(os.path.join(golden_dir, "paper_iteration_counts.json")))["test_criteria"]
    counts = []
    for n in (5, 9, 13):
        g = grid(4, 4, n)
        m = O.Method(g)
        x, y = g.node_coords()
        _, f = wl.manufactured_cos(x, y, lam=7)
        counts.append(m.solve(f, variant=3, tol=1e-10)[1]["iters"])
    assert max(counts) <= crit["p_independence_ratio_max"] * min(counts), counts
    g = grid(12, 12, 5)
    m = O.Method(g)
    x, y = g.node_coords()
    _, f = wl.manufactured_cos(x, y, lam=7)
    i1 = m.solve(f, variant=1, tol=1e-10)[1]["iters"]
    i3 = m.solve(f, variant=3, tol=1e-10)[1]["iters"]
    assert i3 <= i1, (i1, i3)
