"""Pins of the oracle's adjoint (the transpose of the forward solution map) to the
forward oracle and to the mathematics: the dot-product identity, the explicit
transpose on a tiny grid, exact central differences of a quadratic loss, the
constraints the adjoint satisfies, and its invariance to the part of the
cotangent the forward map cannot see."""
import numpy as np
import pytest

import smpm_workloads as wl
from oracle import smpm_oracle as O

GRIDS = {
    "uniform_3x3_n5": lambda: O.Grid(5, wl.uniform_breaks(3), wl.uniform_breaks(3)),
    "stretched_4x3_n6": lambda: O.Grid(6, np.array([0.0, 0.1, 0.25, 0.5, 1.0]), np.array([0.0, 0.3, 0.6, 1.0])),
    "two_2x1_n4": lambda: O.Grid(4, wl.uniform_breaks(2), wl.uniform_breaks(1)),
}


def forward(split, f, g=None):
    return O.solve_unreduced(split, f, g)[0]


@pytest.mark.parametrize("name", sorted(GRIDS))
def test_dot_product_identity(name):
    """<c, u(f, g)> = <K^T c, f> + <T^T K^T c, g> for random f, g, c."""
    g = GRIDS[name]()
    split = O.Split(g)
    V = wl.random_vectors(71, 3, g.r)
    gb = wl.random_vectors(72, 1, g.nbdry)[0]
    u = forward(split, V[0], gb)
    mu, lam, _ = O.solve_adjoint_unreduced(split, V[1])
    lhs = V[1] @ u
    rhs = mu @ V[0] + O.boundary_adjoint(split, mu) @ gb
    assert abs(lam) < 1e-9 * np.linalg.norm(V[1])
    assert abs(lhs - rhs) <= 1e-10 * np.linalg.norm(V[1]) * np.linalg.norm(u)


def test_explicit_transpose_tiny_grid():
    """Brute force: the forward map assembled column by column, then transposed."""
    g = O.Grid(4, wl.uniform_breaks(2), wl.uniform_breaks(2))
    split = O.Split(g)
    K = np.stack([forward(split, e) for e in np.eye(g.r)], axis=1)
    for c in wl.random_vectors(73, 3, g.r):
        mu, _, _ = O.solve_adjoint_unreduced(split, c)
        assert np.abs(mu - K.T @ c).max() <= 1e-10 * np.abs(K.T @ c).max()


def test_constraints_and_invariance():
    """L^T mu = c~, 1^T c~ = 0, u_L^T mu = 0; adding any multiple of w to c leaves mu
    unchanged (the forward output always has w^T u = 0)."""
    g = GRIDS["stretched_4x3_n6"]()
    split = O.Split(g)
    c = wl.random_vectors(74, 1, g.r)[0]
    mu, _, ct = O.solve_adjoint_unreduced(split, c)
    uL = O.left_null_vector(split.L, np.ones(g.r))
    assert abs(ct.sum()) < 1e-12 * np.abs(c).sum()
    assert np.abs(split.L.T @ mu - ct).max() < 1e-9 * np.abs(ct).max()
    assert abs(uL @ mu) < 1e-12 * np.linalg.norm(mu)
    mu2, _, _ = O.solve_adjoint_unreduced(split, c + 3.7 * g.quad_weights())
    assert np.abs(mu2 - mu).max() <= 1e-10 * np.abs(mu).max()


def test_quadratic_loss_central_differences():
    """Loss = |u(f, g) - u_t|^2 is quadratic in (f, g), so central differences are
    exact up to rounding; they must equal <mu, df> + <T^T mu, dg> with c = 2(u - u_t)."""
    g = GRIDS["uniform_3x3_n5"]()
    split = O.Split(g)
    x, y = g.node_coords()
    f = wl.eval_fourier(wl.random_fourier_params(75, 20, 4), x, y, 1.0, 1.0)
    gb = wl.eval_edge(wl.random_edge_params(76), *g.boundary_arc(), 1.0, 1.0)
    ut = wl.eval_fourier(wl.random_fourier_params(77, 20, 4), x, y, 1.0, 1.0)

    def loss(ff, gg):
        d = forward(split, ff, gg) - ut
        return d @ d

    u = forward(split, f, gb)
    mu, _, _ = O.solve_adjoint_unreduced(split, 2.0 * (u - ut))
    dg_grad = O.boundary_adjoint(split, mu)
    h = 1e-3
    for df, dg in zip(wl.random_directions(78, 4, g.r), wl.random_directions(79, 4, g.nbdry)):
        fd = (loss(f + h * df, gb + h * dg) - loss(f - h * df, gb - h * dg)) / (2 * h)
        an = mu @ df + dg_grad @ dg
        assert abs(fd - an) <= 1e-8 * max(1.0, abs(an)), (fd, an)
