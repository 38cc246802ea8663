"""Pins of the oracle's block GMRES (all right-hand sides of Algorithm 3's step 4 in
one block Krylov space) against facts fixed by the mathematics rather than by the
oracle's own code: the minimal-residual property over an explicitly built block
Krylov basis (brute force), reduction to plain GMRES for one column, termination at
the dimension of the space, rank deflation of dependent columns, the monotone
advantage over separate Krylov spaces, and the direct solution of the paper's
system."""
import numpy as np
import pytest

import smpm_workloads as wl
from oracle import smpm_oracle as O


def _krylov_min_residual(A, B, j):
    """min over x in span{B, AB, ..., A^{j-1} B} of |b_c - A x| per column, from an
    orthonormal basis of the explicit block Krylov matrix (numpy QR with a rank cut)."""
    blocks = [B]
    for _ in range(j - 1):
        blocks.append(A @ blocks[-1])
    K = np.hstack(blocks)
    U, sv, _ = np.linalg.svd(K, full_matrices=False)
    U = U[:, sv > 1e-13 * sv[0]]
    AU = A @ U
    out = []
    for c in range(B.shape[1]):
        y, *_ = np.linalg.lstsq(AU, B[:, c], rcond=None)
        out.append(np.linalg.norm(B[:, c] - AU @ y))
    return np.array(out)


@pytest.mark.parametrize("steps", [1, 2, 3, 4])
def test_minimal_residual_over_block_krylov_space(steps):
    rng = np.random.default_rng(11)
    n, s = 40, 3
    A = np.eye(n) * 3.0 + rng.standard_normal((n, n)) / np.sqrt(n)
    B = rng.standard_normal((n, s))
    X, it, hist = O.block_gmres(lambda Z: A @ Z, B, tol=0.0, maxit=steps)
    assert it == steps
    want = _krylov_min_residual(A, B, steps)
    got = np.linalg.norm(B - A @ X, axis=0)
    assert np.allclose(got, want, rtol=1e-9, atol=1e-12)
    # the least-squares residuals it reports are the true ones
    assert np.allclose(hist[-1], got, rtol=1e-8, atol=1e-12)


def test_one_column_is_plain_gmres():
    rng = np.random.default_rng(5)
    n = 30
    A = np.eye(n) * 2.0 + rng.standard_normal((n, n)) / np.sqrt(n)
    b = rng.standard_normal(n)
    x1, it1, h1 = O.gmres(lambda v: A @ v, b, tol=1e-12, maxit=60)
    X, it, h = O.block_gmres(lambda Z: A @ Z, b[:, None], tol=1e-12, maxit=60)
    assert it == it1
    assert np.allclose([v[0] for v in h], h1, rtol=1e-8, atol=1e-14)
    assert np.linalg.norm(X[:, 0] - x1) <= 1e-10 * np.linalg.norm(x1)


def test_terminates_at_the_dimension():
    """With s = 4 columns a 12-dimensional system is solved in 3 block steps."""
    rng = np.random.default_rng(3)
    n, s = 12, 4
    A = np.eye(n) + rng.standard_normal((n, n)) / 2
    B = rng.standard_normal((n, s))
    X, it, hist = O.block_gmres(lambda Z: A @ Z, B, tol=1e-14, maxit=10)
    assert it <= 3
    assert np.linalg.norm(A @ X - B) <= 1e-11 * np.linalg.norm(B)


def test_dependent_columns_are_deflated():
    """A column equal to a combination of earlier ones adds no basis vector, and its
    solution is the same combination of theirs."""
    rng = np.random.default_rng(8)
    n = 25
    A = np.eye(n) * 2.5 + rng.standard_normal((n, n)) / np.sqrt(n)
    b0, b1 = rng.standard_normal(n), rng.standard_normal(n)
    B = np.column_stack([b0, b1, 2.0 * b0 - 0.5 * b1])
    Q, R = O.block_orthonormalize(B, 1e-6)
    assert Q.shape[1] == 2 and R.shape == (2, 3)
    assert np.abs(Q.T @ Q - np.eye(2)).max() <= 1e-14
    assert np.linalg.norm(Q @ R - B) <= 1e-13 * np.linalg.norm(B)
    X, it, _ = O.block_gmres(lambda Z: A @ Z, B, tol=1e-12, maxit=40)
    assert np.linalg.norm(A @ X - B, axis=0).max() <= 1e-11 * np.linalg.norm(B)
    assert np.linalg.norm(X[:, 2] - (2.0 * X[:, 0] - 0.5 * X[:, 1])) <= 1e-10 * np.linalg.norm(X)


@pytest.fixture(scope="module")
def small_method():
    g = O.Grid(6, wl.uniform_breaks(4), wl.uniform_breaks(4))
    return O.Method(g)


def _rhs_block(m, s, seed):
    x, y = m.grid.node_coords()
    return np.column_stack([wl.eval_fourier(wl.random_fourier_params(seed + i, 20, 4), x, y, 1.0, 1.0)
                            for i in range(s)])


def test_block_space_beats_separate_spaces(small_method):
    """Every column's residual after j block steps is at most its residual after j
    steps of its own GMRES (its own Krylov space lies inside the block space)."""
    m = small_method
    F = _rhs_block(m, 3, 40)
    sys = m.sys
    P = m.defl.P
    S = sys.S
    Minv = lambda v: m.M.solve(v)
    op1 = lambda v: P(S @ Minv(v))
    opb = lambda Z: np.column_stack([op1(Z[:, c]) for c in range(Z.shape[1])])
    Bh = np.column_stack([P(sys.schur_rhs(F[:, c])[2]) for c in range(3)])
    _, itb, hb = O.block_gmres(opb, Bh, tol=0.0, maxit=6)
    for c in range(3):
        _, _, h1 = O.gmres(op1, Bh[:, c], tol=0.0, maxit=6)
        for j in range(1, len(h1)):
            assert hb[j][c] <= h1[j] * (1 + 1e-9) + 1e-14


@pytest.mark.parametrize("variant", [1, 2, 3])
def test_block_solve_matches_direct(small_method, variant):
    m = small_method
    F = _rhs_block(m, 4, 60)
    U, info = m.solve_block(F, variant=variant, tol=1e-12)
    for c in range(4):
        u_ref, *_ = O.solve_unreduced(m.split, F[:, c])
        assert np.linalg.norm(U[:, c] - u_ref) <= 1e-9 * np.linalg.norm(u_ref)
    assert info["true_rel_res"].max() < 1e-10
    single = [m.solve(F[:, c], variant=variant, tol=1e-12)[1]["iters"] for c in range(4)]
    assert info["iters"] <= max(single)
