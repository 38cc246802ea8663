"""GPU parity of the adjoint solve (transposed Algorithm 3) and of the autograd
wrapper against the oracle's dense adjoint, plus central differences of the GPU
forward solve.

Tolerances: the adjoint solves run to tol 1e-12 and must match the oracle to the
FP64 bar (relative L2 <= 1e-10); mixed precision to 1e-6.  Central differences of
the quadratic loss |u - u_t|^2 have no truncation error; with step h the
difference quotient carries the forward solves' error e_u as about
|u - u_t| |e_u| / h, so the bar is set per step size (h = 1e-6 and h = 1e-3)."""
import numpy as np
import pytest

import smpm_workloads as wl
from oracle import smpm_oracle as O

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
smpm = pytest.importorskip("paper_1601_03432_amd.smpm")

GRIDS = {
    "c1": (8, wl.uniform_breaks(4), wl.uniform_breaks(4)),
    "nonsquare_5x3": (6, wl.uniform_breaks(5, 2.0), wl.uniform_breaks(3, 1.0)),
    "stretched_4x3": (7, np.array([0.0, 0.1, 0.25, 0.5, 1.0]), np.array([0.0, 0.3, 0.6, 1.0])),
    "ragged_9x7": (5, wl.uniform_breaks(9), wl.uniform_breaks(7)),
    "two_2x1": (5, wl.uniform_breaks(2), wl.uniform_breaks(1)),
}
_cache = {}
# central differences of the quadratic loss at tol 1e-12: the difference quotient
# carries ~|u - u_t| * tol * |u| / h of solve error (no truncation error)
TOL_FD_H6 = 1e-3
TOL_FD_H3 = 1e-6


def setup(name):
    if name not in _cache:
        n, xb, yb = GRIDS[name]
        print(f"[gpu-adjoint] setup {name}", flush=True)
        ctx = smpm.Context(len(yb) - 1, len(xb) - 1, n, xb, yb, O.DEFAULT_ALPHA, device=True)
        _cache[name] = (ctx, O.Split(O.Grid(n, xb, yb)))
    return _cache[name]


def dev(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.mark.parametrize("name", sorted(GRIDS))
def test_adjoint_solve_matches_oracle(name):
    ctx, split = setup(name)
    Cs = wl.random_vectors(81, 2, ctx.r)
    mu, info = ctx.solve(dev(Cs), tol=1e-12, maxit=600, transpose=True)
    mu = mu.cpu().numpy()
    print(f"[gpu-adjoint] {name}: {info.iterations} iterations, true residual {info.rel_residual:.2e}")
    for c in range(2):
        want = O.solve_adjoint_unreduced(split, Cs[c])[0]
        assert rel(mu[c], want) <= 1e-10, (name, c, rel(mu[c], want))
    assert info.rel_residual <= 1e-11


@pytest.mark.parametrize("name", ["c1", "stretched_4x3", "ragged_9x7"])
def test_boundary_transpose(name):
    ctx, split = setup(name)
    M = wl.random_vectors(82, 3, ctx.r)
    got = ctx.boundary_transpose(dev(M)).cpu().numpy()
    for c in range(3):
        assert rel(got[c], O.boundary_adjoint(split, M[c])) <= 1e-14


@pytest.mark.parametrize("name", ["c1", "stretched_4x3"])
def test_adjoint_mixed_precision(name):
    ctx, split = setup(name)
    c = wl.random_vectors(83, 1, ctx.r)
    mu, info = ctx.solve(dev(c), tol=1e-10, maxit=600, transpose=True, precision=smpm.MIXED_FP32,
                         inner_tol=1e-6, max_refine=30)
    want = O.solve_adjoint_unreduced(split, c[0])[0]
    assert info.rel_residual <= 1e-10
    assert rel(mu.cpu().numpy()[0], want) <= 1e-6


def _loss_problem(g, seed):
    x, y = g.node_coords()
    Lx, Ly = g.xb[-1] - g.xb[0], g.yb[-1] - g.yb[0]
    f = wl.eval_fourier(wl.random_fourier_params(seed, 20, 4), x, y, Lx, Ly)
    gb = wl.eval_edge(wl.random_edge_params(seed + 1), *g.boundary_arc(), Lx, Ly)
    ut = wl.eval_fourier(wl.random_fourier_params(seed + 2, 20, 4), x, y, Lx, Ly)
    return f, gb, ut


@pytest.mark.parametrize("name", ["c1", "stretched_4x3", "two_2x1"])
def test_autograd_matches_oracle_gradient(name):
    """Loss = |u(f, g) - u_t|^2 through the differentiable solve: dLoss/df and dLoss/dg
    from autograd equal the oracle's mu and T^T mu for c = 2 (u - u_t)."""
    ctx, split = setup(name)
    f, gb, ut = _loss_problem(split.grid, 84)
    ft = dev(f).requires_grad_(True)
    gt = dev(gb).requires_grad_(True)
    u = smpm.solve_differentiable(ctx, ft, gt, tol=1e-12, maxit=600)
    loss = ((u - dev(ut)) ** 2).sum()
    loss.backward()
    u_or = O.solve_unreduced(split, f, gb)[0]
    mu = O.solve_adjoint_unreduced(split, 2.0 * (u_or - ut))[0]
    assert rel(ft.grad.cpu().numpy(), mu) <= 1e-9
    assert rel(gt.grad.cpu().numpy(), O.boundary_adjoint(split, mu)) <= 1e-9


def test_central_differences_32x32_n10():
    """The differentiation workload: 32 x 32 elements, n = 10 on [0,1]^2, FP64; 50
    seeded unit directions in (f, g), h = 1e-6, against the adjoint gradient."""
    n, m = 10, 32
    ctx = smpm.Context(m, m, n, wl.uniform_breaks(m), wl.uniform_breaks(m), O.DEFAULT_ALPHA)
    x, y = ctx.node_coords()
    f = wl.eval_fourier(wl.random_fourier_params(wl.SEED_BASE + 40, 20, 8), x, y, 1.0, 1.0)
    gb = wl.eval_edge(wl.random_edge_params(wl.SEED_BASE + 41), *ctx.boundary_arc(), 1.0, 1.0)
    ut = wl.eval_fourier(wl.random_fourier_params(wl.SEED_BASE + 42, 20, 8), x, y, 1.0, 1.0)
    utd = dev(ut)
    opts = dict(tol=1e-12, maxit=800)
    ft, gt = dev(f).requires_grad_(True), dev(gb).requires_grad_(True)
    u = smpm.solve_differentiable(ctx, ft, gt, **opts)
    ((u - utd) ** 2).sum().backward()
    nd = 50
    Df = dev(wl.random_directions(wl.SEED_BASE + 43, nd, ctx.r))
    Dg = dev(wl.random_directions(wl.SEED_BASE + 44, nd, ctx.nbdry))
    ad = ((Df * ft.grad).sum(dim=1) + (Dg * gt.grad).sum(dim=1)).cpu().numpy()
    errs = {}
    for h in (1e-6, 1e-3):
        # all 2*nd perturbed problems as one batched solve
        F = torch.cat([dev(f) + h * Df, dev(f) - h * Df])
        G = torch.cat([dev(gb) + h * Dg, dev(gb) - h * Dg])
        U, _ = ctx.solve(F, G, **opts)
        L = ((U - utd) ** 2).sum(dim=1)
        fd = ((L[:nd] - L[nd:]) / (2 * h)).cpu().numpy()
        errs[h] = np.abs(fd - ad).max() / np.abs(ad).max()
        print(f"[gpu-adjoint] 32x32 n=10, h={h:g}: max |FD - AD| / max|AD| = {errs[h]:.2e} "
              f"over {nd} directions", flush=True)
    assert errs[1e-6] <= TOL_FD_H6
    assert errs[1e-3] <= TOL_FD_H3
