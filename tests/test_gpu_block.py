"""Block GMRES on the GPU (step 4 of Algorithm 3 for all right-hand sides in one block
Krylov space) against the oracle's block GMRES: block step counts, the per-step
least-squares residuals of column 0, and the solutions, for Algorithms 1-3, at
order 6 and at order 16 (the full-width matrix-core tiles), with dependent columns
(rank deflation), one column, 32 advected sources (nearly dependent columns, the
batched workload's shape at a smaller grid), the adjoint, block GMRES as the inner
solve of mixed-precision refinement, and the error paths."""
import numpy as np
import pytest

import smpm_workloads as wl
from oracle import smpm_oracle as O

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
smpm = pytest.importorskip("paper_1601_03432_amd.smpm")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


_cache = {}


def _pair(m, n):
    key = (m, n)
    if key not in _cache:
        g = O.Grid(n, wl.uniform_breaks(m), wl.uniform_breaks(m))
        ctx = smpm.Context(m, m, n, wl.uniform_breaks(m), wl.uniform_breaks(m), O.DEFAULT_ALPHA, device=True)
        _cache[key] = (O.Method(g), ctx)
    return _cache[key]


def _sources(meth, s, seed):
    x, y = meth.grid.node_coords()
    return np.column_stack([wl.eval_fourier(wl.random_fourier_params(seed + i, 20, 4), x, y, 1.0, 1.0)
                            for i in range(s)])


def _gpu_solve(ctx, F, **kw):
    Ft = torch.tensor(np.ascontiguousarray(F.T), dtype=torch.float64, device="cuda")
    U, info = ctx.solve(Ft, block=True, **kw)
    return U.cpu().numpy().T, info


def _check_against_oracle(meth, ctx, F, variant, tol):
    print(f"[gpu-block] m={meth.grid.m_x} n={meth.grid.n} cols={F.shape[1]} variant={variant}", flush=True)
    Uo, io = meth.solve_block(F, variant=variant, tol=tol)
    Ug, ig = _gpu_solve(ctx, F, tol=tol, variant=variant, maxit=200)
    assert ig.refinements == 1, ig
    assert abs(ig.iterations - io["iters"]) <= 1, (ig.iterations, io["iters"])
    # column 0's least-squares residual per block step, relative to |b_hat_0|
    ref0 = np.linalg.norm(io["Bhat"][:, 0])
    ho = [h[0] / ref0 for h in io["history"]]
    hg = list(ig.history)
    for j in range(min(len(ho), len(hg))):
        if ho[j] > 1e-8:
            assert abs(hg[j] - ho[j]) <= 1e-6 * ho[j], (j, hg[j], ho[j])
    for c in range(F.shape[1]):
        err = np.linalg.norm(Ug[:, c] - Uo[:, c]) / max(np.linalg.norm(Uo[:, c]), 1e-300)
        assert err <= 1e-9, (c, err)
    assert ig.rel_residual <= tol


@pytest.mark.parametrize("variant", [1, 2, 3])
def test_block_matches_oracle_order6(variant):
    meth, ctx = _pair(4, 6)
    _check_against_oracle(meth, ctx, _sources(meth, 4, 60), variant, 1e-10)


def test_block_matches_oracle_order16():
    meth, ctx = _pair(4, 16)
    _check_against_oracle(meth, ctx, _sources(meth, 8, 80), 3, 1e-10)


def test_dependent_columns():
    """Columns 2 and 3 are combinations of columns 0 and 1: the start block keeps two
    vectors, and the solutions are the same combinations."""
    meth, ctx = _pair(4, 6)
    F = _sources(meth, 2, 90)
    F = np.column_stack([F[:, 0], F[:, 1], 2.0 * F[:, 0] - 0.5 * F[:, 1], F[:, 1]])
    _check_against_oracle(meth, ctx, F, 3, 1e-10)
    U, _ = _gpu_solve(ctx, F, tol=1e-10)
    assert np.linalg.norm(U[:, 2] - (2.0 * U[:, 0] - 0.5 * U[:, 1])) <= 1e-9 * np.linalg.norm(U[:, 2])
    assert np.linalg.norm(U[:, 3] - U[:, 1]) <= 1e-9 * np.linalg.norm(U[:, 1])


def test_one_column_equals_plain_solve():
    meth, ctx = _pair(4, 6)
    F = _sources(meth, 1, 95)
    Ub, ib = _gpu_solve(ctx, F, tol=1e-11)
    Ft = torch.tensor(F.T.copy(), dtype=torch.float64, device="cuda")
    Up, ip = ctx.solve(Ft, tol=1e-11)
    Up = Up.cpu().numpy().T
    assert abs(ib.iterations - ip.iterations) <= 1
    assert np.linalg.norm(Ub - Up) <= 1e-9 * np.linalg.norm(Up)


def test_advected_sources_32_columns():
    """32 advected sources plus noise (the batched workload's recipe) on a 16 x 16 grid
    of order 8: a basis of several hundred vectors, many chunks of the dot kernel."""
    meth, ctx = _pair(16, 8)
    x, y = meth.grid.node_coords()
    F = np.asarray(wl.advected_sources(wl.SEED_BASE + 3, x, y, count=32))
    F = F if F.shape[0] == x.size else F.T
    _check_against_oracle(meth, ctx, F, 3, 1e-10)


def test_adjoint_block_equals_batched():
    meth, ctx = _pair(4, 6)
    F = _sources(meth, 3, 120)
    Ft = torch.tensor(F.T.copy(), dtype=torch.float64, device="cuda")
    Ub, _ = ctx.solve(Ft, tol=1e-11, transpose=True, block=True)
    Up, _ = ctx.solve(Ft, tol=1e-11, transpose=True)
    assert (Ub - Up).norm().item() <= 1e-9 * Up.norm().item()
    # the adjoint with block GMRES as the inner solve of FP32 refinement
    Um, im = ctx.solve(Ft, tol=1e-10, transpose=True, block=True, precision=smpm.MIXED_FP32)
    assert im.rel_residual <= 1e-10
    assert (Um - Up).norm().item() <= 1e-6 * Up.norm().item()


@pytest.mark.parametrize("precision", ["MIXED_FP32", "MIXED_BF16"])
def test_mixed_precision_block(precision):
    """Block GMRES as the inner solve of the refinement cycles (FP32 / BF16 operators):
    within 1e-6 of the oracle's block solution, FP64 true residual <= 1e-10."""
    meth, ctx = _pair(16, 8)
    F = _sources(meth, 8, 140)
    print(f"[gpu-block] mixed {precision} m=16 n=8 cols=8", flush=True)
    Uo, io = meth.solve_block(F, tol=1e-11)
    Ug, ig = _gpu_solve(ctx, F, tol=1e-10, maxit=200, precision=getattr(smpm, precision), inner_tol=1e-5,
                        max_refine=30)
    assert ig.rel_residual <= 1e-10
    for c in range(F.shape[1]):
        assert np.linalg.norm(Ug[:, c] - Uo[:, c]) <= 1e-6 * np.linalg.norm(Uo[:, c]), c


def test_zero_columns():
    """A zero column inside the block adds no vector and returns u = 0; an all-zero
    right-hand side returns u = 0 without a block step."""
    meth, ctx = _pair(4, 6)
    F = _sources(meth, 3, 150)
    F[:, 1] = 0.0
    _check_against_oracle(meth, ctx, F, 3, 1e-10)
    U, _ = _gpu_solve(ctx, F, tol=1e-10)
    assert np.abs(U[:, 1]).max() == 0.0
    U0, i0 = _gpu_solve(ctx, np.zeros_like(F), tol=1e-10)
    assert np.abs(U0).max() == 0.0 and i0.iterations == 0


def test_non_finite_input_is_rejected():
    meth, ctx = _pair(4, 6)
    F = _sources(meth, 2, 160)
    F[5, 1] = np.nan
    with pytest.raises(smpm.SmpmError):
        _gpu_solve(ctx, F, tol=1e-10)
    # the context stays usable
    U, info = _gpu_solve(ctx, _sources(meth, 2, 170), tol=1e-10)
    assert info.rel_residual <= 1e-10


def test_block_error_paths():
    meth, ctx = _pair(4, 6)
    F = torch.tensor(_sources(meth, 2, 130).T.copy(), dtype=torch.float64, device="cuda")
    F33 = F[:1].repeat(33, 1).contiguous()
    with pytest.raises(smpm.SmpmError):
        ctx.solve(F33, block=True)
