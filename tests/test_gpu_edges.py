"""Edge cases and error paths of the device solve, through the C ABI: a column that
exhausts maxit, a zero right-hand side inside a batch, invalid options, the maxit
limit, non-convergence reported by a group solve, run-to-run determinism, and the
cache policy of the basis loads leaving the bits unchanged."""
import os

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


_ctx = {}


def ctx_c1():
    if "c1" not in _ctx:
        _ctx["c1"] = smpm.Context(4, 4, 8, wl.uniform_breaks(4), wl.uniform_breaks(4), O.DEFAULT_ALPHA)
    return _ctx["c1"]


def source(ctx, seed, ncol):
    x, y = ctx.node_coords()
    F = np.stack([wl.eval_fourier(wl.random_fourier_params(seed + i, 20, 4), x, y, 1.0, 1.0) for i in range(ncol)])
    return torch.tensor(F, dtype=torch.float64, device="cuda")


def test_maxit_exhausted_reports_no_convergence():
    ctx = ctx_c1()
    F = source(ctx, 900, 2)
    with pytest.raises(smpm.SmpmError):
        ctx.solve(F, tol=1e-12, maxit=3)
    u, info = ctx.solve(F, tol=1e-12, maxit=3, raise_on_noconv=False)
    assert info.status == smpm.ENOCONV
    assert info.iterations == 3
    assert info.rel_residual > 1e-12
    assert torch.isfinite(u).all()
    # the same problem converges with room to iterate
    _, ok = ctx.solve(F, tol=1e-12, maxit=600)
    assert ok.status == smpm.OK and ok.iterations > 3


def test_zero_column_in_batch():
    """A zero right-hand side retires at once with u = 0; its neighbour in the batch
    is unaffected (bit-identical to its single solve)."""
    ctx = ctx_c1()
    F = source(ctx, 910, 1)
    B = torch.cat([torch.zeros_like(F), F])
    u, info = ctx.solve(B, tol=1e-12, maxit=600)
    assert torch.count_nonzero(u[0]) == 0
    single, _ = ctx.solve(F, tol=1e-12, maxit=600)
    assert torch.allclose(u[1], single[0], rtol=0, atol=1e-13 * float(single.abs().max()))
    assert info.rel_residual <= 1e-12


@pytest.mark.parametrize("bad", [dict(maxit=0), dict(maxit=1001), dict(tol=0.0), dict(tol=-1.0), dict(variant=4),
                                 dict(precision=7), dict(precision=smpm.MIXED_FP32, inner_tol=1.5),
                                 dict(precision=smpm.MIXED_FP32, max_refine=0)])
def test_invalid_options_rejected(bad):
    ctx = ctx_c1()
    kw = dict(tol=1e-10, maxit=100)
    kw.update(bad)
    with pytest.raises(smpm.SmpmError):
        ctx.solve(source(ctx, 920, 1), **kw)


def test_maxit_limit_accepted():
    ctx = ctx_c1()
    _, info = ctx.solve(source(ctx, 930, 1), tol=1e-12, maxit=1000)
    assert info.status == smpm.OK


def test_group_reports_no_convergence():
    a = ctx_c1()
    b = smpm.Context(3, 5, 6, wl.uniform_breaks(5), wl.uniform_breaks(3), O.DEFAULT_ALPHA)
    fa, fb = source(a, 940, 1), source(b, 950, 1)
    with pytest.raises(smpm.SmpmError):
        smpm.solve_group([a, b], [fa, fb], tol=1e-12, maxit=2)
    out = smpm.solve_group([a, b], [fa, fb], tol=1e-12, maxit=2, raise_on_noconv=False)
    assert all(i.status == smpm.ENOCONV for _, i in out)


@pytest.mark.parametrize("precision", ["fp64", "mixed_fp32"])
def test_repeated_solves_are_bit_identical(precision):
    ctx = ctx_c1()
    F = source(ctx, 960, 3)
    kw = dict(tol=1e-11, maxit=600)
    if precision != "fp64":
        kw["precision"] = smpm.MIXED_FP32
    ref, _ = ctx.solve(F, **kw)
    for _ in range(3):
        u, _ = ctx.solve(F, **kw)
        assert torch.equal(u, ref)


def _with_env(env, fn):
    old = {k: os.environ.get(k) for k in env}
    os.environ.update(env)
    try:
        return fn()
    finally:
        for k, v in old.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v


@pytest.mark.parametrize("ncol,prereduce", [(1, "0"), (4, "1")])
def test_streaming_basis_loads_keep_the_bits(ncol, prereduce):
    """Non-temporal basis loads (forced on a small grid, where the library would use
    ordinary ones) change only the cache policy: the solution and the iteration count
    are bit-identical (one column through the single-column update; four columns
    through the multi-column update with pre-reduced sums)."""
    print(f"[gpu-edges] streaming basis loads, {ncol} columns", flush=True)
    ctx = ctx_c1()
    F = source(ctx, 940, ncol)
    kw = dict(tol=1e-12, maxit=600)
    ref, info = _with_env({"SMPM_STREAM_BASIS": "0", "SMPM_PREREDUCE": prereduce}, lambda: ctx.solve(F, **kw))
    u, info_s = _with_env({"SMPM_STREAM_BASIS": "1", "SMPM_PREREDUCE": prereduce}, lambda: ctx.solve(F, **kw))
    assert torch.equal(u, ref)
    assert info_s.iterations == info.iterations
