"""Failure paths of the solve that must not report success: non-finite input data
returns SMPM_EINVAL (forward, mixed precision, one bad column of a batch, adjoint,
non-finite Neumann data), the context stays usable afterwards, and the null-vector
solve reports the residual it reached (||S^T u_S|| / ||S|| <= 1e-12, checked
independently through the transposed Schur apply)."""
import numpy as np
import pytest

import smpm_workloads as wl
from oracle import smpm_oracle as O

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
smpm = pytest.importorskip("paper_1601_03432_amd.smpm")

_cache = {}


def ctx_c1():
    if "c1" not in _cache:
        w = wl.workload("c1")
        _cache["c1"] = smpm.Context.from_workload(w)
    return _cache["c1"]


def dev(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _source(ctx, cols):
    return wl.random_vectors(301, cols, ctx.r)


@pytest.mark.parametrize("bad", [np.nan, np.inf, -np.inf])
@pytest.mark.parametrize("form", ["fp64", "mixed_fp32", "mixed_bf16", "adjoint"])
def test_nonfinite_source_is_rejected(bad, form):
    ctx = ctx_c1()
    F = _source(ctx, 3)
    F[1, 17] = bad  # one bad entry in the middle column of a batch
    kw = dict(tol=1e-10, maxit=400)
    if form == "mixed_fp32":
        kw.update(precision=smpm.MIXED_FP32)
    elif form == "mixed_bf16":
        kw.update(precision=smpm.MIXED_BF16, inner_tol=1e-3)
    elif form == "adjoint":
        kw.update(transpose=True)
    with pytest.raises(smpm.SmpmError) as ei:
        ctx.solve(dev(F), **kw)
    assert ei.value.code == smpm.EINVAL, str(ei.value)
    assert "non-finite" in str(ei.value)
    # the context still solves a good problem
    u, info = ctx.solve(dev(_source(ctx, 1)), tol=1e-10)
    assert info.status == smpm.OK and info.rel_residual <= 1e-10
    assert torch.isfinite(u).all()


def test_nonfinite_boundary_data_is_rejected():
    ctx = ctx_c1()
    F = _source(ctx, 2)
    G = wl.random_vectors(302, 2, ctx.nbdry)
    G[0, 5] = np.nan
    with pytest.raises(smpm.SmpmError) as ei:
        ctx.solve(dev(F), dev(G), tol=1e-10)
    assert ei.value.code == smpm.EINVAL


def test_fp64_solve_reports_its_true_residual():
    """An FP64 solve that returns OK has an FP64 true Schur residual at or below tol."""
    ctx = ctx_c1()
    for tol in (1e-8, 1e-10, 1e-12):
        _, info = ctx.solve(dev(_source(ctx, 2)), tol=tol)
        assert info.status == smpm.OK and info.rel_residual <= tol, (tol, info)


@pytest.mark.parametrize("name", ["c1", "c2", "c4"])
def test_null_vector_residual(name):
    """smpm_stats reports ||S^T u_S|| / ||S|| of the computed left null vector; the
    transposed Schur apply of u_S gives the same bound independently."""
    w = wl.workload(name)
    ctx = smpm.Context.from_workload(w)
    uL, uS = ctx.null_vectors()
    st = ctx.stats()
    print(f"[gpu-failures] {name}: null residual {st['null_residual']:.2e} after "
          f"{st['null_iterations']} iterations, ||S|| <= {st['schur_norm_bound']:.3g}", flush=True)
    assert 0 <= st["null_residual"] <= 1e-12
    sty = ctx.schur_apply(dev(uS), transpose=True).cpu().numpy()[0]
    assert np.linalg.norm(sty) <= 1e-12 * st["schur_norm_bound"]
    assert abs(np.linalg.norm(uS) - 1.0) < 1e-12 and abs(np.linalg.norm(uL) - 1.0) < 1e-12
