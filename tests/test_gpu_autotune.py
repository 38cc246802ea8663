"""The autotuner (smpm_autotune) picks launch shapes only: every candidate computes
each column with the same arithmetic in the same order, so solves after tuning equal
the untuned solves bit for bit, for every column-count class.  Checked on a grid with
the dense coarse solve (Schur apply with fused per-side sums, n = 16 so the matrix
cores take full 16-row tiles) and on one with the substructured coarse solve forced
(plain Schur apply, where the persistent kernel is a candidate)."""
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


def _context(m, n, substructured):
    old = {k: os.environ.get(k) for k in ("SMPM_DENSE_COARSE_MAX", "SMPM_COARSE_PATCH")}
    if substructured:
        os.environ["SMPM_DENSE_COARSE_MAX"] = "0"
        os.environ["SMPM_COARSE_PATCH"] = "4"
    try:
        return smpm.Context(m, m, n, wl.uniform_breaks(m), wl.uniform_breaks(m), O.DEFAULT_ALPHA, device=True)
    finally:
        for k, v in old.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v


def _rhs(ctx, seed, ncol):
    x, y = ctx.node_coords()
    F = np.stack([wl.eval_fourier(wl.random_fourier_params(seed + i, 20, 4), x, y, 1.0, 1.0) for i in range(ncol)])
    return torch.tensor(F, dtype=torch.float64, device="cuda")


@pytest.mark.parametrize("grid", ["dense_12x12_n16", "substructured_16x16_n8"])
def test_tuned_solves_equal_untuned(grid):
    m, n, sub = (12, 16, False) if grid.startswith("dense") else (16, 8, True)
    print(f"[gpu-autotune] {grid}", flush=True)
    ctx = _context(m, n, sub)
    kw = dict(tol=1e-11, maxit=600)
    cases = {}
    for ncol in (1, 3, 8):
        F = _rhs(ctx, 300 + 10 * ncol, ncol)
        ref, info = ctx.solve(F, **kw)
        mixed, info_m = ctx.solve(F, precision=smpm.MIXED_FP32, **kw)
        cases[ncol] = (F, ref, info.iterations, mixed, info_m.iterations)
    for ncol in (1, 3, 8):
        choice = ctx.autotune(ncol)
        print(f"[gpu-autotune] {grid} {ncol} columns: {choice}", flush=True)
        assert choice["nrhs"] == ncol
        assert choice["schur_us"] > 0 and choice["step_us"] > 0
        assert choice["prereduce"] in (0, 1)
        assert choice["schur_columns_per_workgroup"] in (1, 2, 4)
    for ncol, (F, ref, it, mixed, it_m) in cases.items():
        u, info = ctx.solve(F, **kw)
        assert torch.equal(u, ref), (grid, ncol)
        assert info.iterations == it
        um, info_m = ctx.solve(F, precision=smpm.MIXED_FP32, **kw)
        assert torch.equal(um, mixed), (grid, ncol)
        assert info_m.iterations == it_m


def test_autotune_rejects_bad_column_count():
    ctx = _context(4, 6, False)
    with pytest.raises(smpm.SmpmError):
        ctx.autotune(0)


@pytest.mark.parametrize("shape", [
    (("SMPM_SCHUR_PERSIST", "1"),),
    (("SMPM_SCHUR_PERSIST", "2"), ("SMPM_SCHUR_NC", "1")),
    (("SMPM_SCHUR_PERSIST", "2"), ("SMPM_SCHUR_NC", "2")),
    (("SMPM_SCHUR_PERSIST", "3"), ("SMPM_SCHUR_CPW", "4")),
    (("SMPM_SCHUR_PERSIST", "3"), ("SMPM_SCHUR_CPW", "8")),
    (("SMPM_PREREDUCE", "1"),),
    (("SMPM_PREREDUCE", "0"),),
], ids=["persistent", "ws_nc1", "ws_nc2", "cols_cpw4", "cols_cpw8", "prereduce1", "prereduce0"])
def test_launch_shapes_give_identical_solves(shape, monkeypatch):
    """Every Schur launch shape and either reduction of the Gram-Schmidt sums gives the
    solutions of the default choice bit for bit (8 columns, substructured coarse
    solve, the shape the autotuner may pick)."""
    base = _context(16, 8, True)
    F = _rhs(base, 700, 8)
    kw = dict(tol=1e-11, maxit=600)
    ref, info = base.solve(F, **kw)
    for name, val in shape:
        monkeypatch.setenv(name, val)
    ctx = _context(16, 8, True)
    u, info2 = ctx.solve(F, **kw)
    diff = (u - ref).abs().max().item()
    print(f"[gpu-autotune] {shape}: max |diff| {diff:.3e}, iterations {info2.iterations} vs {info.iterations}")
    assert torch.equal(u, ref), (shape, diff)
