"""GPU parity at full benchmark sizes against the oracle's direct solutions.

The oracle factors the bordered SMPM operator with sparse LU, which takes minutes
at these sizes, so tests/golden/make_reference_solutions.py (oracle calls only)
stored its solutions:

* the 16 x 16, n = 16 headline grid (r = 65,536; matrix-core depth KT = 16): the
  FP64 solve as the benchmark runs it and at tol 1e-12, and the mixed FP32 / BF16
  solves after refinement;
* the 32 x 32, n = 10 differentiation grid (r = 102,400; KT = 12): the forward
  solve with Neumann data and the gradient of |u - u_t|^2 through the
  differentiable solve (the adjoint solve), dLoss/df = mu and dLoss/dg = T^T mu.

Bars: FP64 relative L2 1e-10 (the benchmark's own tol 1e-10 stops on the Schur
residual, so the error it leaves is checked against a bar derived from the measured
conditioning: 1e-8), mixed precision 1e-6."""
import os

import numpy as np
import pytest

import smpm_workloads as wl
from oracle import smpm_oracle as O

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
smpm = pytest.importorskip("paper_1601_03432_amd.smpm")

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def golden(name):
    return np.load(os.path.join(GOLDEN, name), allow_pickle=False)


def dev(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


_ctx = {}


def c2():
    if "c2" not in _ctx:
        w = wl.workload("c2")
        print("[gpu-fullsize] setup c2", flush=True)
        ctx = smpm.Context.from_workload(w)
        x, y = ctx.node_coords()
        f = wl.eval_fourier(wl.random_fourier_params(wl.SEED_BASE + 2, 20, 8), x, y, w.Lx, w.Ly)
        _ctx["c2"] = (ctx, f, golden("c2_u_ref.npy"))
    return _ctx["c2"]


@pytest.mark.parametrize("tol,bar", [(1e-12, 1e-10), (1e-10, 1e-8)])
def test_c2_fp64(tol, bar):
    ctx, f, want = c2()
    u, info = ctx.solve(dev(f), tol=tol, maxit=600)
    err = rel(u.cpu().numpy()[0], want)
    print(f"[gpu-fullsize] c2 fp64 tol {tol:g}: {info.iterations} iterations, residual {info.rel_residual:.2e}, "
          f"error vs oracle {err:.2e}", flush=True)
    assert info.rel_residual <= tol
    assert err <= bar


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_c2_mixed(precision):
    ctx, f, want = c2()
    prec = smpm.MIXED_FP32 if precision == "fp32" else smpm.MIXED_BF16
    inner = 1e-5 if precision == "fp32" else 1e-3
    u, info = ctx.solve(dev(f), tol=1e-10, maxit=600, precision=prec, inner_tol=inner, max_refine=30)
    err = rel(u.cpu().numpy()[0], want)
    print(f"[gpu-fullsize] c2 mixed {precision}: {info.iterations} iterations, {info.refinements} cycles, "
          f"residual {info.rel_residual:.2e}, error vs oracle {err:.2e}", flush=True)
    assert info.rel_residual <= 1e-10
    assert err <= 1e-6


def test_c4_forward_and_gradient():
    n, m = 10, 32
    print("[gpu-fullsize] setup c4", flush=True)
    ctx = smpm.Context(m, m, n, wl.uniform_breaks(m), wl.uniform_breaks(m), O.DEFAULT_ALPHA)
    x, y = ctx.node_coords()
    f = wl.eval_fourier(wl.random_fourier_params(wl.SEED_BASE + 40, 20, 8), x, y, 1.0, 1.0)
    gb = wl.eval_edge(wl.random_edge_params(wl.SEED_BASE + 41), *ctx.boundary_arc(), 1.0, 1.0)
    ut = wl.eval_fourier(wl.random_fourier_params(wl.SEED_BASE + 42, 20, 8), x, y, 1.0, 1.0)
    u_want, mu_want = golden("c4_u_ref.npy"), golden("c4_mu_ref.npy")
    ft, gt = dev(f).requires_grad_(True), dev(gb).requires_grad_(True)
    u = smpm.solve_differentiable(ctx, ft, gt, tol=1e-12, maxit=800)
    ((u - dev(ut)) ** 2).sum().backward()
    e_u = rel(u.detach().cpu().numpy(), u_want)
    e_f = rel(ft.grad.cpu().numpy(), mu_want)
    # dLoss/dg = T^T mu with the oracle's T (a sparse product, cheap at this size)
    split_T = O.boundary_operator(O.Grid(n, wl.uniform_breaks(m), wl.uniform_breaks(m)))
    e_g = rel(gt.grad.cpu().numpy(), split_T.T @ mu_want)
    print(f"[gpu-fullsize] c4: forward error {e_u:.2e}, dL/df error {e_f:.2e}, dL/dg error {e_g:.2e}", flush=True)
    assert e_u <= 1e-10
    # the cotangent 2 (u - u_t) carries the forward error into the adjoint's input
    assert e_f <= 1e-9 and e_g <= 1e-9
