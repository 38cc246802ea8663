"""The paper's own experiments on the GPU path (Sec. 3.1 error; Sec. 3.2
h-refinement: n = 5, m = 4..32; Sec. 3.3 p-refinement: m = 4, p = 4..14), for
Algorithm 1 (no preconditioner), 2 (block-Jacobi) and 3 (block-Jacobi + deflation)
with the lambda = 7 cosine source and zero Neumann data, tolerance 1e-10.

The three algorithms solve the same system, so their solutions must agree; the
iteration counts must show the trends the paper reports (deflation no worse than
the unpreconditioned method as h shrinks, preconditioned counts nearly
independent of p; thresholds in tests/golden/paper_iteration_counts.json).
Algorithm 3 is also run under the paper's stopping rule (relative to the initial
GMRES residual |P b_hat|).  The discretization error against the analytic solution
falls with h and spectrally with p, and equals the oracle's error for the same
grids (the solutions agree to the FP64 bar).  The paper's penalty value is
unknown, so its printed counts are context only."""
import json
import os

import numpy as np
import pytest

import smpm_workloads as wl
from oracle import smpm_oracle as O

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
smpm = pytest.importorskip("paper_1601_03432_amd.smpm")

H_GRIDS = (4, 8, 12, 16, 20, 24, 28, 32)
P_ORDERS = (4, 6, 8, 10, 12, 14)


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _l2(w, a):
    a = a - (w @ a) / w.sum()
    return float(np.sqrt(w @ (a * a)))


def _run(m, n):
    ctx = smpm.Context(m, m, n, wl.uniform_breaks(m), wl.uniform_breaks(m), O.DEFAULT_ALPHA)
    x, y = ctx.node_coords()
    ua, f = wl.manufactured_cos(x, y, lam=7)
    fd = torch.tensor(f, dtype=torch.float64, device="cuda").reshape(1, -1)
    out, sols = [], []
    for variant in (1, 2, 3):
        u, info = ctx.solve(fd, tol=1e-10, maxit=1000, variant=variant)
        assert info.rel_residual <= 1e-10, (m, n, variant, info.rel_residual)
        out.append(info.iterations)
        sols.append(u.cpu().numpy()[0])
    for s in sols[:2]:
        assert np.linalg.norm(s - sols[2]) <= 1e-7 * np.linalg.norm(sols[2]), (m, n)
    up, info_p = ctx.solve(fd, tol=1e-10, maxit=1000, variant=3, stop_rule=1)
    assert info_p.rel_residual <= 1e-10
    # the paper's rule: the first GMRES run stops at 1e-10 |P b_hat|; where |P b_hat| >
    # |b_hat| the FP64 true residual then misses 1e-10 |b_hat| and a correction cycle
    # follows, whose history (relative to its own initial residual) is the one reported
    out.append(info_p.cycle_iterations[0])
    hs = info_p.history
    assert hs[0] == pytest.approx(1.0) and all(b <= a * (1 + 1e-12) for a, b in zip(hs, hs[1:])), hs[:5]
    if info_p.refinements == 1:
        assert hs[-1] <= 1e-10 * (1 + 1e-12)
    w = ctx.quadrature_weights()
    err = _l2(w, sols[2] - ua) / _l2(w, ua)
    return out, err, sols[2]


def test_h_and_p_refinement_trends(golden_dir):
    crit = json.load(open(os.path.join(golden_dir, "paper_iteration_counts.json")))["test_criteria"]
    h = {m: _run(m, 5) for m in H_GRIDS}
    p = {q: _run(4, q + 1) for q in P_ORDERS}
    for m, (c, e, _) in h.items():
        print(f"[gpu-paper] n=5 m={m}: Alg1 {c[0]}, Alg2 {c[1]}, Alg3 {c[2]} (paper rule {c[3]}), "
              f"error {e:.2e}", flush=True)
    for q, (c, e, _) in p.items():
        print(f"[gpu-paper] m=4 p={q}: Alg1 {c[0]}, Alg2 {c[1]}, Alg3 {c[2]} (paper rule {c[3]}), "
              f"error {e:.2e}", flush=True)
    # Sec. 3.2: deflation is not worse than no preconditioner from m = 12 on, and the
    # unpreconditioned count grows with m
    for m in H_GRIDS[2:]:
        assert h[m][0][2] <= h[m][0][0], (m, h[m][0])
    assert h[32][0][0] > h[4][0][0]
    # Sec. 3.3: the preconditioned counts are nearly independent of p
    for v in (1, 2):
        vals = [p[q][0][v] for q in P_ORDERS]
        assert max(vals) <= crit["p_independence_ratio_max"] * min(vals), (v, vals)
    # Sec. 3.1: the error falls with h (halving h from m = 16 to 32 and from 8 to 16
    # gains more than 10x: order above 3.3 at N = 4, measured ~4) and spectrally with
    # p until the rounding plateau
    eh = [h[m][1] for m in H_GRIDS]
    assert eh[-1] < eh[3] / 10 and eh[3] < eh[1] / 10, eh
    ep = [p[q][1] for q in P_ORDERS]
    for a, b in zip(ep[:3], ep[1:4]):
        assert b < a / 20, ep
    assert ep[-1] < 1e-8, ep


@pytest.mark.parametrize("m,n", [(4, 5), (8, 5), (12, 5), (4, 9), (4, 15)])
def test_error_matches_oracle(m, n):
    """The GPU solution of the lambda = 7 problem (tol 1e-12) equals the oracle's direct
    solution to the FP64 bar, and so does its error against the analytic solution: the
    error study measures the discretization, not the solver."""
    ctx = smpm.Context(m, m, n, wl.uniform_breaks(m), wl.uniform_breaks(m), O.DEFAULT_ALPHA)
    x, y = ctx.node_coords()
    ua, f = wl.manufactured_cos(x, y, lam=7)
    u, _ = ctx.solve(torch.tensor(f, dtype=torch.float64, device="cuda").reshape(1, -1), tol=1e-12, maxit=1000)
    u = u.cpu().numpy()[0]
    g = O.Grid(n, wl.uniform_breaks(m), wl.uniform_breaks(m))
    u_or = O.solve_unreduced(O.Split(g), f)[0]
    assert np.linalg.norm(u - u_or) <= 1e-10 * np.linalg.norm(u_or)
    w = g.quad_weights()
    err, err_or = _l2(w, u - ua) / _l2(w, ua), _l2(w, u_or - ua) / _l2(w, ua)
    assert err == pytest.approx(err_or, rel=1e-6, abs=1e-12), (err, err_or)
