"""GPU parity against the oracle at every polynomial order the library instantiates
separately, through the C ABI.

The Schur apply runs on matrix cores with a contraction depth KT = 4 ceil(4n/16):
KT = 4 for n <= 4, 12 for n = 9..12 (the 64x64 n = 12 and 32x32 n = 10 workloads),
16 for n = 13..16 (the 16x16 n = 16 headline grid and the 128x128 n = 16 stretched
grid); orders 17..32 take the vector kernels.  Each order is checked on a ragged
5 x 3 element grid (tiles of one element class hold 1 to 3 elements) and on a
stretched 4 x 3 grid (aspect up to 4, nonsingular coarse matrix): the Schur apply
forward and transposed in FP64, FP32 and BF16, with 1, 2 and 4 columns per
workgroup, the persistent kernel, the warp-specialized persistent kernel and the
column-pipelined kernel, the block-Jacobi preconditioner (blocks of up to 8n slots), the null vectors, the projections and full solves.

Bars: single FP64 operator applies 1e-12 (two independent FP64 setups, measured
~1e-13); FP32 / BF16 operators 1e-5 / 2e-2 (operand rounding 2^-24 / 2^-8 over at
most 4n = 64 terms of the B A^{-1} E part); FP64 solves 1e-10 (tol 1e-12); mixed
precision 1e-6 after refinement with FP64 true residual <= 1e-10."""
import numpy as np
import pytest

import smpm_workloads as wl
from oracle import smpm_oracle as O

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
smpm = pytest.importorskip("paper_1601_03432_amd.smpm")

ORDERS = (4, 10, 12, 16, 20)
GEOMS = {
    "ragged_5x3": (wl.uniform_breaks(5, 1.5), wl.uniform_breaks(3, 1.0)),
    "stretched_4x3": (np.array([0.0, 0.1, 0.25, 0.5, 1.0]), np.array([0.0, 0.3, 0.6, 1.0])),
}
_ctx = {}
_orc = {}


def oracle(geom, n):
    key = (geom, n)
    if key not in _orc:
        xb, yb = GEOMS[geom]
        _orc[key] = O.Method(O.Grid(n, xb, yb))
    return _orc[key]


def context(geom, n, env=(), monkeypatch=None):
    """A context built with the launch-shape overrides in env (read at setup)."""
    key = (geom, n, env)
    if key not in _ctx:
        xb, yb = GEOMS[geom]
        for name, val in env:
            monkeypatch.setenv(name, val)
        print(f"[gpu-orders] setup {geom} n={n} {dict(env)}", flush=True)
        _ctx[key] = smpm.Context(len(yb) - 1, len(xb) - 1, n, xb, yb, O.DEFAULT_ALPHA, device=True)
        for name, _ in env:
            monkeypatch.delenv(name)
    return _ctx[key]


def dev(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


SHAPES = {
    "nc1": (("SMPM_SCHUR_NC", "1"), ("SMPM_SCHUR_PERSIST", "-1")),
    "nc2": (("SMPM_SCHUR_NC", "2"), ("SMPM_SCHUR_PERSIST", "-1")),
    "nc4": (("SMPM_SCHUR_NC", "4"), ("SMPM_SCHUR_PERSIST", "-1")),
    "persistent": (("SMPM_SCHUR_PERSIST", "1"),),
    "ws_nc1": (("SMPM_SCHUR_NC", "1"), ("SMPM_SCHUR_PERSIST", "2")),
    "ws_nc2": (("SMPM_SCHUR_NC", "2"), ("SMPM_SCHUR_PERSIST", "2")),
    "ws_nc4": (("SMPM_SCHUR_NC", "4"), ("SMPM_SCHUR_PERSIST", "2")),
    "cols_cpw2": (("SMPM_SCHUR_CPW", "2"), ("SMPM_SCHUR_PERSIST", "3")),
    "cols_cpw8": (("SMPM_SCHUR_CPW", "8"), ("SMPM_SCHUR_PERSIST", "3")),
}


@pytest.mark.parametrize("n", ORDERS)
@pytest.mark.parametrize("geom", sorted(GEOMS))
@pytest.mark.parametrize("shape", sorted(SHAPES))
@pytest.mark.parametrize("transpose", [False, True])
def test_schur_apply_fp64(n, geom, shape, transpose, monkeypatch):
    if n > 16 and shape != "nc1":
        pytest.skip("orders above 16 take the vector kernels, which have no launch-shape choice")
    ctx = context(geom, n, SHAPES[shape], monkeypatch)
    m = oracle(geom, n)
    V = wl.random_vectors(101 + n, 5, ctx.k)   # 5 columns: ragged for 2 and 4 per workgroup
    S = m.sys.S
    want = (S.T @ V.T).T if transpose else (S @ V.T).T
    got = ctx.schur_apply(dev(V), transpose=transpose).cpu().numpy()
    for c in range(5):
        assert rel(got[c], want[c]) <= 1e-12, (n, geom, shape, c, rel(got[c], want[c]))


@pytest.mark.parametrize("n", ORDERS)
@pytest.mark.parametrize("precision", ["fp32", "bf16"])
@pytest.mark.parametrize("shape", ["nc1", "nc4", "persistent", "ws_nc2", "cols_cpw2"])
@pytest.mark.parametrize("transpose", [False, True])
def test_schur_apply_low_precision(n, precision, shape, transpose, monkeypatch):
    if n > 16 and shape != "nc1":
        pytest.skip("orders above 16 take the vector kernels, which have no launch-shape choice")
    geom = "ragged_5x3"
    ctx = context(geom, n, SHAPES[shape], monkeypatch)
    m = oracle(geom, n)
    V = wl.random_vectors(111 + n, 3, ctx.k)
    S = m.sys.S
    want = (S.T @ V.T).T if transpose else (S @ V.T).T
    prec = smpm.MIXED_FP32 if precision == "fp32" else smpm.MIXED_BF16
    out = torch.empty(3, ctx.k, dtype=torch.float64, device="cuda")
    got = ctx.schur_apply_prec(dev(V), out, prec, transpose=transpose).cpu().numpy()
    bound = 1e-5 if precision == "fp32" else 2e-2
    for c in range(3):
        assert rel(got[c], want[c]) <= bound, (n, precision, shape, c, rel(got[c], want[c]))


@pytest.mark.parametrize("n", ORDERS)
@pytest.mark.parametrize("geom", sorted(GEOMS))
@pytest.mark.parametrize("transpose", [False, True])
def test_block_jacobi(n, geom, transpose, monkeypatch):
    ctx = context(geom, n, SHAPES["nc1"], monkeypatch)
    m = oracle(geom, n)
    V = wl.random_vectors(121 + n, 2, ctx.k)
    want = np.stack([m.M.solve_transpose(v) if transpose else m.M.solve(v) for v in V])
    got = ctx.precond_apply(dev(V), transpose=transpose).cpu().numpy()
    assert max(len(b) for b in m.M.members) <= 8 * n
    for c in range(2):
        assert rel(got[c], want[c]) <= 1e-11, (n, geom, c, rel(got[c], want[c]))


def rel_sign(a, b):
    return min(rel(a, b), rel(-a, b))


@pytest.mark.parametrize("n", ORDERS)
@pytest.mark.parametrize("geom", sorted(GEOMS))
def test_null_vectors(n, geom, monkeypatch):
    ctx = context(geom, n, SHAPES["nc1"], monkeypatch)
    m = oracle(geom, n)
    uL, uS = ctx.null_vectors()
    assert rel_sign(uS, m.sys.uS) <= 1e-10
    assert rel_sign(uL, m.sys.uL) <= 1e-10
    st = ctx.stats()
    assert 0 <= st["null_residual"] <= 1e-12, st["null_residual"]


@pytest.mark.parametrize("n", ORDERS)
@pytest.mark.parametrize("which", ["P", "Q"])
@pytest.mark.parametrize("transpose", [False, True])
def test_projections(n, which, transpose, monkeypatch):
    geom = "stretched_4x3"
    ctx = context(geom, n, SHAPES["nc1"], monkeypatch)
    m = oracle(geom, n)
    D = m.defl
    S = m.sys.S.toarray()
    Z = D.Z.toarray()
    X = wl.random_vectors(131 + n, 2, ctx.k)
    want = []
    for x in X:
        if which == "P":
            want.append(x - Z @ (D.G.T @ (Z.T @ (S.T @ x))) if transpose else D.P(x))
        else:
            want.append(x - S.T @ (Z @ (D.G.T @ (Z.T @ x))) if transpose else D.Q(x))
    code = smpm.PROJ_P if which == "P" else smpm.PROJ_Q
    got = ctx.project(code, dev(X), transpose=transpose).cpu().numpy()
    for c in range(2):
        assert rel(got[c], want[c]) <= 1e-10, (n, which, transpose, rel(got[c], want[c]))


def _problem(g, seed):
    x, y = g.node_coords()
    Lx, Ly = g.xb[-1] - g.xb[0], g.yb[-1] - g.yb[0]
    f = wl.eval_fourier(wl.random_fourier_params(seed, 20, 4), x, y, Lx, Ly)
    gb = wl.eval_edge(wl.random_edge_params(seed + 1), *g.boundary_arc(), Lx, Ly)
    return f, gb


@pytest.mark.parametrize("n", ORDERS)
@pytest.mark.parametrize("geom", sorted(GEOMS))
def test_solve_fp64(n, geom, monkeypatch):
    ctx = context(geom, n, SHAPES["nc1"], monkeypatch)
    m = oracle(geom, n)
    F, G, U = [], [], []
    for seed in (141, 143):
        f, gb = _problem(m.grid, seed)
        F.append(f)
        G.append(gb)
        U.append(O.solve_unreduced(m.split, f, gb)[0])
    u, info = ctx.solve(dev(np.stack(F)), dev(np.stack(G)), tol=1e-12, maxit=800)
    u = u.cpu().numpy()
    print(f"[gpu-orders] {geom} n={n}: {info.iterations} iterations, residual {info.rel_residual:.2e}")
    for c in range(2):
        assert rel(u[c], U[c]) <= 1e-10, (n, geom, c, rel(u[c], U[c]))
    assert info.rel_residual <= 1e-12


@pytest.mark.parametrize("n", ORDERS)
@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_solve_mixed(n, precision, monkeypatch):
    geom = "stretched_4x3"
    ctx = context(geom, n, SHAPES["nc1"], monkeypatch)
    m = oracle(geom, n)
    f, gb = _problem(m.grid, 151)
    want = O.solve_unreduced(m.split, f, gb)[0]
    prec = smpm.MIXED_FP32 if precision == "fp32" else smpm.MIXED_BF16
    inner = 1e-6 if precision == "fp32" else 1e-3
    u, info = ctx.solve(dev(f), dev(gb), tol=1e-10, maxit=800, precision=prec, inner_tol=inner, max_refine=30)
    err = rel(u.cpu().numpy()[0], want)
    print(f"[gpu-orders] mixed {precision} n={n}: {info.refinements} cycles, residual {info.rel_residual:.2e}, "
          f"error {err:.2e}")
    assert info.rel_residual <= 1e-10
    assert err <= 1e-6


@pytest.mark.parametrize("n", ORDERS)
def test_adjoint_solve(n, monkeypatch):
    geom = "ragged_5x3"
    ctx = context(geom, n, SHAPES["nc1"], monkeypatch)
    m = oracle(geom, n)
    c = wl.random_vectors(161 + n, 1, ctx.r)
    mu, info = ctx.solve(dev(c), tol=1e-12, maxit=800, transpose=True)
    want = O.solve_adjoint_unreduced(m.split, c[0])[0]
    assert rel(mu.cpu().numpy()[0], want) <= 1e-10
    assert info.rel_residual <= 1e-12
