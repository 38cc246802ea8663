"""GPU parity of libsmpm against the CPU FP64 oracle, through the C ABI.

Grids span several kernel tiles and ragged tails (element counts not multiples
of the 4 elements a Schur block handles), a non-square domain, a stretched grid
with a nonsingular coarse matrix, and the degenerate two-element grid.  FP64
tolerance: relative L2 <= 1e-10 for solves (the stated FP64 bar) and <= 1e-12
for single operator applies, whose only error source is the two independent FP64
setups (measured agreement ~1e-13)."""
import math

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


def setup(name):
    if name not in _cache:
        n, xb, yb = GRIDS[name]
        print(f"[gpu-parity] setup {name} n={n} m_x={len(xb) - 1} m_y={len(yb) - 1}", flush=True)
        ctx = smpm.Context(len(yb) - 1, len(xb) - 1, n, xb, yb, O.DEFAULT_ALPHA, device=True)
        m = O.Method(O.Grid(n, xb, yb))
        _cache[name] = (ctx, m)
    return _cache[name]


def dev(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def rel_sign(a, b):
    """Relative difference of two vectors defined up to sign (null vectors)."""
    return min(rel(a, b), rel(-a, b))


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.mark.parametrize("name", sorted(GRIDS))
@pytest.mark.parametrize("transpose", [False, True])
def test_schur_apply(name, transpose):
    ctx, m = setup(name)
    V = wl.random_vectors(11, 3, ctx.k)
    S = m.sys.S
    want = (S.T @ V.T).T if transpose else (S @ V.T).T
    got = ctx.schur_apply(dev(V), transpose=transpose).cpu().numpy()
    for c in range(3):
        assert rel(got[c], want[c]) <= 1e-12, (name, c, rel(got[c], want[c]))


@pytest.mark.parametrize("name", sorted(GRIDS))
@pytest.mark.parametrize("transpose", [False, True])
def test_precond_apply(name, transpose):
    ctx, m = setup(name)
    V = wl.random_vectors(12, 2, ctx.k)
    want = np.stack([m.M.solve_transpose(v) if transpose else m.M.solve(v) for v in V])
    got = ctx.precond_apply(dev(V), transpose=transpose).cpu().numpy()
    for c in range(2):
        assert rel(got[c], want[c]) <= 1e-11, (name, c, rel(got[c], want[c]))


@pytest.mark.parametrize("name", sorted(GRIDS))
def test_null_vectors(name):
    ctx, m = setup(name)
    uL, uS = ctx.null_vectors()
    assert rel_sign(uS, m.sys.uS) <= 1e-10
    assert rel_sign(uL, m.sys.uL) <= 1e-10


@pytest.mark.parametrize("name", ["c1", "stretched_4x3", "ragged_9x7"])
@pytest.mark.parametrize("which", ["P", "Q", "S", "L", "MEAN"])
@pytest.mark.parametrize("transpose", [False, True])
def test_projections(name, which, transpose):
    ctx, m = setup(name)
    D = m.defl
    S = m.sys.S.toarray()
    Z = D.Z.toarray()
    G = D.G
    g = m.grid
    w = g.quad_weights()
    if which in ("L", "MEAN"):
        X = wl.random_vectors(13, 2, ctx.r)
    else:
        X = wl.random_vectors(13, 2, ctx.k)
    want = []
    for x in X:
        if which == "P":
            y = x - Z @ (G.T @ (Z.T @ (S.T @ x))) if transpose else D.P(x)
        elif which == "Q":
            y = x - S.T @ (Z @ (G.T @ (Z.T @ x))) if transpose else D.Q(x)
        elif which == "S":
            u = m.sys.v0 / np.linalg.norm(m.sys.v0) if transpose else m.sys.uS
            y = x - u * (u @ x)
        elif which == "L":
            u = np.ones(g.r) / math.sqrt(g.r) if transpose else m.sys.uL
            y = x - u * (u @ x)
        else:
            y = x - w * x.sum() / w.sum() if transpose else x - (w @ x) / w.sum()
        want.append(y)
    code = {"P": smpm.PROJ_P, "Q": smpm.PROJ_Q, "S": smpm.PROJ_S, "L": smpm.PROJ_L, "MEAN": smpm.PROJ_MEAN}[which]
    got = ctx.project(code, dev(X), transpose=transpose).cpu().numpy()
    for c in range(2):
        assert rel(got[c], want[c]) <= 1e-10, (name, which, transpose, rel(got[c], want[c]))


def _problem(g, seed, with_g=True):
    x, y = g.node_coords()
    p = wl.random_fourier_params(seed, 20, 4)
    f = wl.eval_fourier(p, x, y, g.xb[-1] - g.xb[0], g.yb[-1] - g.yb[0])
    gb = None
    if with_g:
        b = wl.random_edge_params(seed + 1)
        gb = wl.eval_edge(b, *g.boundary_arc(), g.xb[-1] - g.xb[0], g.yb[-1] - g.yb[0])
    return f, gb


@pytest.mark.parametrize("name", sorted(GRIDS))
def test_solve_matches_direct(name):
    ctx, m = setup(name)
    g = m.grid
    F, Gs, U = [], [], []
    for seed in (21, 22):
        f, gb = _problem(g, seed)
        u_ref, *_ = O.solve_unreduced(m.split, f, gb)
        F.append(f)
        Gs.append(gb)
        U.append(u_ref)
    u, info = ctx.solve(dev(np.stack(F)), dev(np.stack(Gs)), tol=1e-12, maxit=600)
    u = u.cpu().numpy()
    print(f"[gpu-parity] {name}: iterations {info.iterations} true residual {info.rel_residual:.2e}")
    for c in range(2):
        assert rel(u[c], U[c]) <= 1e-10, (name, c, rel(u[c], U[c]))
    assert info.rel_residual <= 1e-11


@pytest.mark.parametrize("variant", [1, 2, 3])
def test_solve_variants_c1_manufactured(variant):
    ctx, m = setup("c1")
    g = m.grid
    x, y = g.node_coords()
    u_exact, f = wl.manufactured_cos(x, y)
    u_ref, *_ = O.solve_unreduced(m.split, f)
    u, info = ctx.solve(dev(f), tol=1e-12, maxit=600, variant=variant)
    u = u.cpu().numpy()[0]
    assert rel(u, u_ref) <= 1e-10
    # discretization error of the manufactured solution (spectral at n = 8)
    assert np.abs(u - O.mean_zero(g, u_exact)).max() < 1e-6
    # iteration count close to the oracle's textbook GMRES, both stopping at the same
    # absolute Schur residual (the library's rule is relative to |b_hat|, the oracle's
    # to the initial GMRES residual |P b_hat|)
    _, _, bhat = m.sys.schur_rhs(f)
    r0 = np.linalg.norm(m.defl.P(bhat)) if variant == 3 else np.linalg.norm(bhat)
    it_or = m.solve(f, variant=variant, tol=1e-12 * np.linalg.norm(bhat) / r0)[1]["iters"]
    assert abs(info.iterations - it_or) <= 3, (info.iterations, it_or)


@pytest.mark.parametrize("name", ["c1", "nonsquare_5x3", "ragged_9x7", "stretched_4x3"])
@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_solve_mixed_precision(name, precision):
    """FP32 / BF16 Schur and block-Jacobi operators inside FP64 iterative refinement:
    the FP64 true residual reaches 1e-10 and the solution matches the oracle to the
    1e-6 mixed-precision bar."""
    ctx, m = setup(name)
    g = m.grid
    f, gb = _problem(g, 31)
    u_ref, *_ = O.solve_unreduced(m.split, f, gb)
    prec = smpm.MIXED_FP32 if precision == "fp32" else smpm.MIXED_BF16
    inner = 1e-6 if precision == "fp32" else 1e-3
    u, info = ctx.solve(dev(f), dev(gb), tol=1e-10, maxit=600, precision=prec, inner_tol=inner, max_refine=30)
    u = u.cpu().numpy()[0]
    print(f"[gpu-parity] mixed {precision} {name}: {info.iterations} inner iterations, "
          f"{info.refinements} refinements, true residual {info.rel_residual:.2e}, error {rel(u, u_ref):.2e}")
    assert info.rel_residual <= 1e-10
    assert rel(u, u_ref) <= 1e-6
    assert info.refinements >= 1


def test_batched_columns_match_single():
    """A batched solve returns, column by column, what single-column solves return."""
    ctx, m = setup("ragged_9x7")
    g = m.grid
    F = np.stack([_problem(g, 40 + i, with_g=False)[0] for i in range(5)])
    ub, _ = ctx.solve(dev(F), tol=1e-12, maxit=600)
    ub = ub.cpu().numpy()
    for i in range(5):
        us, _ = ctx.solve(dev(F[i]), tol=1e-12, maxit=600)
        assert rel(ub[i], us.cpu().numpy()[0]) <= 1e-12


@pytest.mark.parametrize("mode", ["fp64", "mixed_fp32", "adjoint"])
def test_graph_replays_match_eager(mode):
    """Arnoldi steps replayed from the captured hipGraph give, bit for bit, the solutions
    of the same steps launched one by one, over repeated solves with eager work (other
    solves, Schur applies, synchronizations) in between."""
    ctx, m = setup("ragged_9x7")
    g = m.grid
    F = dev(np.stack([_problem(g, 60 + i, with_g=False)[0] for i in range(3)]))
    kw = dict(tol=1e-11, maxit=600)
    if mode == "mixed_fp32":
        kw.update(precision=smpm.MIXED_FP32, inner_tol=1e-6, max_refine=30)
    if mode == "adjoint":
        kw.update(transpose=True)
    ref, info_ref = ctx.solve(F, graph=False, **kw)
    for rep in range(3):
        u, info = ctx.solve(F, graph=True, **kw)
        assert torch.equal(u, ref), (mode, rep)
        assert info.iterations == info_ref.iterations
        ctx.schur_apply(dev(wl.random_vectors(70 + rep, 2, ctx.k)))
        ctx.solve(F[:1], graph=False, **kw)
        torch.cuda.synchronize()


def test_prereduced_sums_match_per_block_sums(monkeypatch):
    """The orthogonalization sums reduced once per column (large batched grids) and
    reduced by every consumer block (small grids) add the same partials in the same
    order: the solutions agree bit for bit."""
    ctx, m = setup("ragged_9x7")
    g = m.grid
    F = dev(np.stack([_problem(g, 80 + i, with_g=False)[0] for i in range(4)]))
    sols = []
    for flag in ("0", "1"):
        monkeypatch.setenv("SMPM_PREREDUCE", flag)
        u, info = ctx.solve(F, tol=1e-11, maxit=600)
        sols.append((u, info.iterations))
    assert torch.equal(sols[0][0], sols[1][0]) and sols[0][1] == sols[1][1]


_pers_cache = {}


@pytest.mark.parametrize("name", ["c1", "stretched_4x3", "ragged_9x7", "two_2x1"])
@pytest.mark.parametrize("transpose", [False, True])
@pytest.mark.parametrize("ncol", [1, 3])
def test_schur_apply_persistent(name, transpose, ncol, monkeypatch):
    """The persistent, pipelined Schur kernel (forced on; large grids choose it by
    themselves) against the oracle's S, for one column and for a ragged column group."""
    if name not in _pers_cache:
        monkeypatch.setenv("SMPM_SCHUR_PERSIST", "1")
        n, xb, yb = GRIDS[name]
        _pers_cache[name] = smpm.Context(len(yb) - 1, len(xb) - 1, n, xb, yb, O.DEFAULT_ALPHA, device=True)
    ctx = _pers_cache[name]
    _, m = setup(name)
    V = wl.random_vectors(15, ncol, ctx.k)
    S = m.sys.S
    want = (S.T @ V.T).T if transpose else (S @ V.T).T
    got = ctx.schur_apply(dev(V), transpose=transpose).cpu().numpy()
    for c in range(ncol):
        assert rel(got[c], want[c]) <= 1e-12, (name, c, rel(got[c], want[c]))


@pytest.mark.parametrize("name", ["c1", "stretched_4x3", "ragged_9x7"])
@pytest.mark.parametrize("precision", ["fp32", "bf16"])
@pytest.mark.parametrize("transpose", [False, True])
def test_schur_apply_low_precision(name, precision, transpose):
    """S v with FP32 / BF16 element operators and FP32 accumulation against the oracle's
    FP64 S.  Bound: the operator rounding (2^-24 resp. 2^-8 relative) accumulated over
    at most 64 terms, applied to the B A^{-1} E part only (the identity part is FP64):
    1e-5 for FP32, 2e-2 for BF16."""
    ctx, m = setup(name)
    V = wl.random_vectors(16, 3, ctx.k)
    S = m.sys.S
    want = (S.T @ V.T).T if transpose else (S @ V.T).T
    prec = smpm.MIXED_FP32 if precision == "fp32" else smpm.MIXED_BF16
    out = torch.empty(3, ctx.k, dtype=torch.float64, device="cuda")
    got = ctx.schur_apply_prec(dev(V), out, prec, transpose=transpose).cpu().numpy()
    bound = 1e-5 if precision == "fp32" else 2e-2
    for c in range(3):
        assert rel(got[c], want[c]) <= bound, (name, precision, c, rel(got[c], want[c]))
