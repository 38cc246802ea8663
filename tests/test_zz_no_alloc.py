"""smpm_project_noalloc (the projections with the library's static scratch, no device
allocation) against smpm_project through the C ABI: the same kernels in the same
order, so every output must be bit-identical.  Two calls in a row share the one
static array: the second on a smaller input (a smaller grid, fewer columns) than
the first, for every projection and both directions; a call over the stated
scratch maximum and an L/S projection before the null vectors exist are rejected."""
import numpy as np
import pytest

import smpm_workloads as wl
from oracle import smpm_oracle as O

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
smpm = pytest.importorskip("paper_1601_03432_amd.smpm")

KINDS = {"L": 0, "S": 1, "P": 2, "Q": 3, "MEAN": 4}


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


_ctx = {}


def ctx_of(name):
    if name not in _ctx:
        if name == "big":  # substructured coarse solve (d > 4096 interfaces)
            w = wl.workload("c3")
            c = smpm.Context.from_workload(w)
        elif name == "mid":
            w = wl.workload("c2")
            c = smpm.Context.from_workload(w)
        else:
            c = smpm.Context(3, 5, 6, wl.uniform_breaks(5, 1.5), wl.uniform_breaks(3), O.DEFAULT_ALPHA)
        c.null_vectors()
        _ctx[name] = c
    return _ctx[name]


def dev(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


@pytest.mark.parametrize("kind", sorted(KINDS))
@pytest.mark.parametrize("transpose", [False, True])
@pytest.mark.parametrize("first,second", [(("mid", 3), ("small", 1)), (("big", 2), ("mid", 1))])
def test_noalloc_matches_project(kind, transpose, first, second):
    which = KINDS[kind]
    for seed, (name, cols) in enumerate((first, second)):
        ctx = ctx_of(name)
        length = ctx.r if kind in ("L", "MEAN") else ctx.k
        X = dev(wl.random_vectors(400 + seed, cols, length))
        want = ctx.project(which, X, transpose=transpose)
        out = torch.full_like(X, float("nan"))
        got = ctx.project_noalloc(which, X, out, transpose=transpose)
        torch.cuda.synchronize()
        assert torch.equal(got, want), (kind, transpose, name, cols)
        # in place
        Y = X.clone()
        ctx.project_noalloc(which, Y, Y, transpose=transpose)
        assert torch.equal(Y, want), (kind, transpose, name, cols, "in place")


def test_noalloc_rejects_oversized_call():
    ctx = ctx_of("mid")
    cols = 300  # ~ (k + 2 d) * 300 doubles > 4 Mi doubles
    X = torch.zeros(cols, ctx.k, dtype=torch.float64, device="cuda")
    with pytest.raises(smpm.SmpmError) as ei:
        ctx.project_noalloc(smpm.PROJ_Q, X, torch.empty_like(X))
    assert ei.value.code == smpm.EINVAL and "scratch" in str(ei.value)


def test_noalloc_needs_null_vectors_first():
    c = smpm.Context(2, 3, 5, wl.uniform_breaks(3), wl.uniform_breaks(2), O.DEFAULT_ALPHA)
    X = dev(wl.random_vectors(410, 1, c.r))
    with pytest.raises(smpm.SmpmError) as ei:
        c.project_noalloc(smpm.PROJ_L, X, torch.empty_like(X))
    assert ei.value.code == smpm.EINVAL
    # the transposed L projection and the other kinds need no null vector
    want = c.project(smpm.PROJ_MEAN, X)
    assert torch.equal(c.project_noalloc(smpm.PROJ_MEAN, X, torch.empty_like(X)), want)
