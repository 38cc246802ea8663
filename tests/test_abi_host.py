"""CPU tests of libsmpm's host side: the library loads and exports every symbol the
header declares, argument validation, and the FP64 setup operators (S, B A^{-1},
M^{-1}, C, C^+) against the oracle.  No device call is made."""
import os
import re

import numpy as np
import pytest

import smpm_workloads as wl
from oracle import smpm_oracle as O

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
smpm = pytest.importorskip("paper_1601_03432_amd.smpm")


def _lib():
    if not os.path.exists(smpm.LIB_PATH):
        pytest.skip("libsmpm.so not built")
    return smpm.load_library()


def header_symbols():
    text = open(os.path.join(ROOT, "include", "smpm.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(smpm_[a-z_]+)\s*\(", text)))


def test_exports_every_declared_symbol():
    lib = _lib()
    syms = header_symbols()
    assert len(syms) >= 15
    for name in syms:
        assert hasattr(lib, name), name
    assert set(syms) == set(smpm.ABI_SYMBOLS)


@pytest.mark.parametrize("args", [
    (1, 1, 5, [0, 1], [0, 1], 8.0),          # one element: no interface
    (2, 2, 2, [0, .5, 1], [0, .5, 1], O.DEFAULT_ALPHA),  # n < 3
    (2, 2, 5, [0, .5, .4], [0, .5, 1], O.DEFAULT_ALPHA),  # non-increasing breaks
    (2, 2, 5, [0, .5, 1], [0, .5, 1], 0.0),     # zero penalty
])
def test_plan_rejects_bad_input(args):
    _lib()
    with pytest.raises(smpm.SmpmError) as ei:
        smpm.Context(*args, device=False)
    assert ei.value.code == smpm.EINVAL


def test_device_call_on_plan_context_fails_loudly():
    _lib()
    w = wl.workload("c1")
    ctx = smpm.Context.from_workload(w, device=False)
    with pytest.raises(smpm.SmpmError) as ei:
        ctx.null_vectors()
    assert ei.value.code == smpm.ENODEVICE


GRIDS = {
    "c1": lambda: (wl.workload("c1").n, wl.workload("c1").x_breaks, wl.workload("c1").y_breaks),
    "nonsquare": lambda: (6, wl.uniform_breaks(5, 2.0), wl.uniform_breaks(3, 1.0)),
    "stretched": lambda: (7, [0.0, 0.1, 0.25, 0.5, 1.0], [0.0, 0.3, 0.6, 1.0]),
    "two": lambda: (5, wl.uniform_breaks(2), wl.uniform_breaks(1)),
}


def test_plan_rejects_unknown_robin_mode():
    _lib()
    with pytest.raises(smpm.SmpmError) as ei:
        smpm.Context(2, 2, 5, [0, .5, 1], [0, .5, 1], 8.0, device=False, robin=7)
    assert ei.value.code == smpm.EINVAL


@pytest.mark.parametrize("robin", O.ROBIN_MODES)
@pytest.mark.parametrize("name", sorted(GRIDS))
def test_setup_operators_match_oracle(name, robin):
    _lib()
    n, xb, yb = GRIDS[name]()
    xb, yb = np.asarray(xb, float), np.asarray(yb, float)
    ctx = smpm.Context(len(yb) - 1, len(xb) - 1, n, xb, yb, O.DEFAULT_ALPHA, device=False, robin=robin)
    g = O.Grid(n, xb, yb, robin=robin)
    m = O.Method(g)
    assert (ctx.r, ctx.k, ctx.d) == (g.r, m.split.k, m.defl.d)
    assert np.array_equal(ctx.slot_map(), m.split.slot_node)
    x, y = ctx.node_coords()
    xo, yo = g.node_coords()
    assert np.abs(x - xo).max() < 1e-14 and np.abs(y - yo).max() < 1e-14
    assert np.abs(ctx.quadrature_weights() - g.quad_weights()).max() < 1e-15
    S = ctx.export(smpm.EXPORT_SCHUR).toarray()
    So = m.sys.S.toarray()
    assert np.abs(S - So).max() <= 1e-11 * np.abs(So).max()
    F = ctx.export(smpm.EXPORT_FLUX_SOLVE).toarray()
    Fo = (m.split.B @ m.split.Ainv).toarray()
    assert np.abs(F - Fo).max() <= 1e-11 * np.abs(Fo).max()
    Mi = ctx.export(smpm.EXPORT_PRECOND_INV).toarray()
    Mio = np.zeros_like(So)
    for mem, bi in zip(m.M.members, m.M.inv):
        Mio[np.ix_(mem, mem)] = bi
    assert np.abs(Mi - Mio).max() <= 1e-10 * np.abs(Mio).max()
    Cl = ctx.export(smpm.EXPORT_COARSE)
    Gl = ctx.export(smpm.EXPORT_COARSE_PINV)
    assert np.abs(Cl - m.defl.C).max() <= 1e-11 * max(1.0, np.abs(m.defl.C).max())
    assert np.abs(Gl - m.defl.G).max() <= 1e-9 * max(1e-300, np.abs(m.defl.G).max()) + 1e-14


def test_stretched_grid_has_nonsingular_coarse_matrix():
    """Unequal widths across vertical interfaces make tau differ on the two sides, so
    B 1 leaves range(Z) and C is nonsingular; then G = C^{-1}."""
    _lib()
    xb = np.array([0.0, 0.1, 0.25, 0.5, 1.0])
    yb = np.array([0.0, 0.3, 0.6, 1.0])
    ctx = smpm.Context(3, 4, 6, xb, yb, O.DEFAULT_ALPHA, device=False)
    Cl = ctx.export(smpm.EXPORT_COARSE)
    Gl = ctx.export(smpm.EXPORT_COARSE_PINV)
    assert np.abs(Cl @ Gl - np.eye(ctx.d)).max() < 1e-9


@pytest.mark.parametrize("name", sorted(GRIDS))
@pytest.mark.parametrize("patch", [1, 2, 3])
def test_substructured_coarse_matches_oracle(name, patch, monkeypatch):
    """The substructured coarse solve (forced on small grids; patch 1 makes every
    interface a separator) reproduces C^+ (C^{-1} when nonsingular) column by column."""
    _lib()
    monkeypatch.setenv("SMPM_DENSE_COARSE_MAX", "0")
    monkeypatch.setenv("SMPM_COARSE_PATCH", str(patch))
    n, xb, yb = GRIDS[name]()
    xb, yb = np.asarray(xb, float), np.asarray(yb, float)
    ctx = smpm.Context(len(yb) - 1, len(xb) - 1, n, xb, yb, O.DEFAULT_ALPHA, device=False)
    m = O.Method(O.Grid(n, xb, yb))
    Cl = ctx.export(smpm.EXPORT_COARSE)
    Gl = ctx.export(smpm.EXPORT_COARSE_PINV)
    assert np.abs(Cl - m.defl.C).max() <= 1e-11 * max(1.0, np.abs(m.defl.C).max())
    assert np.abs(Gl - m.defl.G).max() <= 1e-9 * max(1e-300, np.abs(m.defl.G).max()) + 1e-14


def test_dense_coarse_limit_is_capped(monkeypatch):
    """A dense-coarse limit above what the dense coarse kernel stages (4096
    interfaces) is capped: a grid with more interfaces still takes the substructured
    solve."""
    _lib()
    monkeypatch.setenv("SMPM_DENSE_COARSE_MAX", "1000000")
    m = 48
    xb = yb = np.linspace(0.0, 1.0, m + 1)
    ctx = smpm.Context(m, m, 4, xb, yb, O.DEFAULT_ALPHA, device=False)
    assert ctx.d == 2 * m * (m - 1) > 4096
    st = ctx.stats()
    assert st["has_coarse"] == 1
    assert 0 < st["coarse_bytes"] < ctx.d * ctx.d * 8


def test_struct_layouts_match_header(tmp_path):
    """The ctypes mirrors of the ABI structs have the header's field offsets and sizes
    (a tiny C program compiled against include/smpm.h prints them)."""
    import ctypes
    import shutil
    import subprocess
    if shutil.which("gcc") is None:
        pytest.skip("no C compiler")
    mirrors = {"smpm_solve_opts": smpm.SolveOpts, "smpm_solve_info": smpm.SolveInfo,
               "smpm_plan_stats": smpm.PlanStats, "smpm_tune_result": smpm.TuneResult}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "smpm.h"', "int main(void) {"]
    for cname, py in mirrors.items():
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for field, _ in py._fields_:
            if field.endswith("_"):
                continue  # explicit padding of the mirror
            lines.append(f'  printf("{cname} {field} %zu\\n", offsetof({cname}, {field}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    seen = 0
    for line in out:
        if not line:
            continue
        cname, field, value = line.split()
        py = mirrors[cname]
        want = ctypes.sizeof(py) if field == "size" else getattr(py, field).offset
        assert int(value) == want, (cname, field, int(value), want)
        seen += 1
    assert seen >= sum(len(p._fields_) for p in mirrors.values())
