"""Seeded synthetic inputs for the SMPM Poisson-Neumann solver.

This module is shared by the CPU oracle, the tests and the benchmark.  It holds
only the workload recipes (grid breakpoints, random draws and the closed-form
source fields evaluated at caller-supplied coordinates).  It contains none of
the method's arithmetic: no quadrature, no differentiation, no projection.
Node coordinates are computed by whoever calls it (the oracle computes its own,
the library reports its own).

All random numbers come from ``numpy.random.default_rng(seed)`` (PCG64) and are
drawn in the order documented in each function, so a seed fixes the input bit
for bit.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

SEED_BASE = 160103432  # the arXiv identifier 1601.03432 as an integer


# ---------------------------------------------------------------------------
# geometry recipes
# ---------------------------------------------------------------------------

def uniform_breaks(m: int, length: float = 1.0) -> np.ndarray:
    """m equal elements on [0, length]: m + 1 breakpoints."""
    return np.linspace(0.0, length, m + 1)


def stretched_breaks(m: int, ratio: float = 1.05, cap: float = 8.0):
    """Element widths growing geometrically away from the wall x = 0.

    w_j = w0 * min(ratio**j, cap), j = 0..m-1, scaled so the widths sum to 1.
    Returns (x_breaks, w0).  With a uniform y spacing h = cap * w0 the aspect
    ratio is ``cap`` at the wall and 1 far from it.
    """
    rel = np.minimum(ratio ** np.arange(m, dtype=np.float64), cap)
    w0 = 1.0 / rel.sum()
    widths = w0 * rel
    xb = np.concatenate([[0.0], np.cumsum(widths)])
    xb[-1] = 1.0
    return xb, w0


@dataclass
class Workload:
    name: str
    n: int
    x_breaks: np.ndarray
    y_breaks: np.ndarray
    nrhs: int = 1
    note: str = ""
    extra: dict = field(default_factory=dict)

    @property
    def m_x(self) -> int:
        return len(self.x_breaks) - 1

    @property
    def m_y(self) -> int:
        return len(self.y_breaks) - 1

    @property
    def Lx(self) -> float:
        return float(self.x_breaks[-1] - self.x_breaks[0])

    @property
    def Ly(self) -> float:
        return float(self.y_breaks[-1] - self.y_breaks[0])


def workload(name: str) -> Workload:
    """The named workloads.

    c1  4x4 elements, n=8 on [0,1]^2, manufactured cos(pi x) cos(pi y)
    c2  16x16 elements, n=16 on [0,2]^2, random-Fourier source (k<=8)
    c3  64x64 elements, n=12 on [0,1]^2, 32 advected sources
    c4  32x32 elements, n=10 on [0,1]^2, differentiation workload
    c5  128x128 elements, n=16, x-stretched (ratio 1.05, aspect <= 8), 8 RHS
    c5a/c5b/c5c  the three side grids 16x16 n=8, 32x32 n=12, 48x48 n=10
    paper_h{m}  m x m elements, n=5 on [0,1]^2 (h-refinement study)
    paper_p{n}  4x4 elements, n points on [0,1]^2 (p-refinement study)
    """
    if name == "c1":
        return Workload("c1", 8, uniform_breaks(4), uniform_breaks(4), 1,
                        "4x4 n=8 [0,1]^2 manufactured cos(pi x)cos(pi y)")
    if name == "c2":
        return Workload("c2", 16, uniform_breaks(16, 2.0), uniform_breaks(16, 2.0), 1,
                        "16x16 n=16 [0,2]^2 random-Fourier source k<=8")
    if name == "c3":
        return Workload("c3", 12, uniform_breaks(64), uniform_breaks(64), 32,
                        "64x64 n=12 [0,1]^2 32 advected sources")
    if name == "c4":
        return Workload("c4", 10, uniform_breaks(32), uniform_breaks(32), 1,
                        "32x32 n=10 [0,1]^2 differentiation")
    if name == "c5":
        xb, w0 = stretched_breaks(128)
        yb = np.arange(129, dtype=np.float64) * (8.0 * w0)
        return Workload("c5", 16, xb, yb, 8,
                        "128x128 n=16 x-stretched (1.05, aspect<=8)", {"w0": w0})
    if name == "c5a":
        return Workload("c5a", 8, uniform_breaks(16), uniform_breaks(16), 8, "16x16 n=8")
    if name == "c5b":
        return Workload("c5b", 12, uniform_breaks(32), uniform_breaks(32), 8, "32x32 n=12")
    if name == "c5c":
        return Workload("c5c", 10, uniform_breaks(48), uniform_breaks(48), 8, "48x48 n=10")
    if name.startswith("paper_h"):
        m = int(name[len("paper_h"):])
        return Workload(name, 5, uniform_breaks(m), uniform_breaks(m), 1, f"{m}x{m} n=5")
    if name.startswith("paper_p"):
        n = int(name[len("paper_p"):])
        return Workload(name, n, uniform_breaks(4), uniform_breaks(4), 1, f"4x4 n={n}")
    raise KeyError(name)


# ---------------------------------------------------------------------------
# source fields
# ---------------------------------------------------------------------------

def manufactured_cos(x, y, lam: int = 1, Lx: float = 1.0, Ly: float = 1.0):
    """u = cos(lam pi x/Lx) cos(lam pi y/Ly) and f = lap u.

    Its normal derivative vanishes on the walls of [0,Lx]x[0,Ly], so g = 0.
    Returns (u, f).
    """
    kx = lam * math.pi / Lx
    ky = lam * math.pi / Ly
    u = np.cos(kx * x) * np.cos(ky * y)
    f = -(kx * kx + ky * ky) * u
    return u, f


@dataclass
class FourierParams:
    kx: np.ndarray
    ky: np.ndarray
    amp: np.ndarray
    phx: np.ndarray
    phy: np.ndarray


def random_fourier_params(seed: int, modes: int = 20, kmax: int = 8) -> FourierParams:
    """Draw `modes` random Fourier modes.

    Draw order per mode m: kx, ky ~ U{0..kmax} (both redrawn while both are 0),
    amplitude ~ N(0,1), phase_x, phase_y ~ U[0, 2 pi).
    """
    rng = np.random.default_rng(seed)
    kx = np.zeros(modes, np.int64)
    ky = np.zeros(modes, np.int64)
    amp = np.zeros(modes)
    phx = np.zeros(modes)
    phy = np.zeros(modes)
    for m in range(modes):
        while True:
            a = int(rng.integers(0, kmax + 1))
            b = int(rng.integers(0, kmax + 1))
            if a != 0 or b != 0:
                break
        kx[m], ky[m] = a, b
        amp[m] = rng.standard_normal()
        phx[m] = rng.uniform(0.0, 2.0 * math.pi)
        phy[m] = rng.uniform(0.0, 2.0 * math.pi)
    return FourierParams(kx, ky, amp, phx, phy)


def eval_fourier(p: FourierParams, x, y, Lx: float, Ly: float):
    """sum_m amp_m cos(pi kx_m x/Lx + phx_m) cos(pi ky_m y/Ly + phy_m)."""
    x = np.asarray(x, np.float64)
    y = np.asarray(y, np.float64)
    out = np.zeros(np.broadcast(x, y).shape)
    for m in range(len(p.amp)):
        out += p.amp[m] * np.cos(math.pi * p.kx[m] * x / Lx + p.phx[m]) \
            * np.cos(math.pi * p.ky[m] * y / Ly + p.phy[m])
    return out


def random_edge_params(seed: int, terms: int = 4) -> np.ndarray:
    """Coefficients b[edge, l] ~ N(0,1), edges in the order south, north, west, east."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal((4, terms))


def eval_edge(b: np.ndarray, s_south, s_north, s_west, s_east, Lx: float, Ly: float):
    """Neumann data g(s) = sum_l b[edge,l] cos(l pi s/len) on each edge.

    s_* are the arc-length coordinates of the boundary nodes (x for south and
    north, y for west and east).  Returns the concatenation south, north, west,
    east, which is the boundary-data layout the library takes.
    """
    parts = []
    for e, (s, length) in enumerate(((s_south, Lx), (s_north, Lx), (s_west, Ly), (s_east, Ly))):
        s = np.asarray(s, np.float64)
        g = np.zeros_like(s)
        for l in range(b.shape[1]):
            g += b[e, l] * np.cos(l * math.pi * s / length)
        parts.append(g)
    return np.concatenate(parts)


def advected_sources(seed: int, x, y, count: int = 32, dt: float = 1e-3,
                     noise_std: float = 1e-3, kmax: int = 4, Lx: float = 1.0, Ly: float = 1.0):
    """A smooth random-Fourier field carried by a uniform velocity.

    Draw order: the base field's modes (as random_fourier_params(seed, 20, kmax)),
    then the velocity c ~ U[-1,1]^2, then per step k = 1..count the node noise
    N(0, noise_std^2).  f_k(x,y) = f0(x - c_x k dt, y - c_y k dt) + noise, with its
    plain nodal mean subtracted.  Returns an array (count, len(x)).
    """
    p = random_fourier_params(seed, 20, kmax)
    rng = np.random.default_rng(seed + 1_000_003)
    c = rng.uniform(-1.0, 1.0, size=2)
    out = np.zeros((count, np.size(x)))
    for k in range(1, count + 1):
        fk = eval_fourier(p, np.asarray(x) - c[0] * k * dt, np.asarray(y) - c[1] * k * dt, Lx, Ly)
        fk = fk.ravel() + noise_std * rng.standard_normal(np.size(x))
        out[k - 1] = fk - fk.mean()
    return out


C5_SIDE_GRIDS = ("c5a", "c5b", "c5c")


def c5_sources(name: str, x, y, arc, Lx: float, Ly: float, count: int = 8):
    """Right-hand sides of the large stretched grid ("c5": seeds B+50+i for f_i and
    B+60+i for g_i) and of its side grids ("c5a"/"c5b"/"c5c" = G 0/1/2: seeds
    B+70+10G+i for f_i and B+100+10G+i for g_i): random-Fourier sources (20 modes,
    k <= 8) and nonzero cosine-series Neumann data on every edge.
    Returns (F (count, len(x)), G (count, len(arc concatenated)))."""
    if name == "c5":
        sf, sg = SEED_BASE + 50, SEED_BASE + 60
    else:
        G = C5_SIDE_GRIDS.index(name)
        sf, sg = SEED_BASE + 70 + 10 * G, SEED_BASE + 100 + 10 * G
    F = np.stack([eval_fourier(random_fourier_params(sf + i, 20, 8), x, y, Lx, Ly) for i in range(count)])
    Gd = np.stack([eval_edge(random_edge_params(sg + i), *arc, Lx, Ly) for i in range(count)])
    return F, Gd


def random_directions(seed: int, count: int, size: int) -> np.ndarray:
    """`count` N(0,1) directions of length `size`, each scaled to unit 2-norm."""
    rng = np.random.default_rng(seed)
    d = rng.standard_normal((count, size))
    return d / np.linalg.norm(d, axis=1, keepdims=True)


def random_vectors(seed: int, count: int, size: int) -> np.ndarray:
    """Plain N(0,1) test vectors (count, size)."""
    return np.random.default_rng(seed).standard_normal((count, size))
