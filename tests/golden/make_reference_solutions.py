"""Writes the oracle's direct solutions at full benchmark sizes, which the oracle
needs minutes to factor (too slow to recompute inside a GPU test):

* c2_u_ref.npy   -- u* of the 16 x 16, n = 16 grid on [0,2]^2 (r = 65,536) for the
                    random-Fourier source (20 modes, k <= 8, seed B+2), g = 0:
                    oracle.solve_unreduced (bordered sparse LU of L).
* c4_u_ref.npy   -- u* of the 32 x 32, n = 10 grid on [0,1]^2 (r = 102,400) for the
                    differentiation workload's f (seed B+40) and g (seed B+41).
* c4_mu_ref.npy  -- the adjoint mu = K^T c for the cotangent c = 2 (u* - u_t) of the
                    loss |u - u_t|^2, u_t from seed B+42: oracle.solve_adjoint_unreduced.

Only the oracle and the seeded input generators are called.  Penalty 8, Robin
length min(w, h)/2 (the defaults).  Run from the repository root:

    python tests/golden/make_reference_solutions.py
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import smpm_workloads as wl  # noqa: E402
from oracle import smpm_oracle as O  # noqa: E402


def c2():
    w = wl.workload("c2")
    g = O.Grid(w.n, w.x_breaks, w.y_breaks)
    split = O.Split(g)
    x, y = g.node_coords()
    f = wl.eval_fourier(wl.random_fourier_params(wl.SEED_BASE + 2, 20, 8), x, y, w.Lx, w.Ly)
    u, mu, _, _ = O.solve_unreduced(split, f)
    print(f"c2: bordered multiplier {mu:.2e}", flush=True)
    np.save(os.path.join(HERE, "c2_u_ref.npy"), u)


def c4():
    n, m = 10, 32
    g = O.Grid(n, wl.uniform_breaks(m), wl.uniform_breaks(m))
    split = O.Split(g)
    x, y = g.node_coords()
    f = wl.eval_fourier(wl.random_fourier_params(wl.SEED_BASE + 40, 20, 8), x, y, 1.0, 1.0)
    gb = wl.eval_edge(wl.random_edge_params(wl.SEED_BASE + 41), *g.boundary_arc(), 1.0, 1.0)
    ut = wl.eval_fourier(wl.random_fourier_params(wl.SEED_BASE + 42, 20, 8), x, y, 1.0, 1.0)
    u, mu_f, _, _ = O.solve_unreduced(split, f, gb)
    print(f"c4 forward: bordered multiplier {mu_f:.2e}", flush=True)
    np.save(os.path.join(HERE, "c4_u_ref.npy"), u)
    mu, lam, _ = O.solve_adjoint_unreduced(split, 2.0 * (u - ut))
    print(f"c4 adjoint: bordered multiplier {lam:.2e}", flush=True)
    np.save(os.path.join(HERE, "c4_mu_ref.npy"), mu)


if __name__ == "__main__":
    for fn in (c2, c4):
        t0 = time.perf_counter()
        fn()
        print(f"{fn.__name__}: {time.perf_counter() - t0:.0f} s", flush=True)
