"""Pins of the oracle's GLL grid (Sec. 1.2) against closed forms and exactness."""
import math
import os

import numpy as np
import pytest

from oracle.smpm_oracle import gll


def test_gll_n5_closed_form(golden_dir):
    data = np.loadtxt(os.path.join(golden_dir, "gll_n5.txt"), comments="#")
    x, w, _ = gll(5)
    assert np.allclose(x, data[:, 0], atol=1e-15, rtol=0)
    assert np.allclose(w, data[:, 1], atol=1e-15, rtol=0)
    assert abs(x[3] - math.sqrt(3.0 / 7.0)) < 1e-15


@pytest.mark.parametrize("n", [2, 3, 4, 5, 8, 12, 16, 20])
def test_gll_quadrature_exactness(n):
    """GLL quadrature integrates x^j exactly for j <= 2N-1 and not for j = 2N."""
    x, w, _ = gll(n)
    Np = n - 1
    assert abs(w.sum() - 2.0) < 1e-14
    for j in range(0, 2 * Np):
        exact = 0.0 if j % 2 else 2.0 / (j + 1)
        assert abs(w @ x ** j - exact) < 1e-13, j
    if Np >= 1:
        j = 2 * Np
        assert abs(w @ x ** j - 2.0 / (j + 1)) > 1e-12


@pytest.mark.parametrize("n", [3, 5, 8, 12, 16])
def test_gll_nodes_symmetric_and_sorted(n):
    x, w, _ = gll(n)
    assert np.all(np.diff(x) > 0)
    assert np.allclose(x, -x[::-1], atol=1e-15)
    assert np.allclose(w, w[::-1], atol=1e-15)


@pytest.mark.parametrize("n", [3, 5, 8, 12, 16])
def test_differentiation_matrix_exact_on_polynomials(n):
    """D differentiates every polynomial of degree <= N exactly at the nodes."""
    x, _, D = gll(n)
    Np = n - 1
    assert np.abs(D @ np.ones(n)).max() < 1e-12 * n * n
    for j in range(1, Np + 1):
        got = D @ x ** j
        want = j * x ** (j - 1)
        assert np.abs(got - want).max() < 1e-11 * max(1, j * j), j


def test_differentiation_matrix_corner_entries():
    x, _, D = gll(7)
    Np = 6
    assert abs(D[0, 0] + Np * (Np + 1) / 4) < 1e-14
    assert abs(D[-1, -1] - Np * (Np + 1) / 4) < 1e-14
