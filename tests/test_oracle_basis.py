"""Pins of the oracle's GLL basis, interpolation and random generator (CPU only).

Sec. 2.1: GLL quadrature and the degree-p cardinal basis on the GLL points.
"""
import math
import os

import numpy as np
import pytest

from oracle import gll, rng

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _parse_expr(s):
    return float(eval(s.strip(), {"sqrt": math.sqrt}))


def test_gll_textbook_values():
    rows = [l for l in open(os.path.join(GOLDEN, "gll_textbook.txt")) if not l.startswith("#")]
    assert len(rows) == 3
    for row in rows:
        p, nodes, weights = row.split(":")
        xi, w = gll.gll_nodes_weights(int(p))
        np.testing.assert_allclose(xi, [_parse_expr(t) for t in nodes.split(",")], atol=1e-15)
        np.testing.assert_allclose(w, [_parse_expr(t) for t in weights.split(",")], atol=1e-15)


@pytest.mark.parametrize("p", range(1, 12))
def test_gll_quadrature_exactness(p):
    """sum w x^k = int_{-1}^{1} x^k for k <= 2p-1 and not for k = 2p."""
    xi, w = gll.gll_nodes_weights(p)
    for k in range(2 * p):
        exact = 0.0 if k % 2 else 2.0 / (k + 1)
        assert abs(np.dot(w, xi ** k) - exact) < 1e-13
    k = 2 * p
    assert abs(np.dot(w, xi ** k) - 2.0 / (k + 1)) > 1e-9


@pytest.mark.parametrize("p", range(1, 11))
def test_derivative_matrix_exact_on_polynomials(p):
    xi, _, D = gll.gll(p)
    for k in range(p + 1):
        dk = k * xi ** (k - 1) if k else np.zeros_like(xi)
        np.testing.assert_allclose(D @ xi ** k, dk, atol=1e-11 * max(1, k * k))
    np.testing.assert_allclose(D.sum(axis=1), 0.0, atol=1e-12)
    # textbook closed form (Deville et al. App. B) for the diagonal corners
    assert abs(D[0, 0] + p * (p + 1) / 4.0) < 1e-11
    assert abs(D[p, p] - p * (p + 1) / 4.0) < 1e-11


def test_derivative_matrix_closed_form_offdiagonal():
    """Dhat_ij = P_p(xi_i) / (P_p(xi_j) (xi_i - xi_j)) for i != j."""
    for p in (2, 5, 7, 9):
        xi, _, D = gll.gll(p)
        P = gll.legendre(p, xi)
        for i in range(p + 1):
            for j in range(p + 1):
                if i != j:
                    assert abs(D[i, j] - P[i] / (P[j] * (xi[i] - xi[j]))) < 1e-11


@pytest.mark.parametrize("pc,pf", [(1, 3), (3, 7), (5, 9), (3, 5), (1, 2)])
def test_interpolation_reproduces_polynomials(pc, pf):
    J = gll.interpolation(pc, pf)
    xc, _ = gll.gll_nodes_weights(pc)
    xf, _ = gll.gll_nodes_weights(pf)
    for k in range(pc + 1):
        np.testing.assert_allclose(J @ xc ** k, xf ** k, atol=1e-13)
    np.testing.assert_allclose(J.sum(axis=1), 1.0, atol=1e-13)


def test_splitmix64_known_answers():
    vals = [int(l) for l in open(os.path.join(GOLDEN, "splitmix64_seed1234567.txt"))
            if l.strip() and not l.startswith("#")]
    s = np.uint64(1234567)
    g = np.uint64(0x9E3779B97F4A7C15)
    got = []
    with np.errstate(over="ignore"):
        for _ in vals:
            got.append(int(rng.splitmix64(s)))
            s = s + g
    assert got == vals


def test_uniform_pm1_range_and_mean():
    u = rng.uniform_pm1(7, np.arange(200000))
    assert u.min() >= -1.0 and u.max() < 1.0
    assert abs(u.mean()) < 0.01 and abs(np.mean(u * u) - 1.0 / 3.0) < 0.01
