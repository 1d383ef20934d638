"""GLL quadrature and Lagrange cardinal basis on [-1, 1] (oracle, test-only).

Follows Sec. 2.1: the local basis h_i is the degree-p Lagrange cardinal
polynomial on the Gauss-Lobatto-Legendre points, and the discrete inner
product (.,.)_p is GLL quadrature on the reference element [-1,1]^3.

Textbook definitions used (Deville, Fischer & Mund, 2002, which the paper
cites for the SE method):
  * nodes: xi_0 = -1, xi_p = +1, interior nodes = roots of P_p'(x);
  * weights: w_j = 2 / (p (p+1) P_p(xi_j)^2);
  * derivative matrix: Dhat[i, j] = h_j'(xi_i);
  * interpolation matrix: J[i, j] = h_j(x_i) for target points x_i.
"""
import numpy as np


def legendre(p, x):
    """P_p(x) by the three-term recurrence (k+1) P_{k+1} = (2k+1) x P_k - k P_{k-1}."""
    x = np.asarray(x, dtype=np.float64)
    p0 = np.ones_like(x)
    if p == 0:
        return p0
    p1 = x.copy()
    for k in range(1, p):
        p0, p1 = p1, ((2 * k + 1) * x * p1 - k * p0) / (k + 1)
    return p1


def legendre_deriv(p, x):
    """P_p'(x) from P_p' = p (x P_p - P_{p-1}) / (x^2 - 1), valid for |x| < 1."""
    x = np.asarray(x, dtype=np.float64)
    return p * (x * legendre(p, x) - legendre(p - 1, x)) / (x * x - 1.0)


def gll_nodes_weights(p):
    """Return (xi, w), the p+1 GLL nodes in increasing order and their weights."""
    if p < 1:
        raise ValueError("GLL needs p >= 1")
    xi = np.empty(p + 1)
    xi[0], xi[p] = -1.0, 1.0
    if p > 1:
        # interior nodes: Newton on f = P_p'.  From Legendre's equation
        # (1-x^2) P'' = 2 x P' - p(p+1) P, so f' = (2 x P' - p(p+1) P)/(1-x^2).
        x = -np.cos(np.pi * np.arange(1, p) / p)
        for _ in range(100):
            dp = legendre_deriv(p, x)
            d2p = (2 * x * dp - p * (p + 1) * legendre(p, x)) / (1 - x * x)
            step = dp / d2p
            x = x - step
            if np.max(np.abs(step)) < 1e-16:
                break
        xi[1:p] = np.sort(x)
    w = 2.0 / (p * (p + 1) * legendre(p, xi) ** 2)
    return xi, w


def lagrange_matrix(xi, x):
    """J[i, j] = h_j(x_i): cardinal polynomial on nodes xi evaluated at x.

    Product formula h_j(x) = prod_{m != j} (x - xi_m) / (xi_j - xi_m).
    """
    xi = np.asarray(xi, dtype=np.float64)
    x = np.asarray(x, dtype=np.float64)
    n = len(xi)
    J = np.ones((len(x), n))
    for j in range(n):
        for m in range(n):
            if m != j:
                J[:, j] *= (x - xi[m]) / (xi[j] - xi[m])
    return J


def derivative_matrix(xi):
    """Dhat[i, j] = h_j'(xi_i) by differentiating the product formula.

    h_j'(x) = sum_{m != j} 1/(xi_j - xi_m) prod_{l != j, m} (x - xi_l)/(xi_j - xi_l)
    """
    xi = np.asarray(xi, dtype=np.float64)
    n = len(xi)
    D = np.zeros((n, n))
    for i in range(n):
        for j in range(n):
            s = 0.0
            for m in range(n):
                if m == j:
                    continue
                t = 1.0 / (xi[j] - xi[m])
                for l in range(n):
                    if l != j and l != m:
                        t *= (xi[i] - xi[l]) / (xi[j] - xi[l])
                s += t
            D[i, j] = s
    return D


def gll(p):
    """Convenience bundle: nodes, weights and Dhat for degree p."""
    xi, w = gll_nodes_weights(p)
    return xi, w, derivative_matrix(xi)


def interpolation(p_from, p_to):
    """J[i, j] = h^{p_from}_j(xi^{p_to}_i), shape (p_to+1, p_from+1)."""
    xf, _ = gll_nodes_weights(p_from)
    xt, _ = gll_nodes_weights(p_to)
    return lagrange_matrix(xf, xt)
