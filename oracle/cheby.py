"""Chebyshev-accelerated smoothing and the Arnoldi spectral proxy (oracle, test-only).

Sec. 2.2.3, Algorithm 2, for a surrogate smoother S (Jacobi or Schwarz):

    theta = (lmax + lmin)/2, delta = (lmax - lmin)/2, sigma = theta/delta, rho_1 = 1/sigma
    r = S(b - A x), d_1 = r/theta, x_1 = 0
    for k = 1..K:   x_{k+1} = x_k + d_k
                    r_{k+1} = r_k - S A d_k
                    rho_{k+1} = 1/(2 sigma - rho_k)
                    d_{k+1} = rho_{k+1} rho_k d_k + (2 rho_{k+1}/delta) r_{k+1}
    x_{K+2} = x_{K+1} + d_{K+1}

Reading: the algorithm accumulates from x_1 = 0 while r uses the caller's x,
so the accumulated sum is the correction e and the caller's iterate becomes
x + e (as in Algorithm 1, x = x + M(b - Ax)).  Order K means K loop passes:
K products with A, K+1 with S.

The bounds come from 10 Arnoldi steps on S A, lambda~ = largest Ritz value
magnitude, and (lmin, lmax) = (0.1, 1.1) lambda~ (Sec. 2.2.3).  Readings: the
start vector is U(-1,1) per global node from SplitMix64(seed XOR gid),
Dirichlet-masked and normalised; inner products are over unique free nodes;
the iteration stops early when h_{k+1,k} <= 1e-14 max|H| (invariant subspace).
"""
import numpy as np


def chebyshev(apply_A, apply_S, b, x, lmin, lmax, K):
    """Return the correction e of Algorithm 2 (x is None means x = 0).

    K = 0 reads as the smoother without Chebyshev acceleration (Sec. 2.2.2):
    e = S (b - A x), undamped."""
    r = apply_S(b if x is None else b - apply_A(x))
    if K == 0:
        return r
    theta = 0.5 * (lmax + lmin)
    delta = 0.5 * (lmax - lmin)
    sigma = theta / delta
    rho = 1.0 / sigma
    d = r / theta
    e = np.zeros_like(b)
    for _ in range(K):
        e = e + d
        r = r - apply_S(apply_A(d))
        rho_new = 1.0 / (2.0 * sigma - rho)
        d = rho_new * rho * d + (2.0 * rho_new / delta) * r
        rho = rho_new
    return e + d


def arnoldi(apply_SA, v0, wdot, m=10):
    """m steps of Arnoldi (modified Gram-Schmidt) on S A.

    Returns (H[k+1, k], V list, k) where k <= m is the number of steps taken.
    """
    V = [v0 / np.sqrt(wdot(v0, v0))]
    H = np.zeros((m + 1, m))
    k = 0
    for j in range(m):
        w = apply_SA(V[j])
        for i in range(j + 1):
            H[i, j] = wdot(V[i], w)
            w = w - H[i, j] * V[i]
        H[j + 1, j] = np.sqrt(wdot(w, w))
        k = j + 1
        if H[j + 1, j] <= 1e-14 * np.max(np.abs(H[:j + 2, :j + 1])):
            break
        V.append(w / H[j + 1, j])
    return H[:k + 1, :k], V, k


def lambda_tilde(H, k):
    """Largest magnitude Ritz value of the k x k Hessenberg block."""
    return float(np.max(np.abs(np.linalg.eigvals(H[:k, :k]))))


def bounds(lam_tilde, lmin_fac=0.1, lmax_fac=1.1):
    """(lmin, lmax) = (0.1, 1.1) lambda~ by default."""
    return lmin_fac * lam_tilde, lmax_fac * lam_tilde
