"""Geometric factors of the isoparametric map (oracle, test-only).

Sec. 2.1: x^e(r,s,t) = sum x^e_ijk h_i(r) h_j(s) h_k(t), and the stiffness
entries are A_ij = (grad phi_i, grad phi_j)_p with GLL quadrature.  Pulled
back to the reference element,

    (grad v, grad u)_p = sum_q w_q det(J_q) (J_q^{-T} grad_r v) . (J_q^{-T} grad_r u)
                       = sum_q (grad_r v)^T G_q (grad_r u),
    G_q = w_q det(J_q) J_q^{-1} J_q^{-T},   (3x3 symmetric, 6 unique entries)

with J_q[a, b] = d x_a / d r_b and w_q = w_i w_j w_k.  The diagonal mass is
B_L = w_q det(J_q) (coincident GLL quadrature and nodal points).

G is returned as [6, E, N, N, N] in the order (rr, rs, rt, ss, st, tt).
"""
import numpy as np

from . import gll as _gll


def reference_gradient(D, u):
    """(du/dr, du/ds, du/dt) of an element field u[e, k, j, i]."""
    ur = np.einsum('il,ekjl->ekji', D, u)
    us = np.einsum('jm,ekmi->ekji', D, u)
    ut = np.einsum('kn,enji->ekji', D, u)
    return ur, us, ut


def jacobian(X, p):
    """Jm[e,k,j,i,a,b] = d x_a / d r_b at the level's GLL nodes."""
    _, _, D = _gll.gll(p)
    E, N = X.shape[1], X.shape[2]
    Jm = np.empty((E, N, N, N, 3, 3))
    for a in range(3):
        g = reference_gradient(D, X[a])
        for b in range(3):
            Jm[..., a, b] = g[b]
    return Jm


def geometric_factors(X, p):
    """Return (G[6,E,N,N,N], B_L[E,N,N,N], detJ[E,N,N,N])."""
    _, w, _ = _gll.gll(p)
    Jm = jacobian(X, p)
    detJ = np.linalg.det(Jm)
    Jinv = np.linalg.inv(Jm)  # Jinv[..., b, a] = d r_b / d x_a
    wq = w[None, :, None, None] * w[None, None, :, None] * w[None, None, None, :]
    M = np.einsum('...ba,...ca->...bc', Jinv, Jinv)  # J^{-1} J^{-T}
    scale = wq * detJ
    G = np.empty((6,) + detJ.shape)
    for c, (a, b) in enumerate(((0, 0), (0, 1), (0, 2), (1, 1), (1, 2), (2, 2))):
        G[c] = scale * M[..., a, b]
    return G, scale, detJ
