"""The SE Poisson operator A = Q^T A_L Q and its pieces (oracle, test-only).

Sec. 2.1, eq. 3 and the sum-factorisation remark: A^e is never formed;
A^e u = sum_{b,c} D_b^T G_bc D_c u with D_r = I x I x Dhat, D_s = I x Dhat x I,
D_t = Dhat x I x I, each applied as a 1D contraction.

On E-vectors (consistent copies on shared nodes), the assembled product is
A u  ->  mask * QQ^T (A_L u_L), which equals Q (Q^T A_L Q) u on the free nodes.
"""
import numpy as np

from . import gll as _gll
from .geom import reference_gradient

_PAIRS = ((0, 0), (0, 1), (0, 2), (1, 1), (1, 2), (2, 2))


def G_full(G):
    """Expand the 6 unique entries into a 3x3 list-of-lists view."""
    Gf = [[None] * 3 for _ in range(3)]
    for c, (a, b) in enumerate(_PAIRS):
        Gf[a][b] = G[c]
        Gf[b][a] = G[c]
    return Gf


def apply_AL(G, p, u):
    """v = A_L u, elementwise sum factorisation (local, unassembled)."""
    _, _, D = _gll.gll(p)
    g = reference_gradient(D, u)
    Gf = G_full(G)
    w = [sum(Gf[a][b] * g[b] for b in range(3)) for a in range(3)]
    v = np.einsum('li,ekjl->ekji', D, w[0])
    v += np.einsum('mj,ekmi->ekji', D, w[1])
    v += np.einsum('nk,enji->ekji', D, w[2])
    return v


def apply_A(num, G, u):
    """A u on a consistent E-vector: mask * QQ^T A_L u."""
    return num.mask * num.QQt(apply_AL(G, num.p, u))


def rhs(num, BL, f_local):
    """b = mask * QQ^T (B_L f), the right side B f of eq. 3 on E-vectors."""
    return num.mask * num.QQt(BL * f_local)


def local_diagonal(G, p):
    """diag(A^e) from the definition A^e_qq = sum_q' sum_bc (D_b)_{q'q} G_bc(q') (D_c)_{q'q}.

    Only q' on the same r-, s- or t-line as q contributes; the cross terms
    (b != c) survive only at q' = q.
    """
    _, _, D = _gll.gll(p)
    D2 = D * D
    d = np.einsum('li,ekjl->ekji', D2, G[0])  # rr: sum over l of D[l,i]^2 G_rr(l,j,k)
    d += np.einsum('mj,ekmi->ekji', D2, G[3])            # ss
    d += np.einsum('nk,enji->ekji', D2, G[5])            # tt
    dd = np.diag(D)
    di = dd[None, None, None, :]
    dj = dd[None, None, :, None]
    dk = dd[None, :, None, None]
    d += 2 * di * dj * G[1] + 2 * di * dk * G[2] + 2 * dj * dk * G[4]
    return d


def assembled_diagonal(num, G):
    """diag(A) on E-vectors (mask * QQ^T diag(A_L)); zero on Dirichlet nodes."""
    return num.mask * num.QQt(local_diagonal(G, num.p))


def jacobi_inverse(num, G):
    """Jacobi surrogate S = diag(A)^{-1} (Sec. 2.2.3), zero on Dirichlet nodes."""
    d = assembled_diagonal(num, G)
    out = np.zeros_like(d)
    np.divide(1.0, d, out=out, where=num.mask > 0)
    return out


# --- dense brute force (tiny meshes only) -----------------------------------
def element_matrix(G, p, e):
    """Dense A^e = sum_bc D_b^T diag(G_bc) D_c, built from Kronecker products."""
    _, _, D = _gll.gll(p)
    N = p + 1
    I = np.eye(N)
    Db = [np.kron(I, np.kron(I, D)), np.kron(I, np.kron(D, I)), np.kron(D, np.kron(I, I))]
    Gf = G_full(G)
    Ae = np.zeros((N ** 3, N ** 3))
    for a in range(3):
        for b in range(3):
            Ae += Db[a].T @ (Gf[a][b][e].reshape(-1)[:, None] * Db[b])
    return Ae


def dense_global_A(num, G):
    """A = Q^T A_L Q assembled densely (no mask): [n, n]."""
    A = np.zeros((num.n, num.n))
    for e in range(num.E):
        idx = num.gid[e].reshape(-1)
        A[np.ix_(idx, idx)] += element_matrix(G, num.p, e)
    return A


def dense_free_system(num, G):
    """(A_ff, free indices): A restricted to the non-Dirichlet global nodes."""
    A = dense_global_A(num, G)
    free = np.nonzero(num.mask_global > 0)[0]
    return A[np.ix_(free, free)], free
