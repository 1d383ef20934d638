"""p-multigrid transfers and the single-pass V-cycle (oracle, test-only).

Sec. 2.2.2, Algorithm 1 (x = 0 on entry when used as a preconditioner):

    x = x + M(b - A x)          smooth
    r = b - A x                 re-evaluate residual
    r_C = P^T r                 coarsen
    e_C = A_C^{-1} r_C          coarse solve, or recurse
    x = x + P e_C               prolongate and update
    x = x + M(b - A x)          post-smooth

Readings: the coarse operator A_C is the SE operator rediscretised at the
coarse degree on the same geometry (not the Galerkin product P^T A P), so
each level carries its own G; P interpolates the coarse cardinal basis to
the fine GLL nodes element by element (J (x) J (x) J with
J[i, j] = h^c_j(xi^f_i)), and P^T is its exact transpose on global vectors:
divide the consistent fine E-vector by the fine multiplicity, contract with
J^T (x) J^T (x) J^T, then assemble (QQ^T) and mask on the coarse level.
"""
import numpy as np


def prolong(J, ec):
    """Fine E-vector P e_c from a coarse E-vector (J[Nf, Nc])."""
    return np.einsum('kc,jb,ia,ecba->ekji', J, J, J, ec)


def restrict(num_f, num_c, J, rf):
    """Coarse E-vector P^T r_f (masked, consistent copies)."""
    t = rf / num_f.Q(num_f.mult)
    rc = np.einsum('kc,jb,ia,ekji->ecba', J, J, J, t)
    return num_c.mask * num_c.QQt(rc)


def vcycle(levels, b, coarse_solve, level=0):
    """One V-cycle of Algorithm 1 from x = 0 on level `level`.

    levels[l] provides .apply_A(u), .smooth(b, x) -> correction, and
    .J_to_coarse (interpolation from level l+1 to l); coarse_solve(b) solves
    on the last level.
    """
    if level == len(levels) - 1:
        return coarse_solve(b)
    L, C = levels[level], levels[level + 1]
    x = L.smooth(b, None)
    r = b - L.apply_A(x)
    rc = restrict(L.num, C.num, L.J_to_coarse, r)
    ec = vcycle(levels, rc, coarse_solve, level + 1)
    x = x + prolong(L.J_to_coarse, ec)
    x = x + L.smooth(b, x)
    return x


def vcycle_additive(levels, b, coarse_solve, level=0):
    """V-cycle for smoothers without Chebyshev acceleration (Sec. 2.2.2): the
    smoother and the coarse-grid correction act on the same right side and are
    added, with no residual re-evaluation and no post-smoothing:
    x = S_l b + P_l V_{l+1}(P_l^T b), the coarsest level solved."""
    if level == len(levels) - 1:
        return coarse_solve(b)
    L, C = levels[level], levels[level + 1]
    x = L.apply_S(b)
    bc = restrict(L.num, C.num, L.J_to_coarse, b)
    ec = vcycle_additive(levels, bc, coarse_solve, level + 1)
    return x + prolong(L.J_to_coarse, ec)
