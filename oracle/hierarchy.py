"""A pMG-preconditioned SE Poisson solver assembled from the oracle parts (test-only).

Ties the modules together the way Sec. 2.2 uses them: per level of the
schedule (p_0 > p_1 > ... > p_L), the operator (geom + operator), a surrogate
smoother (Jacobi or Schwarz, fdm), Chebyshev bounds from Arnoldi (cheby), and
the transfers to the next level (mg); the last level is solved by Jacobi-PCG
(the paper uses one BoomerAMG V-cycle there; this project's reading replaces
it by Jacobi-PCG to a relative tolerance, or a dense solve for pins).
"""
import numpy as np

from . import cheby as _cheby
from . import gll as _gll
from . import krylov as _krylov
from . import mg as _mg
from .fdm import FDM
from .geom import geometric_factors
from .mesh import Numbering, level_coordinates
from .operator import apply_A, jacobi_inverse, rhs, dense_free_system
from .rng import uniform_pm1


class Level:
    def __init__(self, nex, ney, nez, xyz, p_geom, p, bc, smoother):
        self.p = p
        self.num = Numbering(nex, ney, nez, p, bc)
        self.X = level_coordinates(xyz, p_geom, p)
        self.G, self.BL, self.detJ = geometric_factors(self.X, p)
        self.dinv = jacobi_inverse(self.num, self.G)
        self.smoother = smoother
        self.fdm = FDM(self.num, self.X) if smoother in ('ras', 'asm') else None
        self.lmin = self.lmax = None
        self.K = 0
        self.J_to_coarse = None
        self.lam_tilde = None

    def apply_A(self, u):
        return apply_A(self.num, self.G, u)

    def apply_S(self, r):
        if self.smoother == 'jacobi':
            return self.dinv * r
        if self.smoother == 'ras':
            return self.fdm.apply_ras(r)
        if self.smoother == 'asm':
            return self.fdm.apply_asm(r)
        raise ValueError(self.smoother)

    def smooth(self, b, x):
        """Chebyshev correction e (Algorithm 2); the caller adds it to x."""
        return _cheby.chebyshev(self.apply_A, self.apply_S, b, x, self.lmin, self.lmax, self.K)

    def wdot(self, a, b):
        return self.num.wdot(a, b)


class Solver:
    """Oracle counterpart of the library's setup / apply_A / smooth / vcycle / solve."""

    def __init__(self, nex, ney, nez, xyz, p_geom, schedule, bc=(1, 1, 1, 1, 1, 1),
                 smoother='jacobi', cheb_order=2, lmin_fac=0.1, lmax_fac=1.1,
                 arnoldi_steps=10, seed=0, lambda_override=None,
                 coarse_tol=1e-10, coarse_maxit=2000, coarse='pcg'):
        self.schedule = list(schedule)
        self.levels = []
        for l, p in enumerate(self.schedule):
            last = l == len(self.schedule) - 1
            self.levels.append(Level(nex, ney, nez, xyz, p_geom, p, bc,
                                     'jacobi' if last else smoother))
        for l in range(len(self.levels) - 1):
            self.levels[l].J_to_coarse = _gll.interpolation(self.schedule[l + 1], self.schedule[l])
        self.coarse_tol, self.coarse_maxit, self.coarse = coarse_tol, coarse_maxit, coarse
        self.cheb_order = cheb_order
        self.seed = seed
        for l, L in enumerate(self.levels[:-1]):
            L.K = cheb_order
            if lambda_override is not None and lambda_override[l] > 0:
                lt = float(lambda_override[l])
            else:
                lt = self.arnoldi_lambda(l, arnoldi_steps)
            L.lam_tilde = lt
            L.lmin, L.lmax = _cheby.bounds(lt, lmin_fac, lmax_fac)
        self._dense = None

    @property
    def fine(self):
        return self.levels[0]

    def start_vector(self, l):
        L = self.levels[l]
        v = L.num.Q(uniform_pm1(self.seed, np.arange(L.num.n)))
        return L.num.mask * v

    def arnoldi_lambda(self, l, steps):
        L = self.levels[l]
        H, V, k = _cheby.arnoldi(lambda v: L.apply_S(L.apply_A(v)), self.start_vector(l),
                                 L.wdot, steps)
        return _cheby.lambda_tilde(H, k)

    # --- ABI counterparts ------------------------------------------------
    def rhs(self, f_local):
        return rhs(self.fine.num, self.fine.BL, f_local)

    def apply_A(self, u, level=0):
        return self.levels[level].apply_A(u)

    def smooth(self, b, x, level=0):
        """x + Cheb(b - A x) on `level` (x=None means zero)."""
        e = self.levels[level].smooth(b, x)
        return e if x is None else x + e

    def coarse_solve(self, b):
        L = self.levels[-1]
        if self.coarse == 'dense':
            if self._dense is None:
                self._dense = dense_free_system(L.num, L.G)
            A, free = self._dense
            bg = L.num.to_global(b)
            xg = np.zeros(L.num.n)
            xg[free] = np.linalg.solve(A, bg[free])
            return L.num.Q(xg)
        res = _krylov.pcg(L.apply_A, lambda r: L.dinv * r, b, L.wdot,
                          self.coarse_tol, self.coarse_maxit)
        return res.x

    def vcycle(self, r):
        if self.cheb_order == 0:  # smoothers without acceleration: additive cycle
            return _mg.vcycle_additive(self.levels, r, self.coarse_solve)
        return _mg.vcycle(self.levels, r, self.coarse_solve)

    def solve(self, b, tol=1e-8, maxit=500, krylov='fcg', x0=None, restart=20):
        A, M, wdot = self.fine.apply_A, self.vcycle, self.fine.wdot
        if krylov == 'pcg':
            return _krylov.pcg(A, M, b, wdot, tol, maxit, x0)
        if krylov == 'fcg':
            return _krylov.fcg(A, M, b, wdot, tol, maxit, x0)
        if krylov == 'fgmres':
            return _krylov.fgmres(A, M, b, wdot, tol, maxit, restart, x0)
        raise ValueError(krylov)

    def jacobi_pcg(self, b, tol, maxit):
        """Plain Jacobi-PCG on the finest level (no multigrid)."""
        L = self.fine
        return _krylov.pcg(L.apply_A, lambda r: L.dinv * r, b, L.wdot, tol, maxit)
