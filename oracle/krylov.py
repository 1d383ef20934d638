"""Krylov solvers (oracle, test-only).

Sec. 2.2: preconditioners are applied inside restarted GMRES or flexible CG
(FCG).  Readings (the paper names but does not define the variants):
  * pcg: textbook preconditioned CG (fixed SPD preconditioner);
  * fcg: flexible CG with truncation 1 (Polak-Ribiere form),
    beta_k = r_{k+1}.(z_{k+1} - z_k) / (r_k.z_k);
  * fgmres: right-preconditioned flexible GMRES(m); here the small
    least-squares problem is solved directly with lstsq at every step.
CG variants also stop on exact breakdown (p.Ap = 0, so p = 0 and the iterate
is final).  All stop when ||r_k|| / ||r_0|| <= tol (2-norm over unique free nodes, i.e.
E-vector dots weighted by mask/mult).  On exit the true residual b - A x is
recomputed; if it fails the test the iteration restarts from it.
"""
import numpy as np


class Result:
    def __init__(self, x, iters, rel, history, converged):
        self.x, self.iters, self.rel, self.history, self.converged = x, iters, rel, history, converged


def pcg(apply_A, apply_M, b, wdot, tol, maxit, x0=None):
    x = np.zeros_like(b) if x0 is None else x0.copy()
    r = b - apply_A(x) if x0 is not None else b.copy()
    r0 = np.sqrt(wdot(r, r))
    hist = [1.0]
    if r0 == 0.0:
        return Result(x, 0, 0.0, hist, True)
    it = 0
    rel = 1.0
    while it < maxit:
        z = apply_M(r)
        p = z.copy()
        rz = wdot(r, z)
        while it < maxit:
            q = apply_A(p)
            pq = wdot(p, q)
            if not pq > 0.0:  # exact breakdown (p = 0): the iterate is final
                r = b - apply_A(x)
                rel = np.sqrt(wdot(r, r)) / r0
                return Result(x, it, rel, hist, rel <= tol)
            alpha = rz / pq
            x = x + alpha * p
            r = r - alpha * q
            it += 1
            rel = np.sqrt(wdot(r, r)) / r0
            hist.append(rel)
            if rel <= tol:
                break
            z = apply_M(r)
            rz_new = wdot(r, z)
            p = z + (rz_new / rz) * p
            rz = rz_new
        r = b - apply_A(x)
        rel = np.sqrt(wdot(r, r)) / r0
        if rel <= tol:
            return Result(x, it, rel, hist, True)
    return Result(x, it, rel, hist, False)


def fcg(apply_A, apply_M, b, wdot, tol, maxit, x0=None):
    x = np.zeros_like(b) if x0 is None else x0.copy()
    r = b - apply_A(x) if x0 is not None else b.copy()
    r0 = np.sqrt(wdot(r, r))
    hist = [1.0]
    if r0 == 0.0:
        return Result(x, 0, 0.0, hist, True)
    it = 0
    rel = 1.0
    while it < maxit:
        z = apply_M(r)
        p = z.copy()
        rz = wdot(r, z)
        while it < maxit:
            q = apply_A(p)
            pq = wdot(p, q)
            if not pq > 0.0:  # exact breakdown (p = 0): the iterate is final
                r = b - apply_A(x)
                rel = np.sqrt(wdot(r, r)) / r0
                return Result(x, it, rel, hist, rel <= tol)
            alpha = rz / pq
            x = x + alpha * p
            r = r - alpha * q
            it += 1
            rel = np.sqrt(wdot(r, r)) / r0
            hist.append(rel)
            if rel <= tol:
                break
            z_old = z
            z = apply_M(r)
            rz_new = wdot(r, z)
            beta = (rz_new - wdot(r, z_old)) / rz
            p = z + beta * p
            rz = rz_new
        r = b - apply_A(x)
        rel = np.sqrt(wdot(r, r)) / r0
        if rel <= tol:
            return Result(x, it, rel, hist, True)
    return Result(x, it, rel, hist, False)


def fgmres(apply_A, apply_M, b, wdot, tol, maxit, m=20, x0=None):
    x = np.zeros_like(b) if x0 is None else x0.copy()
    r = b - apply_A(x) if x0 is not None else b.copy()
    r0 = np.sqrt(wdot(r, r))
    hist = [1.0]
    if r0 == 0.0:
        return Result(x, 0, 0.0, hist, True)
    it = 0
    rel = 1.0
    while it < maxit:
        beta = np.sqrt(wdot(r, r))
        V = [r / beta]
        Z = []
        H = np.zeros((m + 1, m))
        y = np.zeros(0)
        for j in range(m):
            Z.append(apply_M(V[j]))
            w = apply_A(Z[j])
            for i in range(j + 1):
                H[i, j] = wdot(V[i], w)
                w = w - H[i, j] * V[i]
            H[j + 1, j] = np.sqrt(wdot(w, w))
            it += 1
            rhs = np.zeros(j + 2)
            rhs[0] = beta
            y = np.linalg.lstsq(H[:j + 2, :j + 1], rhs, rcond=None)[0]
            rel = np.linalg.norm(rhs - H[:j + 2, :j + 1] @ y) / r0
            hist.append(rel)
            if rel <= tol or it >= maxit or H[j + 1, j] == 0.0:
                break
            V.append(w / H[j + 1, j])
        x = x + sum(yi * zi for yi, zi in zip(y, Z))
        r = b - apply_A(x)
        rel = np.sqrt(wdot(r, r)) / r0
        if rel <= tol:
            return Result(x, it, rel, hist, True)
    return Result(x, it, rel, hist, False)


class Projection:
    """Initial guesses for successive right-hand sides (Sec. 3.2 and 4.2: the
    solution is projected onto up to 10 prior solution vectors).  Reading: the
    basis X is A-orthonormal in the weighted (unique free node) inner product,
    (x_i, A x_j) = delta_ij, with A X kept beside it, so the guess
    x0 = sum_i (x_i, b) x_i is the A-norm best approximation of A^{-1} b in
    span(X).  After a solve the correction x - x0 is A-orthogonalised against
    X by classical Gram-Schmidt (two passes) and appended when it adds a new
    direction (A-norm above 1e-10 of its value before orthogonalisation); a
    full basis restarts from the latest solution alone."""

    def __init__(self, apply_A, wdot, lmax):
        self.apply_A, self.wdot, self.lmax = apply_A, wdot, lmax
        self.X, self.AX = [], []

    def guess(self, b):
        x0 = np.zeros_like(b)
        for xi in self.X:
            x0 = x0 + self.wdot(xi, b) * xi
        return x0

    def update(self, x0, x):
        if len(self.X) == self.lmax:
            self.X, self.AX = [], []
            w = x.copy()
        else:
            w = x - x0
        Aw = self.apply_A(w)
        n0 = self.wdot(w, Aw)
        for _ in range(2):
            if not self.X:
                break
            beta = [self.wdot(xi, Aw) for xi in self.X]
            for bi, xi, axi in zip(beta, self.X, self.AX):
                w = w - bi * xi
                Aw = Aw - bi * axi
        nn = self.wdot(w, Aw)
        if nn > 0.0 and nn > 1e-20 * n0:
            s = 1.0 / np.sqrt(nn)
            self.X.append(w * s)
            self.AX.append(Aw * s)


def projected_solve(solver, proj, apply_A, apply_M, b, wdot, tol, maxit, **kw):
    """solver (pcg, fcg or fgmres) from the projected guess, stopping at
    ||b - A x|| <= tol ||b||; the basis is updated afterwards.  Result.rel is
    relative to ||b||."""
    nb = np.sqrt(wdot(b, b))
    x0 = proj.guess(b)
    r = b - apply_A(x0)
    r0 = np.sqrt(wdot(r, r))
    if r0 == 0.0 or r0 <= tol * nb:
        res = Result(x0, 0, r0 / nb if nb > 0 else 0.0, [r0 / nb if nb > 0 else 0.0], True)
    else:
        res = solver(apply_A, apply_M, b, wdot, tol * nb / r0, maxit, x0=x0, **kw)
        res.rel = res.rel * r0 / nb
    proj.update(x0, res.x)
    return res
