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
