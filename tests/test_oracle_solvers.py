"""Pins of the oracle's Chebyshev, Arnoldi, transfers, V-cycle and Krylov solvers (CPU only).

Sec. 2.2 (Krylov), 2.2.2 (Algorithm 1), 2.2.3 (Algorithm 2, Arnoldi bounds).
"""
import numpy as np
import pytest

from oracle import cheby, gll, mg
from oracle.hierarchy import Solver
from oracle.mesh import Numbering, level_coordinates
from oracle.operator import dense_free_system
from paper_2110_07663_amd import workloads as wl


def chebT(n, x):
    return np.cosh(n * np.arccosh(x)) if x >= 1 else np.cos(n * np.arccos(x)) if abs(x) <= 1 \
        else (-1) ** n * np.cosh(n * np.arccosh(-x))


@pytest.mark.parametrize("K", [1, 2, 3, 4])
def test_chebyshev_error_polynomial_closed_form(K):
    """With S = I and A = diag(lam): 1 - lam q(lam) = T_{K+1}((theta-lam)/delta) / T_{K+1}(theta/delta)."""
    lmin, lmax = 0.3, 2.0
    theta, delta = (lmax + lmin) / 2, (lmax - lmin) / 2
    lam = np.concatenate([np.linspace(lmin, lmax, 17), [0.05, 0.1]])
    e = cheby.chebyshev(lambda v: lam * v, lambda v: v, lam * 1.0, None, lmin, lmax, K)
    ref = np.array([chebT(K + 1, (theta - l) / delta) for l in lam]) / chebT(K + 1, theta / delta)
    np.testing.assert_allclose(1.0 - e, ref, atol=1e-13)
    # with an initial guess the correction is applied to the current error
    x0 = np.full_like(lam, 0.25)
    e2 = cheby.chebyshev(lambda v: lam * v, lambda v: v, lam * 1.0, x0, lmin, lmax, K)
    np.testing.assert_allclose(1.0 - (x0 + e2), 0.75 * ref, atol=1e-13)


def _small_solver(p_sched, smoother="jacobi", coarse="dense", n=2, lam=None, **kw):
    pf = p_sched[0]
    xi, _ = gll.gll_nodes_weights(pf)
    xyz = wl.sampled_mesh(n, n, n, xi, wl.sin_map(0.05))
    return Solver(n, n, n, xyz, pf, p_sched, smoother=smoother, coarse=coarse,
                  lambda_override=lam, **kw)


def _dense_operator(S, level=0):
    L = S.levels[level]
    A, free = dense_free_system(L.num, L.G)
    return A, free


def test_arnoldi_bounds_jacobi():
    S = _small_solver([4, 1])
    L = S.levels[0]
    A, free = _dense_operator(S)
    d = np.diag(A)
    lmax = np.max(np.linalg.eigvals(A / d[:, None]).real)
    H, V, k = cheby.arnoldi(lambda v: L.apply_S(L.apply_A(v)), S.start_vector(0), L.wdot, 10)
    lt = cheby.lambda_tilde(H, k)
    assert lt <= lmax * (1 + 1e-12)
    assert lt > 0.9 * lmax
    assert abs(lt - S.levels[0].lam_tilde) < 1e-12 * lt
    # orthonormal basis, Hessenberg structure
    G = np.array([[L.wdot(a, b) for b in V] for a in V])
    np.testing.assert_allclose(G, np.eye(len(V)), atol=1e-12)
    assert np.all(np.tril(H, -2) == 0)


def test_arnoldi_bounds_ras_real_dominant():
    S = _small_solver([5, 1], smoother="ras")
    L = S.levels[0]
    A, free = _dense_operator(S)
    # dense S*A on the free nodes via unit vectors
    n = L.num
    cols = []
    for g in free:
        u = np.zeros(n.n)
        u[g] = 1
        cols.append(n.to_global(L.apply_S(L.apply_A(n.Q(u))))[free])
    SA = np.array(cols).T
    rho = np.max(np.abs(np.linalg.eigvals(SA)))
    assert S.levels[0].lam_tilde <= rho * (1 + 1e-10)
    assert S.levels[0].lam_tilde > 0.8 * rho


@pytest.mark.parametrize("pc,pf", [(1, 3), (3, 7), (3, 5)])
def test_transfer_adjoint_and_exactness(pc, pf):
    n = 2
    xyz = wl.layer_shift_vertices(n, seed=4)
    nf, nc = Numbering(n, n, n, pf), Numbering(n, n, n, pc)
    J = gll.interpolation(pc, pf)
    r = np.random.default_rng(0)
    ec = nc.mask * nc.Q(r.standard_normal(nc.n))
    rf = nf.mask * nf.Q(r.standard_normal(nf.n))
    lhs = np.dot(nf.to_global(mg.prolong(J, ec)), nf.to_global(rf))
    rhs = np.dot(nc.to_global(ec), nc.to_global(mg.restrict(nf, nc, J, rf)))
    assert abs(lhs - rhs) < 1e-13 * abs(lhs)
    # coarse coordinate fields (trilinear mesh) are reproduced exactly
    Xc = level_coordinates(xyz, 1, pc)
    Xf = level_coordinates(xyz, 1, pf)
    for a in range(3):
        np.testing.assert_allclose(mg.prolong(J, Xc[a]), Xf[a], atol=1e-14)


@pytest.mark.parametrize("smoother", ["jacobi", "ras"])
def test_vcycle_same_degree_schedule_is_exact_solve(smoother):
    """Schedule (p, p): P = I, A_C = A, exact coarse solve -> V-cycle returns A^{-1} r."""
    S = _small_solver([4, 4], smoother=smoother, lam=[3.0, 0])
    L = S.levels[0]
    A, free = _dense_operator(S)
    r = L.num.mask * L.num.Q(np.random.default_rng(2).standard_normal(L.num.n))
    z = S.vcycle(r)
    ref = np.zeros(L.num.n)
    ref[free] = np.linalg.solve(A, L.num.to_global(r)[free])
    np.testing.assert_allclose(L.num.to_global(z), ref, atol=1e-11 * np.abs(ref).max())


@pytest.mark.parametrize("smoother", ["jacobi", "ras", "asm"])
def test_two_level_vcycle_contracts(smoother):
    S = _small_solver([3, 1], smoother=smoother)
    L = S.levels[0]
    A, free = _dense_operator(S)
    cols = []
    for g in free:
        u = np.zeros(L.num.n)
        u[g] = 1
        cols.append(L.num.to_global(S.vcycle(L.num.Q(u)))[free])
    M = np.array(cols).T
    rho = np.max(np.abs(np.linalg.eigvals(np.eye(len(free)) - M @ A)))
    assert rho < 0.5, rho


@pytest.mark.parametrize("krylov", ["pcg", "fcg", "fgmres"])
def test_krylov_matches_dense_solve(krylov):
    S = _small_solver([5, 3, 1], smoother="ras", coarse="pcg")
    L = S.fine
    A, free = _dense_operator(S)
    f, _ = wl.sinusoid(1, 2, 1)
    b = S.rhs(f(L.X[0], L.X[1], L.X[2]))
    res = S.solve(b, tol=1e-13, maxit=200, krylov=krylov)
    assert res.converged
    ref = np.zeros(L.num.n)
    ref[free] = np.linalg.solve(A, L.num.to_global(b)[free])
    np.testing.assert_allclose(L.num.to_global(res.x), ref, atol=1e-11 * np.abs(ref).max())


def test_jacobi_pcg_matches_dense_solve():
    S = _small_solver([3, 1])
    L = S.fine
    A, free = _dense_operator(S)
    b = L.num.mask * L.num.Q(np.random.default_rng(5).standard_normal(L.num.n))
    res = S.jacobi_pcg(b, 1e-13, 500)
    ref = np.zeros(L.num.n)
    ref[free] = np.linalg.solve(A, L.num.to_global(b)[free])
    np.testing.assert_allclose(L.num.to_global(res.x), ref, atol=1e-11 * np.abs(ref).max())


def test_chebyshev_bounds_sensitivity_underestimate_hurts():
    """Underestimating lambda_max costs iterations (Sec. 2.2.3, Table 1 trend)."""
    S_good = _small_solver([5, 3, 1], smoother="jacobi", coarse="pcg", n=3)
    lt = [L.lam_tilde for L in S_good.levels[:-1]] + [0]
    S_bad = _small_solver([5, 3, 1], smoother="jacobi", coarse="pcg", n=3,
                          lam=lt, lmin_fac=0.1, lmax_fac=0.5)
    L = S_good.fine
    f, _ = wl.sinusoid(1, 1, 1)
    b = S_good.rhs(f(L.X[0], L.X[1], L.X[2]))
    it_good = S_good.solve(b, tol=1e-8, maxit=300).iters
    it_bad = S_bad.solve(b, tol=1e-8, maxit=300).iters
    assert it_bad > it_good, (it_good, it_bad)


def _projection_setup():
    from oracle import krylov
    S = _small_solver([4, 2, 1], smoother="jacobi", coarse="dense")
    L = S.fine
    A, free = _dense_operator(S)
    rhs = []
    for fr in [(1, 1, 1), (1, 2, 1), (2, 1, 1), (1, 1, 2)]:
        f, _ = wl.sinusoid(*fr)
        rhs.append(S.rhs(f(L.X[0], L.X[1], L.X[2])))
    return krylov, S, L, A, free, rhs


def test_projection_basis_is_a_orthonormal_and_guess_is_best_in_a_norm():
    """Successive right sides (Sec. 3.2 / 4.2): after three solves the basis is
    A-orthonormal, and the guess for a new b is the A-norm best approximation of
    the exact solution in its span (the error is A-orthogonal to the basis)."""
    krylov, S, L, A, free, rhs = _projection_setup()
    P = krylov.Projection(L.apply_A, L.wdot, 5)
    for b in rhs[:3]:
        res = krylov.projected_solve(krylov.fcg, P, L.apply_A, S.vcycle, b, L.wdot, 1e-12, 200)
        assert res.converged
    G = np.array([[L.wdot(xi, L.apply_A(xj)) for xj in P.X] for xi in P.X])
    np.testing.assert_allclose(G, np.eye(len(P.X)), atol=1e-10)
    b = rhs[3]
    x0 = P.guess(b)
    exact = np.zeros(L.num.n)
    exact[free] = np.linalg.solve(A, L.num.to_global(b)[free])
    err = L.num.Q(exact) - x0
    for xi in P.X:
        assert abs(L.wdot(xi, L.apply_A(err))) < 1e-10 * np.sqrt(L.wdot(b, b))


def test_projection_repeated_right_side_needs_no_iteration():
    """A right side already solved is reproduced by the guess alone, and the
    answer matches the dense solve; a new one converges to tol * ||b||."""
    krylov, S, L, A, free, rhs = _projection_setup()
    P = krylov.Projection(L.apply_A, L.wdot, 4)
    b = rhs[0]
    first = krylov.projected_solve(krylov.fcg, P, L.apply_A, S.vcycle, b, L.wdot, 1e-10, 200)
    again = krylov.projected_solve(krylov.fcg, P, L.apply_A, S.vcycle, b, L.wdot, 1e-8, 200)
    assert first.iters > 0 and again.iters == 0 and again.converged
    ref = np.zeros(L.num.n)
    ref[free] = np.linalg.solve(A, L.num.to_global(b)[free])
    np.testing.assert_allclose(L.num.to_global(again.x), ref, atol=1e-8 * np.abs(ref).max())
    other = krylov.projected_solve(krylov.fcg, P, L.apply_A, S.vcycle, rhs[1], L.wdot, 1e-8, 200)
    r = rhs[1] - L.apply_A(other.x)
    assert np.sqrt(L.wdot(r, r)) <= 1e-8 * np.sqrt(L.wdot(rhs[1], rhs[1]))


def test_projection_restarts_when_full():
    """With room for two vectors the third update restarts from the solution alone."""
    krylov, S, L, A, free, rhs = _projection_setup()
    P = krylov.Projection(L.apply_A, L.wdot, 2)
    sizes = []
    for b in rhs[:3]:
        res = krylov.projected_solve(krylov.fcg, P, L.apply_A, S.vcycle, b, L.wdot, 1e-10, 200)
        sizes.append(len(P.X))
    assert sizes == [1, 2, 1]
    x = res.x / np.sqrt(L.wdot(res.x, L.apply_A(res.x)))  # the third solution, A-normalised
    np.testing.assert_allclose(P.X[0], x, atol=1e-12 * np.abs(x).max())
    np.testing.assert_allclose(P.AX[0], L.apply_A(x), atol=1e-12 * np.abs(L.apply_A(x)).max())


@pytest.mark.parametrize("smoother", ["jacobi", "asm", "ras"])
def test_additive_vcycle_is_the_sum_of_smoother_and_coarse_correction(smoother):
    """Smoothers without Chebyshev acceleration (Sec. 2.2.2) use an additive
    V-cycle: on global free vectors M = S_0 + P_0 (S_1 + P_1 A_2^{-1} P_1^T) P_0^T,
    assembled here column by column from the level operators and a dense coarse
    solve; with the symmetric Jacobi smoother M is symmetric (the Schwarz forms
    carry a diagonal weight after their sum and are not)."""
    S = _small_solver([4, 2, 1], smoother=smoother, coarse="dense", cheb_order=0)
    L0, L1, L2 = S.levels
    f0 = np.nonzero(L0.num.mask_global > 0)[0]
    f1 = np.nonzero(L1.num.mask_global > 0)[0]

    def columns(apply, num_in, num_out, free_in, free_out):
        out = np.zeros((free_out.size, free_in.size))
        for j, g in enumerate(free_in):
            e = np.zeros(num_in.n)
            e[g] = 1.0
            out[:, j] = num_out.to_global(apply(num_in.Q(e)))[free_out]
        return out

    M = columns(S.vcycle, L0.num, L0.num, f0, f0)
    S0 = columns(L0.apply_S, L0.num, L0.num, f0, f0)
    S1 = columns(L1.apply_S, L1.num, L1.num, f1, f1)
    R0 = columns(lambda v: mg.restrict(L0.num, L1.num, L0.J_to_coarse, v), L0.num, L1.num, f0, f1)
    P0 = columns(lambda v: mg.prolong(L0.J_to_coarse, v), L1.num, L0.num, f1, f0)
    f2 = np.nonzero(L2.num.mask_global > 0)[0]
    R1 = columns(lambda v: mg.restrict(L1.num, L2.num, L1.J_to_coarse, v), L1.num, L2.num, f1, f2)
    P1 = columns(lambda v: mg.prolong(L1.J_to_coarse, v), L2.num, L1.num, f2, f1)
    A2, _ = _dense_operator(S, level=2)
    np.testing.assert_allclose(R0, P0.T, atol=1e-13)
    ref = S0 + P0 @ (S1 + P1 @ np.linalg.solve(A2, R1)) @ R0
    np.testing.assert_allclose(M, ref, atol=1e-11 * np.abs(ref).max())
    if smoother == "jacobi":
        np.testing.assert_allclose(M, M.T, atol=1e-11 * np.abs(M).max())


def test_unaccelerated_smoother_is_plain_schwarz():
    """cheb_order = 0: the smoothing step is x + S (b - A x), undamped."""
    S = _small_solver([4, 2, 1], smoother="ras", coarse="dense", cheb_order=0)
    L = S.fine
    rng = np.random.default_rng(3)
    b = L.num.mask * L.num.Q(rng.standard_normal(L.num.n))
    x = L.num.mask * L.num.Q(rng.standard_normal(L.num.n))
    np.testing.assert_allclose(L.smooth(b, x), L.apply_S(b - L.apply_A(x)), atol=1e-14)


@pytest.mark.parametrize("smoother", ["jacobi", "ras", "asm"])
def test_vcycle_is_the_two_grid_composition(smoother):
    """Algorithm 1 with Chebyshev smoothing (order 2) over three levels, as
    matrices on the free nodes: with Q_l the smoother from a zero start (its
    correction is Q_l applied to the residual), C_l = P_l M_{l+1} P_l^T the
    coarse-grid correction and M_2 = A_2^{-1}, one V-cycle from x = 0 is
        M_l = Q_l + (I - Q_l A_l) Q_l + (I - Q_l A_l) C_l (I - A_l Q_l)
    (pre-smooth, correct, post-smooth).  A dropped residual update, a
    correction with the wrong sign or in the wrong place fails this."""
    S = _small_solver([4, 2, 1], smoother=smoother, coarse="dense", lam=[2.2, 2.4])
    Ls = S.levels
    frees = [np.nonzero(L.num.mask_global > 0)[0] for L in Ls]

    def columns(apply, num_in, num_out, free_in, free_out):
        out = np.zeros((free_out.size, free_in.size))
        for j, g in enumerate(free_in):
            e = np.zeros(num_in.n)
            e[g] = 1.0
            out[:, j] = num_out.to_global(apply(num_in.Q(e)))[free_out]
        return out

    A2, _ = _dense_operator(S, level=2)
    M = np.linalg.inv(A2)
    for l in (1, 0):
        L, C = Ls[l], Ls[l + 1]
        f, fc = frees[l], frees[l + 1]
        A, _ = _dense_operator(S, level=l)
        Q = columns(lambda v: L.smooth(v, None), L.num, L.num, f, f)
        R = columns(lambda v: mg.restrict(L.num, C.num, L.J_to_coarse, v), L.num, C.num, f, fc)
        P = columns(lambda v: mg.prolong(L.J_to_coarse, v), C.num, L.num, fc, f)
        np.testing.assert_allclose(R, P.T, atol=1e-13)
        I = np.eye(f.size)
        M = Q + (I - Q @ A) @ Q + (I - Q @ A) @ (P @ M @ R) @ (I - A @ Q)
    Mv = columns(S.vcycle, Ls[0].num, Ls[0].num, frees[0], frees[0])
    np.testing.assert_allclose(Mv, M, atol=1e-10 * np.abs(M).max())
