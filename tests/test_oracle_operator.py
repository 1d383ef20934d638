"""Pins of the oracle's geometry, operator and discretisation (CPU only).

Sec. 2.1, eqs. 1-3: A_ij = (grad phi_i, grad phi_j)_p, B diagonal, A = Q^T A_L Q.
"""
import numpy as np
import pytest

from oracle import gll
from oracle.geom import geometric_factors
from oracle.mesh import Numbering, level_coordinates
from oracle.operator import (apply_A, apply_AL, assembled_diagonal, dense_free_system,
                             dense_global_A, element_matrix, local_diagonal, rhs)
from oracle.krylov import pcg
from paper_2110_07663_amd import workloads as wl


def build(nex, ney, nez, p, xyz, p_geom, bc=(1,) * 6):
    num = Numbering(nex, ney, nez, p, bc)
    X = level_coordinates(xyz, p_geom, p)
    G, BL, detJ = geometric_factors(X, p)
    return num, X, G, BL, detJ


def sin_mesh(n, p):
    xi, _ = gll.gll_nodes_weights(p)
    return wl.sampled_mesh(n, n, n, xi, wl.sin_map(0.05)), p


def test_mass_sums_to_volume_on_trilinear_meshes():
    for xyz, n in ((wl.box_vertices(2, 3, 2), (2, 3, 2)), (wl.layer_shift_vertices(4, seed=3), (4, 4, 4))):
        for p in (2, 3, 5):
            _, _, _, BL, detJ = build(*n, p, xyz, 1)
            assert abs(BL.sum() - 1.0) < 1e-13
            assert detJ.min() > 0


def test_box_element_geometric_factors_closed_form():
    p = 4
    nex, ney, nez = 2, 3, 5
    hx, hy, hz = 1 / nex, 1 / ney, 1 / nez
    _, w = gll.gll_nodes_weights(p)
    _, _, G, BL, _ = build(nex, ney, nez, p, wl.box_vertices(nex, ney, nez), 1)
    wq = w[None, :, None, None] * w[None, None, :, None] * w[None, None, None, :]
    np.testing.assert_allclose(G[0], wq * hy * hz / (2 * hx) * np.ones_like(G[0]), rtol=1e-13)
    np.testing.assert_allclose(G[3], wq * hx * hz / (2 * hy) * np.ones_like(G[0]), rtol=1e-13)
    np.testing.assert_allclose(G[5], wq * hx * hy / (2 * hz) * np.ones_like(G[0]), rtol=1e-13)
    for c in (1, 2, 4):
        assert np.abs(G[c]).max() < 1e-15 * 100
    np.testing.assert_allclose(BL, wq * hx * hy * hz / 8 * np.ones_like(BL), rtol=1e-13)


@pytest.mark.parametrize("p", [1, 2, 4, 7])
def test_box_element_matrix_closed_form(p):
    """A^e = c_x W(x)W(x)Ahat + c_y W(x)Ahat(x)W + c_z Ahat(x)W(x)W on a box."""
    nex, ney, nez = 2, 3, 5
    hx, hy, hz = 1 / nex, 1 / ney, 1 / nez
    _, w, D = gll.gll(p)
    Wm = np.diag(w)
    Ah = D.T @ Wm @ D
    ref = (hy * hz / (2 * hx)) * np.kron(Wm, np.kron(Wm, Ah)) \
        + (hx * hz / (2 * hy)) * np.kron(Wm, np.kron(Ah, Wm)) \
        + (hx * hy / (2 * hz)) * np.kron(Ah, np.kron(Wm, Wm))
    num, _, G, _, _ = build(nex, ney, nez, p, wl.box_vertices(nex, ney, nez), 1)
    N = p + 1
    e = 4
    np.testing.assert_allclose(element_matrix(G, p, e), ref, atol=1e-13 * np.abs(ref).max())
    # the sum-factorised A_L on unit vectors gives the same columns
    U = np.zeros((num.E, N, N, N))
    cols = []
    for q in range(N ** 3):
        U[:] = 0
        U.reshape(num.E, -1)[e, q] = 1.0
        cols.append(apply_AL(G, p, U)[e].reshape(-1))
    np.testing.assert_allclose(np.array(cols).T, ref, atol=1e-13 * np.abs(ref).max())


def test_operator_symmetric_on_curved_mesh():
    p = 5
    xyz, pg = sin_mesh(2, p)
    num, _, G, _, _ = build(2, 2, 2, p, xyz, pg)
    r = np.random.default_rng(0)
    u = num.mask * num.Q(r.standard_normal(num.n))
    v = num.mask * num.Q(r.standard_normal(num.n))
    a = num.wdot(u, apply_A(num, G, v))
    b = num.wdot(v, apply_A(num, G, u))
    assert abs(a - b) < 1e-12 * abs(a)


def test_neumann_operator_annihilates_constants():
    for p in (2, 5, 7):
        xyz, pg = sin_mesh(2, p)
        num, _, G, _, _ = build(2, 2, 2, p, xyz, pg, bc=(0,) * 6)
        Au = apply_A(num, G, np.ones((num.E,) + (p + 1,) * 3))
        assert np.abs(Au).max() < 1e-12 * np.abs(G).max()


def test_dirichlet_operator_spd():
    p = 3
    xyz, pg = sin_mesh(2, p)
    num, _, G, _, _ = build(2, 2, 2, p, xyz, pg)
    A, _ = dense_free_system(num, G)
    np.testing.assert_allclose(A, A.T, atol=1e-13 * np.abs(A).max())
    np.linalg.cholesky(A)


def test_linear_patch_test_on_trilinear_mesh():
    """Interior rows of A x vanish for the coordinate fields (trilinear, p >= 2)."""
    xyz = wl.layer_shift_vertices(3, seed=11)
    for p in (2, 4):
        num, X, G, _, _ = build(3, 3, 3, p, xyz, 1, bc=(0,) * 6)
        interior = num.Q(num.mask_global)  # all ones under Neumann; recompute interior
        gx, gy, gz = num.gx, num.gy, num.gz
        inner = (gx > 0) & (gx < num.nx - 1) & (gy > 0) & (gy < num.ny - 1) & (gz > 0) & (gz < num.nz - 1)
        for a in range(3):
            Ax = apply_A(num, G, X[a])
            assert np.abs(Ax[inner]).max() < 1e-12 * np.abs(G).max(), (p, a)
        assert interior.min() == 1


@pytest.mark.parametrize("p", [2, 3])
def test_sum_factorised_matches_dense_assembly(p):
    xyz, pg = sin_mesh(2, p)
    num, _, G, _, _ = build(2, 2, 2, p, xyz, pg)
    A = dense_global_A(num, G)
    r = np.random.default_rng(1)
    ug = r.standard_normal(num.n) * num.mask_global
    ref = num.mask_global * (A @ ug)
    got = num.to_global(apply_A(num, G, num.Q(ug)))
    np.testing.assert_allclose(got, ref, atol=1e-12 * np.abs(ref).max())
    # closed-form diagonal of A equals the dense diagonal
    d = num.to_global(assembled_diagonal(num, G))
    np.testing.assert_allclose(d, num.mask_global * np.diag(A), rtol=1e-13, atol=1e-15)


def test_local_diagonal_matches_element_matrix():
    p = 4
    xyz, pg = sin_mesh(2, p)
    num, _, G, _, _ = build(2, 2, 2, p, xyz, pg)
    d = local_diagonal(G, p)
    for e in (0, 5):
        np.testing.assert_allclose(d[e].reshape(-1), np.diag(element_matrix(G, p, e)), rtol=1e-13)


def _manufactured_error(n, p, mapping):
    xi, _ = gll.gll_nodes_weights(p)
    xyz = wl.sampled_mesh(n, n, n, xi, mapping)
    num, X, G, BL, _ = build(n, n, n, p, xyz, p)
    f, u = wl.sinusoid(1, 1, 1)
    b = rhs(num, BL, f(X[0], X[1], X[2]))
    dinv = np.where(num.mask > 0, 1.0 / np.where(num.mask > 0, assembled_diagonal(num, G), 1), 0)
    res = pcg(lambda v: apply_A(num, G, v), lambda r: dinv * r, b, num.wdot, 1e-14, 5000)
    assert res.converged
    return np.abs(res.x - u(X[0], X[1], X[2])).max()


def test_spectral_convergence_in_p():
    """Nodal error falls exponentially in p at fixed E (undeformed and curved)."""
    errs = [_manufactured_error(2, p, None) for p in (3, 5, 7, 9)]
    for a, b in zip(errs, errs[1:]):
        assert b < a / 20, errs
    assert errs[-1] < 1e-9, errs
    errs = [_manufactured_error(2, p, wl.sin_map(0.05)) for p in (3, 5, 7, 9)]
    for a, b in zip(errs, errs[1:]):
        assert b < a / 4, errs
    assert errs[-1] < 1e-5, errs


def test_algebraic_convergence_in_h():
    """Fixed p = 3 on the undeformed cube: rate >= p+1 under h-refinement."""
    e4 = _manufactured_error(4, 3, None)
    e8 = _manufactured_error(8, 3, None)
    assert np.log2(e4 / e8) >= 3.9, (e4, e8)
