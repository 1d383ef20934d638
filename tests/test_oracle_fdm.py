"""Pins of the oracle's Schwarz/FDM smoother (CPU only).

Sec. 2.2.2, eqs. 4-9.
"""
import numpy as np
import pytest

from oracle import gll
from oracle.fdm import FDM, extended_1d, generalized_eig
from oracle.geom import geometric_factors
from oracle.mesh import Numbering, level_coordinates
from oracle.operator import apply_A, dense_global_A
from paper_2110_07663_amd import workloads as wl


CASES_1D = [
    # (p, Lm, L, Lp, has_l, has_r, dir_l, dir_r)
    (3, 0.3, 0.5, 0.2, True, True, 0, 0),
    (5, 0.0, 0.25, 0.1, False, True, 1, 0),
    (5, 0.0, 0.25, 0.1, False, True, 0, 0),
    (7, 0.1, 0.05, 0.0, True, False, 0, 1),
    (4, 0.0, 1.0, 0.0, False, False, 1, 1),
    (6, 0.0, 0.4, 0.0, False, False, 0, 1),
]


@pytest.mark.parametrize("case", CASES_1D)
def test_generalized_eigenproblem_similarity(case):
    """S^T A S = Lambda and S^T B S = I on the coupled nodes (eq. 7)."""
    K, M, cpl = extended_1d(*case)
    S, lam = generalized_eig(K, M, cpl)
    c = np.nonzero(cpl)[0]
    m = len(c)
    Sc = S[np.ix_(c, np.arange(m))]
    np.testing.assert_allclose(Sc.T @ K[np.ix_(c, c)] @ Sc, np.diag(lam[:m]), atol=1e-12 * np.abs(lam[:m]).max())
    np.testing.assert_allclose(Sc.T @ M[np.ix_(c, c)] @ Sc, np.eye(m), atol=1e-13)
    assert np.all(np.isinf(lam[m:]))
    # decoupled columns are unit vectors on decoupled nodes
    for col in range(m, len(lam)):
        assert np.count_nonzero(S[:, col]) == 1 and not cpl[np.nonzero(S[:, col])[0][0]]


def test_1d_extended_matrices_are_three_element_assembly():
    """Interior rows of the extended stiffness match the global 1D assembly of 3 elements."""
    p = 4
    _, w, D = gll.gll(p)
    Ah = D.T @ np.diag(w) @ D
    K, M, _ = extended_1d(p, 0.2, 0.5, 0.3, True, True, 0, 0)
    # the element's node 0 (extended index 1) is shared by left and centre
    assert abs(K[1, 1] - (Ah[p, p] * 2 / 0.2 + Ah[0, 0] * 2 / 0.5)) < 1e-12
    assert abs(M[1, 1] - (w[p] * 0.2 / 2 + w[0] * 0.5 / 2)) < 1e-15
    assert abs(K[0, 1] - Ah[p - 1, p] * 2 / 0.2) < 1e-12
    assert abs(K[p + 2, p + 1] - Ah[1, 0] * 2 / 0.3) < 1e-12
    assert K[0, p + 2] == 0.0


def _rectilinear(nx, ny, nz, seed):
    """Tensor-product mesh with random 1D spacings (box lengths are exact)."""
    r = np.random.default_rng(seed)
    gx = np.concatenate([[0], np.cumsum(r.uniform(0.5, 2.0, nx))])
    gy = np.concatenate([[0], np.cumsum(r.uniform(0.5, 2.0, ny))])
    gz = np.concatenate([[0], np.cumsum(r.uniform(0.5, 2.0, nz))])
    gx, gy, gz = gx / gx[-1], gy / gy[-1], gz / gz[-1]
    v = wl.box_vertices(nx, ny, nz)
    ix = np.rint(v[:, :, 0] * nx).astype(int)
    iy = np.rint(v[:, :, 1] * ny).astype(int)
    iz = np.rint(v[:, :, 2] * nz).astype(int)
    return np.stack([gx[ix], gy[iy], gz[iz]], axis=2)


def _level(nex, ney, nez, p, xyz, p_geom, bc):
    num = Numbering(nex, ney, nez, p, bc)
    X = level_coordinates(xyz, p_geom, p)
    G, _, _ = geometric_factors(X, p)
    return num, X, G


@pytest.mark.parametrize("p", [2, 3, 5])
def test_fdm_equals_dense_kronecker_inverse(p):
    """FDM action = solve with Abar of eq. 5 built by Kronecker products."""
    xi, _ = gll.gll_nodes_weights(p)
    xyz = wl.sampled_mesh(3, 3, 2, xi, wl.sin_map(0.05))
    bc = (1, 0, 1, 1, 0, 1)
    num, X, G = _level(3, 3, 2, p, xyz, p, bc)
    fdm = FDM(num, X)
    from oracle.fdm import box_lengths
    L = box_lengths(X)
    r = np.random.default_rng(p)
    pb = p + 3
    for e in (0, 4, num.E - 1):
        ex, ey, ez = e % 3, (e // 3) % 3, e // 9
        pos, cnt, stride = (ex, ey, ez), (3, 3, 2), (1, 3, 9)
        Ks, Ms, Cs = [], [], []
        for d in range(3):
            hl, hr = pos[d] > 0, pos[d] < cnt[d] - 1
            K, M, c = extended_1d(p, L[e - stride[d], d] if hl else 0, L[e, d],
                                  L[e + stride[d], d] if hr else 0, hl, hr, bc[2 * d], bc[2 * d + 1])
            Ks.append(K), Ms.append(M), Cs.append(c)
        Abar = np.kron(Ms[2], np.kron(Ms[1], Ks[0])) + np.kron(Ms[2], np.kron(Ks[1], Ms[0])) \
            + np.kron(Ks[2], np.kron(Ms[1], Ms[0]))
        cpl = (Cs[2][:, None, None] & Cs[1][None, :, None] & Cs[0][None, None, :]).reshape(-1)
        v = r.standard_normal(pb ** 3)
        ref = np.zeros(pb ** 3)
        idx = np.nonzero(cpl)[0]
        ref[idx] = np.linalg.solve(Abar[np.ix_(idx, idx)], v[idx])
        rb = np.zeros((num.E, pb, pb, pb))
        rb[e] = v.reshape(pb, pb, pb)
        got = fdm.local_solve(rb)[e].reshape(-1)
        np.testing.assert_allclose(got, ref, atol=1e-11 * np.abs(ref).max())


@pytest.mark.parametrize("p,bc", [(3, (1,) * 6), (4, (1, 0, 1, 0, 0, 1))])
def test_fdm_equals_galerkin_local_inverse_on_rectilinear_mesh(p, bc):
    """On a tensor-product mesh Abar_e = R_e A R_e^T, so FDM is the exact local inverse."""
    nex, ney, nez = 3, 3, 3
    xyz = _rectilinear(nex, ney, nez, seed=p)
    num, X, G = _level(nex, ney, nez, p, xyz, 1, bc)
    fdm = FDM(num, X)
    A = dense_global_A(num, G)
    r = np.random.default_rng(7)
    pb = p + 3
    for e in (0, 13, 26):
        g = fdm.box_gid[e].reshape(-1)
        ok = g >= 0
        free = ok.copy()
        free[ok] = num.mask_global[g[ok]] > 0
        fi = np.nonzero(free)[0]
        v = r.standard_normal(pb ** 3) * free
        ref = np.zeros(pb ** 3)
        ref[fi] = np.linalg.solve(A[np.ix_(g[fi], g[fi])], v[fi])
        rb = np.zeros((num.E, pb, pb, pb))
        rb[e] = v.reshape(pb, pb, pb)
        got = fdm.local_solve(rb)[e].reshape(-1)
        np.testing.assert_allclose(got, ref, atol=1e-11 * np.abs(ref).max())


def test_ras_on_single_element_is_exact_inverse():
    """E = 1, Dirichlet box: the extended box adds only decoupled nodes, so RAS = A^{-1}."""
    p = 5
    xyz = _rectilinear(1, 1, 1, seed=3)
    num, X, G = _level(1, 1, 1, p, xyz, 1, (1,) * 6)
    fdm = FDM(num, X)
    u = num.mask * num.Q(np.random.default_rng(0).standard_normal(num.n))
    np.testing.assert_allclose(fdm.apply_ras(apply_A(num, G, u)), u, atol=1e-12)
    np.testing.assert_allclose(fdm.apply_asm(apply_A(num, G, u)), u, atol=1e-12)


def test_schwarz_weights_partition_of_unity():
    p = 3
    num = Numbering(3, 2, 2, p)
    W_ras = 1.0 / num.Q(num.mult)
    np.testing.assert_allclose(num.Qt(W_ras), 1.0, atol=1e-15)
    xyz = wl.box_vertices(3, 2, 2)
    X = level_coordinates(xyz, 1, p)
    fdm = FDM(num, X)
    ok = fdm.box_gid >= 0
    nbox = np.bincount(fdm.box_gid[ok], minlength=num.n)
    ones = np.ones(ok.sum())
    s = np.bincount(fdm.box_gid[ok], weights=ones / nbox[fdm.box_gid[ok]], minlength=num.n)
    np.testing.assert_allclose(s, 1.0, atol=1e-15)
    assert nbox.min() >= 1 and nbox.max() <= 27


def _box_nodes(nex, ney, nez, p, e):
    """Global ids of the nodes of element e's box extended by one node per side
    (Sec. 2.2.2), clipped to the domain; written from the node grid alone."""
    ex, ey, ez = e % nex, (e // nex) % ney, e // (nex * ney)
    nx, ny, nz = nex * p + 1, ney * p + 1, nez * p + 1
    xs = [x for x in range(ex * p - 1, ex * p + p + 2) if 0 <= x < nx]
    ys = [y for y in range(ey * p - 1, ey * p + p + 2) if 0 <= y < ny]
    zs = [z for z in range(ez * p - 1, ez * p + p + 2) if 0 <= z < nz]
    return np.array([(z * ny + y) * nx + x for z in zs for y in ys for x in xs])


def _own_nodes(nex, ney, nez, p, e):
    ex, ey, ez = e % nex, (e // nex) % ney, e // (nex * ney)
    nx, ny = nex * p + 1, ney * p + 1
    return np.array([((ez * p + k) * ny + ey * p + j) * nx + ex * p + i
                     for k in range(p + 1) for j in range(p + 1) for i in range(p + 1)])


@pytest.mark.parametrize("p,bc", [(3, (1, 0, 1, 1, 0, 1)), (4, (0, 1, 1, 0, 1, 1))])
def test_schwarz_sum_equals_dense_galerkin_assembly(p, bc):
    """Eq. 4 and the RAS paragraph of Sec. 2.2.2 over many elements, from dense matrices.

    On a rectilinear tensor mesh the box operator equals the Galerkin restriction
    R_e A R_e^T of the assembled A to the box's free nodes, so the two smoothers
    are fixed without any FDM data:
      ASM: s = W * sum_e R_e^T (R_e A R_e^T)^{-1} R_e r with W = 1/#boxes per node;
      RAS: the same local solves, each kept on the element's own nodes only,
           weighted by 1/(number of elements owning the node), then summed.
    Both are compared with the oracle's FDM form on a random consistent r.
    """
    nex, ney, nez = 3, 3, 2
    xyz = _rectilinear(nex, ney, nez, seed=10 + p)
    num, X, G = _level(nex, ney, nez, p, xyz, 1, bc)
    fdm = FDM(num, X)
    A = dense_global_A(num, G)
    free = num.mask_global > 0
    rng = np.random.default_rng(p)
    r_glob = rng.standard_normal(num.n) * free
    r_loc = num.Q(r_glob)

    asm = np.zeros(num.n)
    nbox = np.zeros(num.n)
    ras = np.zeros(num.n)
    owners = np.zeros(num.n)
    for e in range(num.E):
        own = _own_nodes(nex, ney, nez, p, e)
        owners[own] += 1
    for e in range(num.E):
        box = _box_nodes(nex, ney, nez, p, e)
        nbox[box] += 1
        bf = box[free[box]]
        y = np.zeros(num.n)
        y[bf] = np.linalg.solve(A[np.ix_(bf, bf)], r_glob[bf])
        asm += y
        own = _own_nodes(nex, ney, nez, p, e)
        ras[own] += y[own] / owners[own]
    asm /= nbox

    got_asm = fdm.apply_asm(r_loc)
    got_ras = fdm.apply_ras(r_loc)
    scale_a, scale_r = np.abs(asm).max(), np.abs(ras).max()
    np.testing.assert_allclose(got_asm, num.Q(asm), atol=1e-11 * scale_a)
    np.testing.assert_allclose(got_ras, num.Q(ras), atol=1e-11 * scale_r)
    # the two smoothers differ (the overlap matters), and both are consistent E-vectors
    assert np.abs(asm - ras).max() > 1e-3 * scale_a
    # a plausible misreading is caught: RAS weighted by 1/#boxes instead of 1/#owners
    wrong = np.zeros(num.n)
    for e in range(num.E):
        box = _box_nodes(nex, ney, nez, p, e)
        bf = box[free[box]]
        y = np.zeros(num.n)
        y[bf] = np.linalg.solve(A[np.ix_(bf, bf)], r_glob[bf])
        own = _own_nodes(nex, ney, nez, p, e)
        wrong[own] += y[own] / nbox[own]
    assert np.abs(num.Q(wrong) - got_ras).max() > 1e-3 * scale_r
