"""GPU parity of the setup and operator entry points against the oracle.

FP64 results must match the oracle to 1e-12 relative (2-norm over E-vector
entries); FP32 results to 1e-5.
"""
import numpy as np
import pytest

from oracle import gll as ogll
from oracle.operator import apply_A as o_apply_A
from pairs import Pair, dev, global_mask, host, rel_err
from paper_2110_07663_amd import sem
from paper_2110_07663_amd import workloads as wl

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("p", [1, 2, 3, 5, 7, 8, 9, 10, 13])
def test_gll_nodes_and_weights(p):
    xg, wg = sem.gll_nodes(p)
    xo, wo = ogll.gll_nodes_weights(p)
    np.testing.assert_allclose(xg, xo, atol=2e-16 * p * p, rtol=0)
    np.testing.assert_allclose(wg, wo, rtol=1e-14)


@pytest.mark.parametrize("shape,p,mesh,bc", [
    ((3, 2, 5), 3, "sin", (1, 1, 1, 1, 1, 1)),
    ((2, 3, 2), 7, "sin", (1, 0, 0, 1, 1, 0)),
    ((3, 3, 3), 5, "shift", (1, 1, 1, 1, 1, 1)),
    ((1, 1, 1), 4, "box", (0, 0, 0, 0, 0, 0)),
])
def test_numbering_and_coordinates(shape, p, mesh, bc):
    P = Pair(shape if mesh != "shift" else shape[0], p, mesh=mesh, bc=bc)
    info = P.gpu.levels[0]
    num = P.ora.levels[0].num
    assert info.nglobal == num.n and info.nlocal == num.E * (p + 1) ** 3
    shared_or_dir = (num.mult > 1) | (num.mask_global == 0)
    assert info.nshared == int(shared_or_dir.sum())
    X = host(P.gpu.coords(0))
    assert rel_err(X, P.oracle_nodes(0)) < 1e-14
    g, o = P.random_local(11, masked=False)
    np.testing.assert_array_equal(host(g), o.reshape(-1))


@pytest.mark.parametrize("shape,p,mesh", [
    ((3, 2, 5), 1, "sin"), ((3, 2, 5), 2, "sin"), ((3, 2, 5), 3, "sin"), ((2, 3, 2), 5, "sin"),
    ((3, 2, 3), 7, "sin"), ((2, 2, 3), 8, "sin"), ((2, 2, 2), 9, "sin"), ((2, 1, 2), 10, "sin"),
    (4, 7, "shift"), ((5, 3, 2), 6, "box"),
])
def test_apply_A_fp64(shape, p, mesh):
    P = Pair(shape if mesh != "shift" else shape, p, mesh=mesh, bc=(1, 1, 0, 1, 1, 0))
    g, o = P.random_local(3, masked=False)
    Ag = host(P.gpu.apply_A(g))
    Ao = P.ora.levels[0].apply_A(o)
    assert rel_err(Ag, Ao) < 1e-12


@pytest.mark.parametrize("sorted_gs,xfuse,yz", [(False, True, True), (False, False, True),
                                               (False, True, False), (True, True, True)])
@pytest.mark.parametrize("shape,p,bc", [
    ((3, 2, 5), 3, (1, 0, 1, 1, 0, 1)), ((1, 4, 2), 7, (1,) * 6), ((2, 2, 2), 1, (0,) * 6),
    ((4, 3, 2), 7, (0, 1, 1, 0, 0, 1)), ((8, 2, 3), 7, (1, 1, 0, 1, 1, 0)),
    ((12, 1, 2), 7, (0, 0, 1, 1, 1, 1)),
])
def test_gather_scatter_paths(monkeypatch, sorted_gs, xfuse, yz, shape, p, bc):
    """Direction passes (default; at p = 7 with nex a multiple of 4 the Ax
    kernel sums the x-faces inside its workgroups first; the y and z passes run
    as one launch), the same without the x-face fusion, with the y and z passes
    as two launches, and sorted segments for QQ^T: A matches the oracle, every
    copy of a global node holds the same bits, Dirichlet copies are exactly
    zero; FP32 likewise to its tolerance."""
    t = __import__("torch")
    monkeypatch.setenv("SEM_GS_SORTED", "1" if sorted_gs else "0")
    monkeypatch.setenv("SEM_AX_XFUSE", "1" if xfuse else "0")
    monkeypatch.setenv("SEM_GS_YZ", "1" if yz else "0")
    P = Pair(shape, p, mesh="sin", bc=bc, smoother_prec=sem.F32)
    num = P.ora.levels[0].num
    g, o = P.random_local(21, masked=False)
    Ao = P.ora.levels[0].apply_A(o)
    for x, tol in ((g, 1e-12), (g.to(t.float32), 1e-5)):
        Ag = host(P.gpu.apply_A(x)).reshape(-1)
        assert rel_err(Ag, Ao) < tol
        gid = num.gid.reshape(-1)
        order = np.argsort(gid, kind="stable")
        gs, vs = gid[order], Ag[order]
        first = np.r_[0, np.flatnonzero(np.diff(gs)) + 1]
        lead = np.repeat(vs[first], np.diff(np.r_[first, gs.size]))
        np.testing.assert_array_equal(vs, lead)
        assert np.all(Ag[num.mask.reshape(-1) == 0] == 0)


@pytest.mark.parametrize("p", [3, 7])
def test_apply_A_fp32(p):
    t = __import__("torch")
    P = Pair((3, 2, 3), p, mesh="sin", smoother_prec=sem.F32)
    g, o = P.random_local(5, masked=True)
    Ag = host(P.gpu.apply_A(g.to(t.float32)))
    Ao = P.ora.levels[0].apply_A(o)
    assert rel_err(Ag, Ao) < 1e-5


@pytest.mark.parametrize("shape,p", [((4, 3, 2), 7), ((5, 2, 3), 7), ((3, 2, 2), 5), ((2, 3, 2), 3)])
def test_apply_A_fp16_geometry(shape, p):
    """The FP32 product with the geometric factors stored in FP16 (the
    one-wavefront kernel at p = 7, the slab kernel otherwise).

    Each stored factor is the FP64 one scaled by a power of two and rounded to
    nearest in FP16, so it is within 2^-11 of it, relative.  By the sum
    factorisation of Sec. 2.1, the error of every entry of Au is then at most
    2^-11 times the same product taken over absolute values,
    mask * QQ^T (|D|^T |G| |D| |u|), plus the FP32 arithmetic's own share.  A
    factor read in the wrong slot, or an element left unscaled, breaks the
    bound by orders of magnitude.
    """
    t = __import__("torch")
    from oracle import gll as og
    from oracle.geom import reference_gradient
    from oracle.operator import G_full
    # level 0 must be a smoothed level (the coarsest keeps FP32 factors)
    P = Pair(shape, p, mesh="sin", schedule=(p, 1), smoother_prec=sem.F32, geom_prec=sem.F16)
    g, o = P.random_local(11, masked=True)
    Ag = host(P.gpu.apply_A(g.to(t.float32)))
    lev = P.ora.levels[0]
    Ao = lev.apply_A(o)
    Dabs = np.abs(og.gll(p)[2])
    ga = reference_gradient(Dabs, np.abs(o))
    Gf = G_full([np.abs(c) for c in lev.G])
    w = [sum(Gf[a][b] * ga[b] for b in range(3)) for a in range(3)]
    va = np.einsum('li,ekjl->ekji', Dabs, w[0])
    va += np.einsum('mj,ekmi->ekji', Dabs, w[1])
    va += np.einsum('nk,enji->ekji', Dabs, w[2])
    bound = (lev.num.mask * lev.num.QQt(va)).reshape(-1)
    err = np.abs(Ag - Ao.reshape(-1))
    assert np.all(err <= (2.0 ** -11 + 1e-5) * bound + 1e-7 * bound.max())
    # the rounding is really there: above the FP32 path's 1e-5 (test_apply_A_fp32)
    assert 1e-5 < rel_err(Ag, Ao) < 2e-3


def test_apply_A_neumann_annihilates_constants():
    t = __import__("torch")
    P = Pair(3, 6, mesh="sin", bc=(0,) * 6, oracle=False)
    one = t.ones(P.gpu.levels[0].nlocal, dtype=t.float64, device="cuda")
    A1 = host(P.gpu.apply_A(one))
    g, _ = P.random_local(1, masked=False)
    Ag = host(P.gpu.apply_A(g))
    assert np.abs(A1).max() < 1e-12 * np.abs(Ag).max()


def test_apply_A_bitwise_repeatable():
    P = Pair(3, 7, mesh="sin", oracle=False)
    g, _ = P.random_local(2)
    a = host(P.gpu.apply_A(g))
    b = host(P.gpu.apply_A(g))
    np.testing.assert_array_equal(a, b)


def test_rhs_matches_oracle():
    P = Pair((3, 2, 2), 5, mesh="sin")
    f, _ = wl.sinusoid(1, 2, 1)
    X = host(P.gpu.coords(0))
    fl = f(X[0], X[1], X[2])
    bg = host(P.gpu.rhs(dev(fl)))
    Xo = P.ora.fine.X
    bo = P.ora.rhs(f(Xo[0], Xo[1], Xo[2]))
    assert rel_err(bg, bo) < 1e-12


@pytest.mark.parametrize("prec", [sem.F64, sem.F32])
def test_jacobi_surrogate(prec):
    t = __import__("torch")
    P = Pair((2, 3, 2), 5, mesh="sin", schedule=(5, 3, 1),
             smoother_prec=sem.F32 if prec == sem.F32 else sem.F64, lambda_override=[1.0, 1.0])
    g, o = P.random_local(9)
    if prec == sem.F32:
        g = g.to(t.float32)
    for level in range(3):
        gl, ol = P.random_local(20 + level, level=level)
        if prec == sem.F32:
            gl = gl.to(t.float32)
        zg = host(P.gpu.apply_S(gl, level=level))
        zo = P.ora.levels[level].apply_S(ol)
        assert rel_err(zg, zo) < (1e-12 if prec == sem.F64 else 1e-6)


@pytest.mark.parametrize("prec", [sem.F64, sem.F32])
@pytest.mark.parametrize("shape", [(3, 2, 2), (3, 1, 3)])
@pytest.mark.parametrize("sched", [(7, 3, 1), (5, 3, 1), (9, 5, 1), (4, 2, 1)])
def test_transfers(sched, shape, prec):
    """Every pair of the schedules, on 12 and 9 elements (the small pairs
    run four elements per workgroup: a partly filled last one)."""
    t = __import__("torch")
    P = Pair(shape, sched[0], mesh="sin", schedule=sched, lambda_override=[1.0] * 3,
             smoother_prec=prec)
    tol = 1e-12 if prec == sem.F64 else 1e-6
    for l in range(len(sched) - 1):
        gc, oc = P.random_local(30 + l, level=l + 1)
        gf, of = P.random_local(40 + l, level=l)
        if prec == sem.F32:
            gc, gf = gc.to(t.float32), gf.to(t.float32)
        xf = gf.clone()
        P.gpu.prolong(gc, xf, level=l)
        from oracle import mg
        ref = of + mg.prolong(P.ora.levels[l].J_to_coarse, oc)
        assert rel_err(host(xf), ref) < tol
        rc = host(P.gpu.restrict(gf, level=l))
        refc = mg.restrict(P.ora.levels[l].num, P.ora.levels[l + 1].num, P.ora.levels[l].J_to_coarse, of)
        assert rel_err(rc, refc) < tol


def _subgrid_apply(xyz_all, n, p, e_center, u_global, bc):
    """Oracle A u at the nodes of one element from the 3x3x3 element block around it."""
    from oracle.geom import geometric_factors
    from oracle.mesh import Numbering, level_coordinates
    ex, ey, ez = e_center % n, (e_center // n) % n, e_center // (n * n)
    lo = [max(0, c - 1) for c in (ex, ey, ez)]
    hi = [min(n - 1, c + 1) for c in (ex, ey, ez)]
    sx, sy, sz = hi[0] - lo[0] + 1, hi[1] - lo[1] + 1, hi[2] - lo[2] + 1
    els = [((z * n) + y) * n + x for z in range(lo[2], hi[2] + 1) for y in range(lo[1], hi[1] + 1)
           for x in range(lo[0], hi[0] + 1)]
    sub = Numbering(sx, sy, sz, p, (0,) * 6)
    X = level_coordinates(xyz_all[els], 1, p)
    G, _, _ = geometric_factors(X, p)
    nx = n * p + 1
    gx = sub.gx + lo[0] * p
    gy = sub.gy + lo[1] * p
    gz = sub.gz + lo[2] * p
    u = u_global[(gz * nx + gy) * nx + gx]
    Au = o_apply_A(sub, G, u)
    c = els.index(e_center)
    m = global_mask(n, n, n, p, bc)[((gz * nx + gy) * nx + gx)[c]]
    return (Au[c] * m).reshape(-1)


@pytest.mark.parametrize("n,p", [(32, 7), (16, 7)])
def test_apply_A_full_size_sampled(n, p):
    """Full-size layer-shift mesh: sampled elements against the oracle's 3x3x3 sub-mesh."""
    P = Pair(n, p, mesh="shift", oracle=False)
    L = P.gpu.levels[0]
    ug = wl.random_global(L.nglobal, 7) * global_mask(n, n, n, p, (1,) * 6)
    Ag = P.gpu.apply_A(P.gpu.gather(dev(ug)))
    xyz = wl.layer_shift_vertices(n, seed=3)
    N3 = (p + 1) ** 3
    rng = np.random.default_rng(0)
    sample = [0, n ** 3 - 1, n // 2 * (1 + n + n * n)] + list(rng.integers(0, n ** 3, 9))
    gots, refs, per = [], [], []
    for e in sample:
        got = host(Ag[e * N3:(e + 1) * N3])
        ref = _subgrid_apply(xyz, n, p, int(e), ug, (1,) * 6)
        gots.append(got)
        refs.append(ref)
        per.append(rel_err(got, ref))
    # norm-wise over all sampled outputs; single 10:1 elements cancel more, so
    # each element alone is held to 1e-11
    assert rel_err(np.concatenate(gots), np.concatenate(refs)) < 1e-12, per
    assert max(per) < 1e-11, per


@pytest.mark.parametrize("shape,p,bc", [((3, 2, 5), 3, (1, 0, 1, 1, 0, 1)), ((4, 3, 2), 7, (0, 1, 1, 0, 0, 1)),
                                        ((2, 1, 3), 5, (0,) * 6), ((1, 3, 1), 2, (1,) * 6)])
def test_gather_scatter_yz_launch_is_bitwise(monkeypatch, shape, p, bc):
    """The one-launch y/z pass gives the two passes' results bit for bit (same
    sums in the same order), FP64 and FP32, for A and for the smoother."""
    t = __import__("torch")
    out = {}
    for yz in ("1", "0"):
        monkeypatch.setenv("SEM_GS_YZ", yz)
        P = Pair(shape, p, mesh="sin", bc=bc, smoother_prec=sem.F32, schedule=(p, 1),
                 smoother="ras", lambda_override=[2.0], oracle=False)
        g, _ = P.random_local(22, masked=False)
        out[yz] = [host(P.gpu.apply_A(g)), host(P.gpu.apply_A(g.to(t.float32))),
                   host(P.gpu.apply_S(g.to(t.float32)))]
    for a, b in zip(out["1"], out["0"]):
        np.testing.assert_array_equal(a, b)
