"""GPU parity of the smoother, V-cycle and Krylov entry points against the oracle."""
import numpy as np
import pytest

from pairs import Pair, dev, host, rel_err
from paper_2110_07663_amd import sem
from paper_2110_07663_amd import workloads as wl

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    return torch


@pytest.mark.parametrize("smoother,p,shape", [("jacobi", 5, (3, 2, 2)), ("ras", 5, (3, 2, 2)),
                                              ("ras", 7, (2, 3, 2)), ("ras", 3, 3),
                                              ("ras", 6, (3, 2, 2)), ("ras", 8, (2, 2, 3)),
                                              ("ras", 9, (2, 3, 2)), ("ras", 10, (2, 2, 2))])
def test_schwarz_and_jacobi_surrogate_fp64(smoother, p, shape):
    P = Pair(shape, p, mesh="sin", schedule=(p, 1), smoother=smoother, lambda_override=[2.0])
    g, o = P.random_local(4)
    assert rel_err(host(P.gpu.apply_S(g)), P.ora.levels[0].apply_S(o)) < 1e-12


@pytest.mark.parametrize("bc", [(1, 1, 1, 1, 1, 1), (1, 0, 0, 1, 0, 1), (0, 0, 0, 0, 0, 1)])
def test_ras_boundary_conditions(bc):
    P = Pair((3, 2, 2), 4, mesh="sin", schedule=(4, 1), smoother="ras", bc=bc, lambda_override=[2.0])
    g, o = P.random_local(6)
    assert rel_err(host(P.gpu.apply_S(g)), P.ora.levels[0].apply_S(o)) < 1e-12


@pytest.mark.parametrize("p", [7, 9])
def test_ras_fp32(p):
    t = _torch()
    P = Pair(3, p, mesh="shift", schedule=(p, 3, 1), smoother="ras", smoother_prec=sem.F32,
             lambda_override=[2.0, 2.0])
    g, o = P.random_local(8)
    zg = host(P.gpu.apply_S(g.to(t.float32)))
    assert rel_err(zg, P.ora.levels[0].apply_S(o)) < 1e-5


@pytest.mark.parametrize("smoother", ["jacobi", "ras"])
def test_chebyshev_smooth(smoother):
    P = Pair((2, 3, 2), 5, mesh="sin", schedule=(5, 3, 1), smoother=smoother, cheb_order=3,
             lambda_override=[1.7, 1.9])
    b, bo = P.random_local(12)
    x, xo = P.random_local(13)
    P.gpu.smooth(b, x, level=0)
    ref = P.ora.smooth(bo, xo, level=0)
    assert rel_err(host(x), ref) < 1e-12
    # level 1 as well
    b1, bo1 = P.random_local(14, level=1)
    x1, xo1 = P.random_local(15, level=1)
    P.gpu.smooth(b1, x1, level=1)
    assert rel_err(host(x1), P.ora.smooth(bo1, xo1, level=1)) < 1e-12


@pytest.mark.parametrize("p,prec,xdefer,ydefer,bc", [
    (7, sem.F32, "1", "1", (1,) * 6), (7, sem.F32, "0", "1", (1,) * 6),
    (7, sem.F32, "1", "0", (0, 1, 1, 0, 1, 1)), (7, sem.F64, "1", "1", (0, 1, 1, 0, 1, 1)),
    (7, sem.F32, "1", "1", (1, 0, 0, 1, 0, 1)), (3, sem.F32, "1", "1", (1, 0, 1, 1, 0, 1)),
    (5, sem.F64, "1", "1", (0,) * 6), (5, sem.F64, "1", "0", (1,) * 6)])
def test_chebyshev_takes_the_x_step(monkeypatch, p, prec, xdefer, ydefer, bc):
    """Cheby-RAS smoothing where the gather-scatter after each FDM leaves its x
    step, and by default its y step, to the Chebyshev update that reads the
    result (SEM_GS_XDEFER=0 assembles first, SEM_GS_YDEFER=0 defers x only),
    against the oracle; Neumann faces included (Dirichlet ones read as zero)."""
    t = _torch()
    monkeypatch.setenv("SEM_GS_XDEFER", xdefer)
    monkeypatch.setenv("SEM_GS_YDEFER", ydefer)
    P = Pair((3, 2, 2), p, mesh="sin", schedule=(p, 1), smoother="ras", cheb_order=3, bc=bc,
             smoother_prec=prec, lambda_override=[1.8])
    b, bo = P.random_local(16)
    x, xo = P.random_local(17)
    if prec == sem.F32:
        b, x = b.to(t.float32), x.to(t.float32)
    P.gpu.smooth(b, x, level=0)
    ref = P.ora.smooth(bo, xo, level=0)
    assert rel_err(host(x), ref) < (1e-5 if prec == sem.F32 else 1e-12)


@pytest.mark.parametrize("smoother", ["jacobi", "ras"])
def test_arnoldi_lambda_tilde(smoother):
    P = Pair((3, 2, 2), 6, mesh="sin", schedule=(6, 3, 1), smoother=smoother, seed=77)
    for l in range(2):
        got = P.gpu.levels[l].lmax / 1.1
        ref = P.ora.levels[l].lam_tilde
        assert abs(got - ref) < 1e-9 * ref, (l, got, ref)


@pytest.mark.parametrize("smoother,sched", [("jacobi", (7, 3, 1)), ("ras", (7, 3, 1)),
                                            ("ras", (5, 1)), ("jacobi", (4, 2, 1))])
def test_vcycle_fixed_coarse_iterations(smoother, sched):
    # 18 free coarse unknowns, 12 coarse iterations: no exact convergence inside
    P = Pair((4, 4, 3), sched[0], mesh="sin", schedule=sched, smoother=smoother,
             coarse_tol=0.0, coarse_maxit=12, lambda_override=[1.5] * (len(sched) - 1))
    g, o = P.random_local(21)
    zg = host(P.gpu.vcycle(g))
    zo = P.ora.vcycle(o)
    assert rel_err(zg, zo) < 1e-12


def test_vcycle_converged_coarse_matches_to_coarse_tolerance():
    P = Pair(3, 7, mesh="shift", schedule=(7, 3, 1), smoother="ras", coarse_tol=1e-10)
    g, o = P.random_local(22)
    assert rel_err(host(P.gpu.vcycle(g)), P.ora.vcycle(o)) < 1e-8


def test_vcycle_graph_replays_match_every_time():
    """The coarse CG chunk is a replayed HIP graph: check several replays, with
    eager work and synchronisation in between, against the oracle."""
    t = _torch()
    P = Pair(4, 5, mesh="shift", schedule=(5, 3, 1), smoother="ras", coarse_tol=1e-10)
    for seed in (31, 32, 33):
        g, o = P.random_local(seed)
        z = P.gpu.vcycle(g)
        _ = P.gpu.apply_A(g)  # unrelated eager work between replays
        t.cuda.synchronize()
        assert rel_err(host(z), P.ora.vcycle(o)) < 1e-8


@pytest.mark.parametrize("env", [("SEM_COARSE_GRAPH", "0"), ("SEM_COARSE_PERSIST", "1")])
def test_coarse_solve_paths_agree(monkeypatch, env):
    """The coarse CG runs as replayed graph chunks (default), as eager chunks of
    varying length (both alternating copies of r, s, w get used first), or as
    one persistent cooperative launch; all take the same steps."""
    base = Pair(6, 3, mesh="shift", schedule=(3, 1), smoother="jacobi", coarse_tol=1e-10,
                oracle=False, lambda_override=[1.8])
    monkeypatch.setenv(*env)
    other = Pair(6, 3, mesh="shift", schedule=(3, 1), smoother="jacobi", coarse_tol=1e-10,
                 oracle=False, lambda_override=[1.8])
    for seed in (41, 42, 43):
        g, _ = base.random_local(seed)
        za = host(base.gpu.vcycle(g))
        zb = host(other.gpu.vcycle(g))
        assert rel_err(zb, za) < 1e-13, (env, seed)


def _rhs(P, a=1, b=1, c=1):
    f, u = wl.sinusoid(a, b, c)
    X = host(P.gpu.coords(0))
    bg = P.gpu.rhs(dev(f(X[0], X[1], X[2])))
    Xo = P.ora.fine.X
    bo = P.ora.rhs(f(Xo[0], Xo[1], Xo[2]))
    return bg, bo


@pytest.mark.parametrize("krylov,smoother", [(sem.KRYLOV_FCG, "jacobi"), (sem.KRYLOV_FCG, "ras"),
                                             (sem.KRYLOV_PCG, "jacobi"), (sem.KRYLOV_FGMRES, "ras")])
def test_solve_fixed_iterations(krylov, smoother):
    """Same number of outer iterations on both sides: iterates agree to rounding."""
    kname = {sem.KRYLOV_FCG: "fcg", sem.KRYLOV_PCG: "pcg", sem.KRYLOV_FGMRES: "fgmres"}[krylov]
    P = Pair((4, 4, 3), 5, mesh="sin", schedule=(5, 3, 1), smoother=smoother, krylov=krylov,
             coarse_tol=0.0, coarse_maxit=12, lambda_override=[1.6, 1.8], gmres_restart=4)
    bg, bo = _rhs(P)
    xg, info = P.gpu.solve(bg, rtol=1e-30, maxit=6, allow_noconv=True)
    res = P.ora.solve(bo, tol=1e-30, maxit=6, krylov=kname, restart=4)
    assert info.iters == res.iters == 6
    assert rel_err(host(xg), res.x) < 1e-11


@pytest.mark.parametrize("krylov,shape", [(sem.KRYLOV_FCG, (4, 2, 3)), (sem.KRYLOV_PCG, (4, 2, 3)),
                                          (sem.KRYLOV_FCG, (3, 2, 2))])
def test_solve_fixed_iterations_p7(krylov, shape):
    """p = 7: (p, Ap) comes from the Ax kernel's element shares of p^T A_L p
    (with and without the in-workgroup x-face sums: nex = 4 and 3); six
    iterations agree with the oracle's weighted-dot iteration to rounding."""
    kname = {sem.KRYLOV_FCG: "fcg", sem.KRYLOV_PCG: "pcg"}[krylov]
    P = Pair(shape, 7, mesh="sin", schedule=(7, 3, 1), smoother="ras", krylov=krylov,
             coarse_tol=0.0, coarse_maxit=12, lambda_override=[1.6, 1.8])
    bg, bo = _rhs(P)
    xg, info = P.gpu.solve(bg, rtol=1e-30, maxit=6, allow_noconv=True)
    res = P.ora.solve(bo, tol=1e-30, maxit=6, krylov=kname)
    assert info.iters == res.iters == 6
    assert rel_err(host(xg), res.x) < 1e-11


@pytest.mark.parametrize("krylov", [sem.KRYLOV_FCG, sem.KRYLOV_FGMRES])
def test_solve_to_tolerance(krylov):
    P = Pair(3, 7, mesh="shift", schedule=(7, 3, 1), smoother="ras", krylov=krylov)
    bg, bo = _rhs(P)
    xg, info = P.gpu.solve(bg, rtol=1e-8, maxit=100)
    assert info.converged and info.true_rel_res <= 1e-8
    L = P.ora.fine
    x = host(xg).reshape(bo.shape)
    r = bo - L.apply_A(x)
    assert np.sqrt(L.wdot(r, r) / L.wdot(bo, bo)) <= 1e-8
    res = P.ora.solve(bo, tol=1e-8, maxit=100)
    assert abs(info.iters - res.iters) <= 1
    assert rel_err(x, res.x) < 1e-6


@pytest.mark.parametrize("shape,p,sched,smoother,bc,mesh,lam", [
    ((3, 3, 3), 5, (5, 3, 1), "ras", (1,) * 6, "sin", [1.7, 1.9]),
    ((7, 6, 3), 3, (3, 1), "jacobi", (1,) * 6, "sin", [1.9]),             # 8x7 plane: two 32-blocks
    ((9, 8, 3), 2, (2, 1), "jacobi", (1, 0, 0, 1, 0, 1), "sin", [1.9]),   # 10x9 plane: three blocks
    # 4^3 layer-shift: one element per slab, strongly skewed; the oracle's
    # Arnoldi gives lambda~ = 41.9 and 14.6 for RAS here
    (4, 7, (7, 3, 1), "ras", (1,) * 6, "shift", [42.0, 14.6]),
])
@pytest.mark.parametrize("csum", ["1", "0"])
def test_vcycle_direct_coarse_matches_oracle(monkeypatch, csum, shape, p, sched, smoother, bc,
                                             mesh, lam):
    """Exact block-tridiagonal coarse solve against the oracle's dense solve;
    the coarse right side reaches it as the restriction leaves it (its copies
    summed by the mapping to the global numbering) or assembled first
    (SEM_COARSE_SUM=0)."""
    monkeypatch.setenv("SEM_COARSE_SUM", csum)
    P = Pair(shape, p, mesh=mesh, schedule=sched, smoother=smoother, bc=bc, coarse="dense",
             lambda_override=lam)
    for seed in (51, 52):
        g, o = P.random_local(seed)
        assert rel_err(host(P.gpu.vcycle(g)), P.ora.vcycle(o)) < 1e-12


@pytest.mark.parametrize("csum", ["1", "0"])
@pytest.mark.parametrize("prec", [sem.F64, sem.F32])
def test_vcycle_pcg_coarse_summed_right_side(monkeypatch, csum, prec):
    """Coarse Jacobi-PCG (fixed count) with the restricted right side summed
    by its mapping or assembled first: same V-cycle as the oracle's with the
    same coarse iteration count; mixed faces."""
    monkeypatch.setenv("SEM_COARSE_SUM", csum)
    P = Pair((4, 3, 3), 5, mesh="sin", schedule=(5, 3, 1), smoother="ras", coarse="pcg",
             coarse_tol=0.0, coarse_maxit=12, bc=(1, 0, 1, 1, 0, 1), smoother_prec=prec,
             lambda_override=[1.7, 1.9])
    for seed in (56, 57):
        g, o = P.random_local(seed)
        err = rel_err(host(P.gpu.vcycle(g)), P.ora.vcycle(o))
        assert err < (1e-12 if prec == sem.F64 else 1e-5), err


def test_direct_coarse_falls_back_when_singular():
    """All-Neumann: the p = 1 level is singular, the setup keeps the CG."""
    kw = dict(mesh="sin", schedule=(4, 1), smoother="jacobi", bc=(0,) * 6, coarse_tol=0.0,
              coarse_maxit=5, lambda_override=[1.8], oracle=False)
    a = Pair(3, 4, coarse="dense", **kw)
    b = Pair(3, 4, coarse="pcg", **kw)
    g, _ = a.random_local(53, masked=False)
    za, zb = host(a.gpu.vcycle(g)), host(b.gpu.vcycle(g))
    assert np.all(np.isfinite(za))
    assert rel_err(za, zb) < 1e-14


@pytest.mark.parametrize("keep_f64", ["0", "1"])
def test_direct_coarse_fp32_factors(monkeypatch, keep_f64):
    """Under an FP32 smoother the exact coarse sweeps read FP32 copies of the
    factored blocks (FP64 vectors and sums): the single-level solve then meets
    the oracle's dense solve to about 1e-7 rather than 1e-12.  SEM_COARSE_F64=1
    keeps the FP64 blocks.  7x6x3 elements: 8x7 planes, two 32-row blocks."""
    monkeypatch.setenv("SEM_COARSE_F64", keep_f64)
    P = Pair((7, 6, 3), 1, mesh="sin", schedule=(1,), coarse="dense", smoother_prec=sem.F32)
    for seed in (54, 55):
        g, o = P.random_local(seed)
        err = rel_err(host(P.gpu.vcycle(g)), P.ora.vcycle(o))
        if keep_f64 == "1":
            assert err < 1e-12, err
        else:
            assert 1e-12 < err < 2e-6, err


def test_solve_with_direct_coarse():
    P = Pair(3, 7, mesh="shift", schedule=(7, 3, 1), smoother="ras", coarse="dense")
    bg, bo = _rhs(P)
    xg, info = P.gpu.solve(bg, rtol=1e-8, maxit=100)
    assert info.converged and info.true_rel_res <= 1e-8 and info.coarse_iters == 0
    L = P.ora.fine
    x = host(xg).reshape(bo.shape)
    r = bo - L.apply_A(x)
    assert np.sqrt(L.wdot(r, r) / L.wdot(bo, bo)) <= 1e-8
    res = P.ora.solve(bo, tol=1e-8, maxit=100)
    assert abs(info.iters - res.iters) <= 1


@pytest.mark.parametrize("shape", [4, (3, 2, 2)])
def test_solve_fp16_geometry(shape):
    """FP32 Cheby-RAS pMG whose A at p = 7 reads FP16 geometric factors (with
    x-face sums in the Ax kernel when nex is a multiple of 4, without them
    otherwise): the FP64 outer FCG still reaches 1e-8 measured with the oracle's
    A, in at most one iteration more than with FP32 factors."""
    base = dict(mesh="sin", schedule=(7, 3, 1), smoother="ras", smoother_prec=sem.F32,
                coarse="dense")
    P = Pair(shape, 7, geom_prec=sem.F16, **base)
    P32 = Pair(shape, 7, oracle=False, **base)
    bg, bo = _rhs(P)
    xg, info = P.gpu.solve(bg, rtol=1e-8, maxit=100)
    _, info32 = P32.gpu.solve(bg, rtol=1e-8, maxit=100)
    assert info.converged and info.true_rel_res <= 1e-8
    L = P.ora.fine
    x = host(xg).reshape(bo.shape)
    r = bo - L.apply_A(x)
    assert np.sqrt(L.wdot(r, r) / L.wdot(bo, bo)) <= 1e-8
    assert info.iters <= info32.iters + 1


def test_jacobi_pcg_config1_small():
    """Plain Jacobi-PCG on the undeformed cube, p = 3 (the oracle-size workload)."""
    P = Pair(4, 3, mesh="box", krylov=sem.KRYLOV_PCG, precond=sem.PRECOND_JACOBI)
    bg, bo = _rhs(P)
    xg, info = P.gpu.solve(bg, rtol=1e-10, maxit=500)
    res = P.ora.jacobi_pcg(bo, 1e-10, 500)
    assert abs(info.iters - res.iters) <= 1
    assert rel_err(host(xg), res.x) < 1e-9
    # discretisation error against the manufactured solution
    _, u = wl.sinusoid(1, 1, 1)
    X = host(P.gpu.coords(0))
    assert np.abs(host(xg) - u(X[0], X[1], X[2])).max() < 2e-4


def test_mixed_precision_solve():
    P = Pair(4, 7, mesh="shift", schedule=(7, 3, 1), smoother="ras", smoother_prec=sem.F32)
    bg, bo = _rhs(P)
    xg, info = P.gpu.solve(bg, rtol=1e-8, maxit=100)
    assert info.converged
    L = P.ora.fine
    r = bo - L.apply_A(host(xg).reshape(bo.shape))
    assert np.sqrt(L.wdot(r, r) / L.wdot(bo, bo)) <= 1e-8
    res = P.ora.solve(bo, tol=1e-8, maxit=100)
    assert info.iters <= res.iters + 2


@pytest.mark.parametrize("shape,bc", [((4, 3, 2), (1,) * 6), ((3, 2, 3), (0, 1, 1, 0, 1, 1))])
def test_mixed_solve_with_deferred_steps_matches_assembled(monkeypatch, shape, bc):
    """Mixed FCG at p = 7: the outer A p and the smoother's S w leave their x
    and y gather-scatter steps to the pointwise updates that read them, and
    the smoother's A w leaves them to the FDM (default); or everything runs
    assembled (SEM_GS_XDEFER=0, SEM_FDM_XSTEP=0).  Both reach the oracle's
    residual with the same iteration count, and the solutions agree to the
    FP32 preconditioner's rounding."""
    sols = {}
    for xdefer in ("1", "0"):
        monkeypatch.setenv("SEM_GS_XDEFER", xdefer)
        monkeypatch.setenv("SEM_FDM_XSTEP", xdefer)
        P = Pair(shape, 7, mesh="sin", schedule=(7, 3, 1), smoother="ras", smoother_prec=sem.F32,
                 bc=bc, lambda_override=[1.8, 1.6], coarse="dense")
        bg, bo = _rhs(P)
        xg, info = P.gpu.solve(bg, rtol=1e-8, maxit=100)
        assert info.converged
        L = P.ora.fine
        x = host(xg).reshape(bo.shape)
        r = bo - L.apply_A(x)
        assert np.sqrt(L.wdot(r, r) / L.wdot(bo, bo)) <= 1e-8
        sols[xdefer] = (x, info.iters)
    assert abs(sols["1"][1] - sols["0"][1]) <= 1
    assert rel_err(sols["1"][0], sols["0"][0]) < 1e-7


def test_error_paths():
    t = _torch()
    P = Pair(2, 3, mesh="box", schedule=(3, 1), oracle=False)
    bg = t.full((P.gpu.levels[0].nlocal,), float("nan"), dtype=t.float64, device="cuda")
    with pytest.raises(sem.SemError) as ei:
        P.gpu.solve(bg, rtol=1e-8, maxit=10)
    assert ei.value.status == sem.SEM_ENAN
    b, _ = P.random_local(1)
    x, info = P.gpu.solve(b, rtol=1e-12, maxit=1, allow_noconv=True)
    assert info.converged == 0 and info.iters == 1
    # inverted element is rejected at setup
    xyz = wl.box_vertices(2, 2, 2)
    xyz[0, [0, 1]] = xyz[0, [1, 0]]
    with pytest.raises(sem.SemError) as ei:
        sem.Solver(2, 2, 2, xyz, 1, 3, opts=sem.make_opts(schedule=(3, 1)))
    assert ei.value.status == sem.SEM_EGEOM


@pytest.mark.parametrize("fdm_prec,tol", [(sem.F16, 5e-3), (sem.BF16, 4e-2)])
@pytest.mark.parametrize("p", [3, 7, 9])
def test_ras_mfma_low_precision(fdm_prec, tol, p):
    """FDM contractions on MFMA (16-bit operands, FP32 accumulation) against the FP64 oracle."""
    t = _torch()
    P = Pair(3, p, mesh="shift", schedule=(p, 1), smoother="ras", smoother_prec=sem.F32,
             fdm_prec=fdm_prec, lambda_override=[2.0])
    g, o = P.random_local(8)
    zg = host(P.gpu.apply_S(g.to(t.float32)))
    err = rel_err(zg, P.ora.levels[0].apply_S(o))
    assert err < tol, err


@pytest.mark.parametrize("fdm_prec", [sem.F16, sem.BF16])
def test_mixed_mfma_solve_converges(fdm_prec):
    P = Pair(4, 7, mesh="shift", schedule=(7, 3, 1), smoother="ras", smoother_prec=sem.F32,
             fdm_prec=fdm_prec)
    bg, bo = _rhs(P)
    xg, info = P.gpu.solve(bg, rtol=1e-8, maxit=200)
    assert info.converged
    L = P.ora.fine
    r = bo - L.apply_A(host(xg).reshape(bo.shape))
    assert np.sqrt(L.wdot(r, r) / L.wdot(bo, bo)) <= 1e-8


@pytest.mark.parametrize("p,prec", [(4, sem.F64), (7, sem.F64), (5, sem.F32), (9, sem.F32)])
def test_asm_surrogate(p, prec):
    """Additive Schwarz (eq. 4) with 1/#boxes weights against the oracle."""
    t = _torch()
    P = Pair((3, 2, 2), p, mesh="sin", schedule=(p, 1), smoother="asm", lambda_override=[2.0],
             smoother_prec=sem.F32 if prec == sem.F32 else sem.F64, bc=(1, 0, 1, 1, 0, 1))
    g, o = P.random_local(10)
    if prec == sem.F32:
        g = g.to(t.float32)
    err = rel_err(host(P.gpu.apply_S(g)), P.ora.levels[0].apply_S(o))
    assert err < (1e-12 if prec == sem.F64 else 1e-5), err


@pytest.mark.parametrize("p,prec,smoother,group", [
    (3, sem.F32, "ras", "1"), (3, sem.F64, "ras", "1"), (3, sem.F32, "ras", "0"),
    (3, sem.F64, "asm", "0"), (4, sem.F32, "ras", "1"), (4, sem.F64, "asm", "1"),
    (2, sem.F32, "asm", "1"), (3, sem.F32, "asm", "1"), (2, sem.F64, "ras", "0")])
def test_small_box_fdm_groups(monkeypatch, p, prec, smoother, group):
    """p <= 3: one workgroup solves the boxes of several elements (7 at p = 3 in
    FP32); E = 30 leaves the last group partly empty.  SEM_FDM_GROUP=0 keeps one
    wavefront per workgroup."""
    monkeypatch.setenv("SEM_FDM_GROUP", group)
    t = _torch()
    f32 = prec == sem.F32
    P = Pair((5, 3, 2), p, mesh="sin", schedule=(p, 1), smoother=smoother, lambda_override=[2.0],
             smoother_prec=prec, bc=(1, 0, 1, 1, 0, 1))
    g, o = P.random_local(11)
    err = rel_err(host(P.gpu.apply_S(g.to(t.float32) if f32 else g)), P.ora.levels[0].apply_S(o))
    assert err < (1e-5 if f32 else 1e-12), err


def test_asm_vcycle_and_solve():
    P = Pair(3, 5, mesh="shift", schedule=(5, 3, 1), smoother="asm", coarse_tol=0.0,
             coarse_maxit=6, lambda_override=[1.5, 1.5])
    g, o = P.random_local(23)
    assert rel_err(host(P.gpu.vcycle(g)), P.ora.vcycle(o)) < 1e-12
    # the solve uses Arnoldi bounds (the fixed 1.5 above underestimates ASM's spectrum)
    Q = Pair(3, 5, mesh="shift", schedule=(5, 3, 1), smoother="asm")
    bg, bo = _rhs(Q)
    xg, info = Q.gpu.solve(bg, rtol=1e-8, maxit=200)
    assert info.converged and info.true_rel_res <= 1e-8
    L = Q.ora.fine
    r = bo - L.apply_A(host(xg).reshape(bo.shape))
    assert np.sqrt(L.wdot(r, r) / L.wdot(bo, bo)) <= 1e-8


@pytest.mark.parametrize("krylov", [sem.KRYLOV_FCG, sem.KRYLOV_FGMRES])
def test_projection_of_successive_right_sides_matches_oracle(krylov):
    """A-conjugate projection onto prior solutions (Sec. 3.2 / 4.2), room for
    two: the projected initial residual, the iteration counts and the solutions
    follow the oracle; a repeated right side needs no iteration; the third new
    direction restarts the basis; reset empties it."""
    from oracle import krylov as okr
    P = Pair((2, 2, 2), 4, mesh="sin", schedule=(4, 2, 1), smoother="jacobi",
             lambda_override=[1.8, 1.6], coarse="dense", krylov=krylov, proj_max=2)
    L = P.ora.fine
    solver = okr.fcg if krylov == sem.KRYLOV_FCG else okr.fgmres
    proj = okr.Projection(L.apply_A, L.wdot, 2)
    Xg = host(P.gpu.coords(0))
    Xo = L.X
    seq = [(1, 1, 1), (1, 1, 1), (1, 2, 1), (2, 1, 1), (1, 2, 1)]
    for k, fr in enumerate(seq):
        f, _ = wl.sinusoid(*fr)
        bg = P.gpu.rhs(dev(f(Xg[0], Xg[1], Xg[2])))
        bo = P.ora.rhs(f(Xo[0], Xo[1], Xo[2]))
        nb = np.sqrt(L.wdot(bo, bo))
        x0 = proj.guess(bo)
        r = bo - L.apply_A(x0)
        r0 = np.sqrt(L.wdot(r, r))
        xg, ig = P.gpu.solve(bg, rtol=1e-9, maxit=100)
        ro = okr.projected_solve(solver, proj, L.apply_A, P.ora.vcycle, bo, L.wdot, 1e-9, 100)
        assert ig.converged and ro.converged
        assert abs(ig.r0_norm - r0) <= 1e-6 * r0 + 1e-9 * nb, (k, ig.r0_norm, r0)
        assert abs(ig.iters - ro.iters) <= 1, (k, ig.iters, ro.iters)
        if k == 1:
            assert ig.iters == 0 and ro.iters == 0
        assert rel_err(host(xg), ro.x) < 1e-7
        res = bo - L.apply_A(host(xg).reshape(bo.shape))
        assert np.sqrt(L.wdot(res, res)) <= 2e-9 * nb
    P.gpu.projection_reset()
    f, _ = wl.sinusoid(1, 1, 1)
    bg = P.gpu.rhs(dev(f(Xg[0], Xg[1], Xg[2])))
    _, ig = P.gpu.solve(bg, rtol=1e-9, maxit=100)
    b1 = P.ora.rhs(f(Xo[0], Xo[1], Xo[2]))
    nb1 = np.sqrt(L.wdot(b1, b1))
    assert abs(ig.r0_norm - nb1) <= 1e-12 * nb1  # empty basis: x0 = 0, r0 = ||b||


@pytest.mark.parametrize("smoother,sched,prec", [
    ("jacobi", (4, 2, 1), sem.F64), ("ras", (5, 3, 1), sem.F64), ("asm", (5, 3, 1), sem.F64),
    ("ras", (7, 3, 1), sem.F32),
])
def test_additive_vcycle_without_acceleration(smoother, sched, prec):
    """cheb_order = 0 (Sec. 2.2.2, smoothers without Chebyshev acceleration):
    additive V-cycle x = S b + P V(P^T b) against the oracle (FP64 1e-12, FP32
    1e-5), the un-accelerated smoothing step x + S(b - A x), and a solve that
    reaches the tolerance."""
    t = _torch()
    P = Pair((3, 2, 3), sched[0], mesh="sin", schedule=sched, smoother=smoother, cheb_order=0,
             coarse="dense", smoother_prec=prec, lambda_override=[1.5] * (len(sched) - 1))
    tol = 1e-12 if prec == sem.F64 else 1e-5
    for seed in (71, 72):
        g, o = P.random_local(seed)
        assert rel_err(host(P.gpu.vcycle(g)), P.ora.vcycle(o)) < tol
    if prec == sem.F64:
        b, bo = P.random_local(73)
        x, xo = P.random_local(74)
        xs = x.clone()
        P.gpu.smooth(b, xs)
        ref = xo + P.ora.fine.smooth(bo, xo)
        assert rel_err(host(xs), ref) < 1e-12
    bg, bo = _rhs(P)
    xg, info = P.gpu.solve(bg, rtol=1e-8, maxit=300)
    assert info.converged
    L = P.ora.fine
    r = bo - L.apply_A(host(xg).reshape(bo.shape))
    assert np.sqrt(L.wdot(r, r) / L.wdot(bo, bo)) <= 1e-8


def test_profile_classes():
    """Kernel-class timing: every class, or only those of the mask; a negative
    mask is rejected."""
    P = Pair((4, 2, 2), 5, mesh="sin", schedule=(5, 3, 1), smoother="ras", smoother_prec=sem.F32,
             coarse="dense", oracle=False)
    f, _ = wl.sinusoid(1, 1, 1)
    X = host(P.gpu.coords(0))
    import torch
    b = P.gpu.rhs(torch.as_tensor(f(X[0], X[1], X[2])).cuda())
    P.gpu.profile(True)
    P.gpu.solve(b, rtol=1e-8, maxit=100)
    allk = P.gpu.profile_read()
    assert all(allk[k][1] > 0 for k in ("ax64", "ax32", "fdm", "gs32", "vcycle", "coarse"))
    P.gpu.profile(True, kinds=("ax32", "fdm"))
    P.gpu.solve(b, rtol=1e-8, maxit=100)
    some = P.gpu.profile_read()
    P.gpu.profile(False)
    assert some["ax32"][1] == allk["ax32"][1] and some["fdm"][1] == allk["fdm"][1]
    assert all(some[k][1] == 0 for k in ("ax64", "gs32", "gs64", "coarse", "vcycle"))
    assert all(some[k][0] > 0 for k in ("ax32", "fdm"))
    with pytest.raises(sem.SemError) as ei:
        sem.check(sem.lib().sem_profile(P.gpu.ctx, -2))
    assert ei.value.status == sem.SEM_EINVAL
