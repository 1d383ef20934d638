"""GPU parity of the four-level p-multigrid schedules of the paper's tuning
table (Sec. 5: (7,5,3,1) and (9,7,5,1), used with Cheby-Jacobi) against the
oracle: every transfer pair they add (7<->5, 9<->7, 5<->3, 7<->5), the
V-cycle with an exact coarse solve (FP64 to 1e-12, FP32 levels to 1e-5), and a
Cheby-Jacobi(2) solve on (7,5,3,1) judged by the oracle's residual."""
import numpy as np
import pytest

from oracle import mg
from pairs import Pair, host, rel_err
from paper_2110_07663_amd import sem
from paper_2110_07663_amd import workloads as wl

pytestmark = pytest.mark.gpu

SCHEDULES = [(7, 5, 3, 1), (9, 7, 5, 1)]


@pytest.mark.parametrize("sched", SCHEDULES)
@pytest.mark.parametrize("prec", [sem.F64, sem.F32])
def test_four_level_transfers(sched, prec):
    t = __import__("torch")
    P = Pair((3, 2, 2), sched[0], mesh="sin", schedule=sched, lambda_override=[1.0] * 4,
             smoother_prec=prec)
    tol = 1e-12 if prec == sem.F64 else 1e-6
    for l in range(len(sched) - 1):
        gc, oc = P.random_local(60 + l, level=l + 1)
        gf, of = P.random_local(70 + l, level=l)
        if prec == sem.F32:
            gc, gf = gc.to(t.float32), gf.to(t.float32)
        xf = gf.clone()
        P.gpu.prolong(gc, xf, level=l)
        ref = of + mg.prolong(P.ora.levels[l].J_to_coarse, oc)
        assert rel_err(host(xf), ref) < tol, (sched, l)
        rc = host(P.gpu.restrict(gf, level=l))
        refc = mg.restrict(P.ora.levels[l].num, P.ora.levels[l + 1].num,
                           P.ora.levels[l].J_to_coarse, of)
        assert rel_err(rc, refc) < tol, (sched, l)


@pytest.mark.parametrize("sched,shape", [((7, 5, 3, 1), (3, 2, 2)), ((9, 7, 5, 1), (2, 2, 3))])
@pytest.mark.parametrize("smoother", ["jacobi", "ras"])
@pytest.mark.parametrize("prec", [sem.F64, sem.F32])
def test_four_level_vcycle(sched, shape, smoother, prec):
    """One V-cycle of Algorithm 1 over four levels, fixed lambda~ per level
    and the exact coarse solve (GPU block elimination, oracle dense solve)."""
    P = Pair(shape, sched[0], mesh="sin", schedule=sched, smoother=smoother, coarse="dense",
             smoother_prec=prec, lambda_override=[1.6, 1.7, 1.8])
    for seed in (81, 82):
        g, o = P.random_local(seed)
        err = rel_err(host(P.gpu.vcycle(g)), P.ora.vcycle(o))
        assert err < (1e-12 if prec == sem.F64 else 1e-5), (seed, err)


@pytest.mark.parametrize("sched", SCHEDULES)
def test_four_level_smoothing_on_every_level(sched):
    """Chebyshev-Jacobi smoothing on each non-coarse level of the schedule."""
    P = Pair((2, 2, 2), sched[0], mesh="sin", schedule=sched, smoother="jacobi",
             lambda_override=[1.6, 1.7, 1.8])
    for l in range(len(sched) - 1):
        b, bo = P.random_local(90 + l, level=l)
        x, xo = P.random_local(95 + l, level=l)
        P.gpu.smooth(b, x, level=l)
        assert rel_err(host(x), P.ora.smooth(bo, xo, level=l)) < 1e-12, l


@pytest.mark.parametrize("prec", [sem.F64, sem.F32])
def test_cheby_jacobi_four_level_solve(prec):
    """Cheby-Jacobi(2) with the (7,5,3,1) schedule, Arnoldi bounds, coarse
    Jacobi-PCG to 1e-10: the oracle's FP64 operator reports the GPU solution at
    relative residual <= 1e-8, and the oracle's own solve takes about as many
    iterations."""
    P = Pair((3, 3, 2), 7, mesh="sin", schedule=(7, 5, 3, 1), smoother="jacobi",
             smoother_prec=prec, coarse="pcg", coarse_tol=1e-10)
    f, _ = wl.sinusoid(1, 2, 1)
    X = host(P.gpu.coords(0))
    import torch
    bg = P.gpu.rhs(torch.as_tensor(f(X[0], X[1], X[2])).cuda())
    Xo = P.ora.fine.X
    bo = P.ora.rhs(f(Xo[0], Xo[1], Xo[2]))
    xg, info = P.gpu.solve(bg, rtol=1e-8, maxit=200)
    assert info.converged
    L = P.ora.fine
    x = host(xg).reshape(bo.shape)
    r = bo - L.apply_A(x)
    assert np.sqrt(L.wdot(r, r) / L.wdot(bo, bo)) <= 1e-8
    res = P.ora.solve(bo, tol=1e-8, maxit=200)
    assert abs(info.iters - res.iters) <= (1 if prec == sem.F64 else 3), (info.iters, res.iters)
    assert rel_err(x, res.x) < 1e-6
