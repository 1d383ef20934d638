"""GPU tests of the batched (graph-recorded, device-scalar) solve and of the auto-tuner."""
import numpy as np
import pytest

from pairs import Pair, dev, host, rel_err
from paper_2110_07663_amd import sem
from paper_2110_07663_amd import workloads as wl

pytestmark = pytest.mark.gpu


def _rhs_pair(P, a, b, c):
    f, _ = wl.sinusoid(a, b, c)
    X = host(P.gpu.coords(0))
    bg = P.gpu.rhs(dev(f(X[0], X[1], X[2])))
    Xo = P.ora.fine.X
    bo = P.ora.rhs(f(Xo[0], Xo[1], Xo[2]))
    return bg, bo


def _oracle_rel_res(P, x, bo):
    L = P.ora.fine
    r = bo - L.apply_A(x.reshape(bo.shape))
    return np.sqrt(L.wdot(r, r) / L.wdot(bo, bo))


def test_batched_solve_matches_individual_solves():
    import torch
    probs = [((3, 3, 3), 5, (5, 3, 1), "ras"), ((2, 3, 2), 7, (7, 3, 1), "ras"),
             ((4, 4, 4), 3, (3, 1), "jacobi")]
    freqs = [(1, 1, 1), (2, 1, 3)]
    pairs, bs, bos = [], [], []
    for shape, p, sched, sm in probs:
        P = Pair(shape, p, mesh="sin", schedule=sched, smoother=sm, smoother_prec=sem.F32)
        # a second context with batch lanes for the same problem
        opts = sem.make_opts(schedule=sched, smoother={"ras": sem.SMOOTH_RAS, "jacobi": sem.SMOOTH_JACOBI}[sm],
                             smoother_prec=sem.F32, batch_rhs=len(freqs))
        xyz = wl.sampled_mesh(*shape, sem.gll_nodes(p)[0], wl.sin_map(0.05))
        P.batch = sem.Solver(*shape, xyz, p, p, opts=opts)
        row, orow = [], []
        for fr in freqs:
            bg, bo = _rhs_pair(P, *fr)
            row.append(bg)
            orow.append(bo)
        pairs.append(P)
        bs.append(row)
        bos.append(orow)
    xs = [[torch.zeros_like(b) for b in row] for row in bs]
    infos = sem.batch_solve([P.batch for P in pairs], bs, xs, rtol=1e-8, maxit=200)
    for i, P in enumerate(pairs):
        for k in range(len(freqs)):
            inf = infos[i * len(freqs) + k]
            assert inf.converged and inf.true_rel_res <= 1e-8
            xb = host(xs[i][k])
            assert _oracle_rel_res(P, xb, bos[i][k]) <= 1e-8
            xi, ii = P.gpu.solve(bs[i][k], rtol=1e-8, maxit=200)
            assert abs(inf.iters - ii.iters) <= 3, (inf.iters, ii.iters)
            assert rel_err(xb, host(xi)) < 1e-6


def test_batched_solve_uneven_convergence():
    """Lanes that converge at very different iterations (layer-shift meshes,
    whose trapezoidal elements need many iterations, beside smooth sine maps):
    the batch records again as problems finish, and every lane still converges,
    meets the oracle's residual and follows its own individual solve."""
    import torch
    probs = [(4, 7, (7, 3, 1), "ras", "shift"), (3, 5, (5, 3, 1), "ras", "shift"),
             ((2, 2, 2), 3, (3, 1), "jacobi", "sin"), ((3, 2, 2), 5, (5, 3, 1), "ras", "sin")]
    freqs = [(1, 1, 1), (2, 1, 3)]
    pairs, bs, bos = [], [], []
    for n, p, sched, sm, mesh in probs:
        P = Pair(n, p, mesh=mesh, schedule=sched, smoother=sm, smoother_prec=sem.F32)
        shape = P.shape
        if mesh == "shift":
            xyz, pg = wl.layer_shift_vertices(shape[0], seed=3), 1
        else:
            xyz, pg = wl.sampled_mesh(*shape, sem.gll_nodes(p)[0], wl.sin_map(0.05)), p
        opts = sem.make_opts(schedule=sched, smoother={"ras": sem.SMOOTH_RAS, "jacobi": sem.SMOOTH_JACOBI}[sm],
                             smoother_prec=sem.F32, batch_rhs=len(freqs))
        P.batch = sem.Solver(*shape, xyz, pg, p, opts=opts)
        pairs.append(P)
        row, orow = zip(*[_rhs_pair(P, *fr) for fr in freqs])
        bs.append(list(row))
        bos.append(list(orow))
    xs = [[torch.zeros_like(b) for b in row] for row in bs]
    infos = sem.batch_solve([P.batch for P in pairs], bs, xs, rtol=1e-8, maxit=300)
    its = [i.iters for i in infos]
    assert max(its) >= 2 * min(its), its
    for i, P in enumerate(pairs):
        for k in range(len(freqs)):
            inf = infos[i * len(freqs) + k]
            assert inf.converged and inf.true_rel_res <= 1e-8, (i, k, inf.iters)
            xb = host(xs[i][k])
            assert _oracle_rel_res(P, xb, bos[i][k]) <= 1e-8
            xi, ii = P.gpu.solve(bs[i][k], rtol=1e-8, maxit=300)
            assert abs(inf.iters - ii.iters) <= 3, (inf.iters, ii.iters)
            assert rel_err(xb, host(xi)) < 1e-6


def test_batched_solve_repeatable():
    """Identical lanes give identical results, and a second batched call repeats the first."""
    import torch
    opts = sem.make_opts(schedule=(5, 3, 1), smoother=sem.SMOOTH_RAS, smoother_prec=sem.F32,
                         batch_rhs=2)
    xyz = wl.layer_shift_vertices(3, seed=3)
    S = sem.Solver(3, 3, 3, xyz, 1, 5, opts=opts)
    f, _ = wl.sinusoid(1, 2, 1)
    X = host(S.coords(0))
    b = S.rhs(dev(f(X[0], X[1], X[2])))
    xs = [[torch.zeros_like(b), torch.zeros_like(b)]]
    infos = sem.batch_solve([S], [[b, b]], xs, rtol=1e-8)
    assert all(i.converged for i in infos)
    np.testing.assert_array_equal(host(xs[0][0]), host(xs[0][1]))  # same input, same lane code
    x2 = [[torch.zeros_like(b), torch.zeros_like(b)]]
    infos2 = sem.batch_solve([S], [[b, b]], x2, rtol=1e-8)
    assert [i.iters for i in infos2] == [i.iters for i in infos]
    np.testing.assert_array_equal(host(x2[0][0]), host(xs[0][0]))


def test_autotuner_picks_a_converged_fast_candidate():
    P = Pair(3, 5, mesh="shift", schedule=(5, 3, 1), smoother="ras", oracle=False)
    f, _ = wl.sinusoid(1, 1, 1)
    X = host(P.gpu.coords(0))
    b = P.gpu.rhs(dev(f(X[0], X[1], X[2])))
    req = sem.TuneRequest()
    base = sem.make_opts(schedule=(5,))
    sem.check(sem.lib().sem_tune_space(5, base, req))
    n_all = req.ncand
    assert n_all >= 12
    req.ncand = 12  # a slice of the space keeps the test short
    xyz = wl.layer_shift_vertices(3, seed=3)
    best, res, req = sem.tune(3, 3, 3, xyz, 1, 5, b, request=req, repeats=2)
    assert 0 <= res.best < 12
    ok = [k for k in range(12) if res.status[k] == 0]
    assert res.best in ok
    assert res.ms[res.best] == min(res.ms[k] for k in ok) or \
        res.ms[res.best] <= 1.01 * min(res.ms[k] for k in ok)
    # the chosen options solve the problem
    S = sem.Solver(3, 3, 3, xyz, 1, 5, opts=best)
    x, info = S.solve(b, rtol=1e-8, maxit=200)
    assert info.converged


@pytest.mark.parametrize("shape,p,sched,sm,prec,fdm,coarse,geom", [
    ((3, 3, 2), 7, (7, 3, 1), sem.SMOOTH_RAS, sem.F32, None, sem.COARSE_AUTO, sem.F32),
    # four elements along x: the FDM and Ax sum their in-workgroup x-faces
    ((4, 2, 2), 7, (7, 3, 1), sem.SMOOTH_RAS, sem.F32, None, sem.COARSE_AUTO, sem.F32),
    ((2, 3, 3), 5, (5, 3, 1), sem.SMOOTH_RAS, sem.F32, sem.BF16, sem.COARSE_AUTO, sem.F32),
    ((3, 2, 2), 5, (5, 1), sem.SMOOTH_ASM, sem.F64, None, sem.COARSE_AUTO, sem.F32),
    ((2, 2, 3), 4, (4, 2, 1), sem.SMOOTH_JACOBI, sem.F32, None, sem.COARSE_PCG, sem.F32),
    # FP16 geometric factors in the p = 7 smoother's A, with and without x-face sums
    ((3, 3, 2), 7, (7, 3, 1), sem.SMOOTH_RAS, sem.F32, None, sem.COARSE_AUTO, sem.F16),
    ((4, 2, 2), 7, (7, 3, 1), sem.SMOOTH_RAS, sem.F32, sem.F16, sem.COARSE_AUTO, sem.F16),
])
def test_joint_lanes_equal_lanes_in_turn(monkeypatch, shape, p, sched, sm, prec, fdm, coarse, geom):
    """The right sides of one problem sharing each operator application and
    V-cycle (nv vectors per launch) give bit-for-bit the results of running the
    lanes one at a time (same iteration counts, same iterates), both converged."""
    import torch
    freqs = [(1, 1, 1), (2, 1, 3), (1, 3, 2)]
    opts = sem.make_opts(schedule=sched, smoother=sm, smoother_prec=prec, batch_rhs=len(freqs),
                         coarse_solver=coarse, fdm_prec=fdm if fdm else prec, geom_prec=geom)
    xyz = wl.sampled_mesh(*shape, sem.gll_nodes(p)[0], wl.sin_map(0.05))
    S = sem.Solver(*shape, xyz, p, p, opts=opts)
    X = host(S.coords(0))
    bs = []
    for fr in freqs:
        f, _ = wl.sinusoid(*fr)
        bs.append(S.rhs(dev(f(X[0], X[1], X[2]))))
    out = {}
    for mode in ("1", "0"):
        monkeypatch.setenv("SEM_BATCH_JOINT", mode)
        xs = [[torch.zeros_like(b) for b in bs]]
        infos = sem.batch_solve([S], [bs], xs, rtol=1e-8, maxit=200)
        assert all(i.converged and i.true_rel_res <= 1e-8 for i in infos)
        out[mode] = ([i.iters for i in infos], [host(x) for x in xs[0]])
    assert out["1"][0] == out["0"][0]
    for a, b in zip(out["1"][1], out["0"][1]):
        np.testing.assert_array_equal(a, b)


def test_batch_record_once_equals_rerecording(monkeypatch):
    """Replaying the first recorded iteration to the end (SEM_BATCH_RECORD_ONCE=1:
    finished problems keep running their V-cycles, their lane kernels return at
    once), or launching every iteration directly (SEM_BATCH_GRAPH=0), gives the
    same iterates as recording again when problems finish."""
    import torch
    probs = [((3, 3, 3), 5, (5, 3, 1)), ((2, 3, 2), 7, (7, 3, 1)), ((4, 2, 2), 3, (3, 1))]
    solvers, bs = [], []
    for shape, p, sched in probs:
        opts = sem.make_opts(schedule=sched, smoother=sem.SMOOTH_RAS, smoother_prec=sem.F32,
                             batch_rhs=2)
        xyz = wl.sampled_mesh(*shape, sem.gll_nodes(p)[0], wl.sin_map(0.05))
        S = sem.Solver(*shape, xyz, p, p, opts=opts)
        X = host(S.coords(0))
        row = []
        for fr in ((1, 1, 1), (3, 1, 2)):
            f, _ = wl.sinusoid(*fr)
            row.append(S.rhs(dev(f(X[0], X[1], X[2]))))
        solvers.append(S)
        bs.append(row)
    out = {}
    for mode, once, graph in (("rerecord", "0", "1"), ("once", "1", "1"), ("direct", "0", "0")):
        monkeypatch.setenv("SEM_BATCH_RECORD_ONCE", once)
        monkeypatch.setenv("SEM_BATCH_GRAPH", graph)
        xs = [[torch.zeros_like(b) for b in row] for row in bs]
        infos = sem.batch_solve(solvers, bs, xs, rtol=1e-8, maxit=200)
        assert all(i.converged for i in infos)
        out[mode] = ([i.iters for i in infos], [host(x) for row in xs for x in row])
    assert len(set(out["rerecord"][0])) > 1  # the lanes finish at different iterations
    for mode in ("once", "direct"):
        assert out[mode][0] == out["rerecord"][0], mode
        for a, b in zip(out[mode][1], out["rerecord"][1]):
            np.testing.assert_array_equal(a, b)
