"""GPU parity at the benchmark's full size (32^3 layer-shift mesh, p = 7),
in the launch configuration the benchmark uses (32768 FDM workgroups, the
XCD remapping of every kernel, the deferred gather-scatter steps of the
Chebyshev updates), against the oracle on element windows:

* the Schwarz smoother (RAS, eqs. 4, 8, 9): the output on one element's nodes
  depends only on its 3x3x3 neighbourhood and on the neighbours' own local
  solves, so the oracle run on the 5x5x5 window around a sampled element
  (clipped at the domain boundary, which keeps its Dirichlet faces) gives
  that element's output exactly;
* the Chebyshev smoother (Algorithm 2, order 2): with b and x supported on
  one element, every intermediate vector stays within a few elements of it,
  so the oracle on a 17^3 window reproduces the whole result, and the GPU
  output outside that window must be exactly zero.
"""
import numpy as np
import pytest

from oracle import cheby as ocheby
from oracle.hierarchy import Level
from pairs import Pair, dev, global_mask, host, rel_err
from paper_2110_07663_amd import sem
from paper_2110_07663_amd import workloads as wl

pytestmark = pytest.mark.gpu

N_FULL, P_FULL = 32, 7
LAMBDA = [26.4, 20.2]    # close to the Arnoldi values of this mesh (RAS)


def _window(n, centre, radius, bc):
    """Elements of the window around `centre` (clipped to the mesh), its
    shape, its first element coordinates and the face conditions of the
    window: the mesh's own where the window reaches the domain boundary,
    Neumann on cut faces (whose elements never see a nonzero value)."""
    c = (centre % n, (centre // n) % n, centre // (n * n))
    lo = [max(0, v - radius) for v in c]
    hi = [min(n - 1, v + radius) for v in c]
    shape = tuple(h - l + 1 for l, h in zip(lo, hi))
    els = np.array([((z * n) + y) * n + x for z in range(lo[2], hi[2] + 1)
                    for y in range(lo[1], hi[1] + 1) for x in range(lo[0], hi[0] + 1)])
    wbc = []
    for d in range(3):
        wbc += [bc[2 * d] if lo[d] == 0 else 0, bc[2 * d + 1] if hi[d] == n - 1 else 0]
    return els, shape, lo, tuple(wbc)


def _window_level(xyz, n, p, centre, radius, bc, smoother):
    els, shape, lo, wbc = _window(n, centre, radius, bc)
    L = Level(*shape, xyz[els], 1, p, wbc, smoother)
    nx = n * p + 1
    gid_full = ((L.num.gz + lo[2] * p) * nx + (L.num.gy + lo[1] * p)) * nx + (L.num.gx + lo[0] * p)
    return L, els, gid_full


@pytest.fixture(scope="module")
def mesh():
    return wl.layer_shift_vertices(N_FULL, seed=3)


def _sample():
    n = N_FULL
    rng = np.random.default_rng(1)
    corners = [0, n - 1, n * n - 1, n ** 3 - 1, (n - 1) * n * n]
    edges_faces = [n // 2, n // 2 * n, n // 2 * (1 + n * n), n * n * (n // 2) + n - 1]
    return corners + edges_faces + [int(v) for v in rng.integers(0, n ** 3, 6)]


@pytest.mark.parametrize("prec,fdm_prec,tol,tol_inf", [
    (sem.F64, sem.F64, 1e-12, 1e-11), (sem.F32, sem.F32, 1e-5, 1e-5),
    (sem.F32, sem.F16, 5e-3, 1e-2), (sem.F32, sem.BF16, 4e-2, 8e-2)])
def test_ras_apply_full_size_sampled(mesh, prec, fdm_prec, tol, tol_inf):
    """sem_apply_S (RAS) at 32^3, p = 7, sampled elements against the oracle's
    5^3 windows: norm-wise over all samples to `tol`, and each element's
    largest error relative to its largest value to `tol_inf` (a localised
    error, e.g. in the halo rows of a box, cannot hide in a norm)."""
    t = __import__("torch")
    n, p = N_FULL, P_FULL
    P = Pair(n, p, mesh="shift", schedule=(p, 3, 1), smoother="ras", smoother_prec=prec,
             fdm_prec=fdm_prec, lambda_override=LAMBDA, oracle=False)
    Lg = P.gpu.levels[0]
    ug = wl.random_global(Lg.nglobal, 17) * global_mask(n, n, n, p, (1,) * 6)
    r = P.gpu.gather(dev(ug))
    if prec == sem.F32:
        r = r.to(t.float32)
    z = P.gpu.apply_S(r)
    N3 = (p + 1) ** 3
    gots, refs, worst = [], [], 0.0
    for e in _sample():
        L, els, gid = _window_level(mesh, n, p, e, 2, (1,) * 6, "ras")
        ref = L.fdm.apply_ras(ug[gid])[list(els).index(e)].reshape(-1)
        got = host(z[e * N3:(e + 1) * N3])
        gots.append(got)
        refs.append(ref)
        worst = max(worst, np.abs(got - ref).max() / np.abs(ref).max())
    err = rel_err(np.concatenate(gots), np.concatenate(refs))
    assert err < tol, err
    assert worst < tol_inf, worst


@pytest.mark.parametrize("prec", [sem.F64, sem.F32])
@pytest.mark.parametrize("centre", [(16, 9, 21), (0, 31, 1)])
def test_chebyshev_ras_full_size_compact_support(mesh, prec, centre):
    """sem_smooth (Cheby-RAS(2), the benchmark's smoother) at 32^3, p = 7 with
    b and x supported on one element: the oracle on the 17^3 window around it
    gives the result; outside the window the GPU result is exactly zero."""
    t = __import__("torch")
    n, p = N_FULL, P_FULL
    P = Pair(n, p, mesh="shift", schedule=(p, 3, 1), smoother="ras", smoother_prec=prec,
             fdm_prec=prec, lambda_override=LAMBDA, oracle=False)
    e0 = (centre[2] * n + centre[1]) * n + centre[0]
    Lg = P.gpu.levels[0]
    # b and x on the nodes of element e0 only (consistent, zero on Dirichlet nodes)
    L, els, gid = _window_level(mesh, n, p, e0, 8, (1,) * 6, "ras")
    own = np.zeros(Lg.nglobal, dtype=bool)
    own[gid[list(els).index(e0)].reshape(-1)] = True
    mask = global_mask(n, n, n, p, (1,) * 6)
    bglob = np.where(own, wl.random_global(Lg.nglobal, 18), 0.0) * mask
    xglob = np.where(own, wl.random_global(Lg.nglobal, 19), 0.0) * mask
    b, x = P.gpu.gather(dev(bglob)), P.gpu.gather(dev(xglob))
    if prec == sem.F32:
        b, x = b.to(t.float32), x.to(t.float32)
    P.gpu.smooth(b, x, level=0)
    got = host(x).reshape(n ** 3, -1)
    L.lmin, L.lmax = ocheby.bounds(LAMBDA[0], 0.1, 1.1)
    L.K = 2
    bo, xo = bglob[gid], xglob[gid]
    ref = (xo + L.smooth(bo, xo)).reshape(len(els), -1)
    inside = got[els]
    err = rel_err(inside, ref)
    assert err < (1e-12 if prec == sem.F64 else 1e-5), err
    outside = np.ones(n ** 3, dtype=bool)
    outside[els] = False
    assert np.count_nonzero(got[outside]) == 0
    # the support really stays inside: the window's outer layer holds zeros
    w_shape = [len(set(v)) for v in (els % n, (els // n) % n, els // (n * n))]
    assert np.abs(ref).max() > 0 and all(s >= 9 for s in w_shape)


@pytest.fixture(scope="module")
def oracle_full(mesh):
    """The oracle's finest level of the full mesh (FP64 operator and right side;
    about 20 s and 6 GB of host memory)."""
    return Level(N_FULL, N_FULL, N_FULL, mesh, 1, P_FULL, (1,) * 6, "jacobi")


@pytest.mark.parametrize("prec", [sem.F32, sem.F64])
def test_pmg_fcg_solve_full_size_oracle_residual(mesh, oracle_full, prec):
    """The benchmark's solve at full size (FCG + pMG (7, 3, 1) Cheby-RAS(2),
    exact coarse solve, tol 1e-8; FP32 smoother or all FP64), in the launch
    shapes the benchmark times: the FCG update over 4096 blocks taking the
    deferred gather-scatter steps of A p, the 32768-wavefront Ax and FDM
    kernels, the finest-level reductions.  The right side matches the oracle's
    (sem_rhs, mask QQ^T B f), and the oracle's FP64 residual of the GPU's
    solution, ||b - A x|| / ||b|| over unique free nodes, is at most 1e-8 and
    equals the residual the solver reports."""
    from oracle.operator import rhs as orhs
    f = wl.sinusoid(1, 1, 1)[0]
    n, p = N_FULL, P_FULL
    opts = sem.make_opts(schedule=(p, 3, 1), smoother=sem.SMOOTH_RAS, cheb_order=2,
                         smoother_prec=prec, fdm_prec=prec, krylov=sem.KRYLOV_FCG)
    s = sem.Solver(n, n, n, mesh, 1, p, opts=opts)
    try:
        X = host(s.coords(0))
        b = s.rhs(dev(f(X[0], X[1], X[2])))
        x, info = s.solve(b, rtol=1e-8, maxit=200)
        bg, xg = host(b), host(x)
    finally:
        s.close()
    L = oracle_full
    bo = orhs(L.num, L.BL, f(L.X[0], L.X[1], L.X[2]))
    assert rel_err(bg.reshape(bo.shape), bo) < 1e-12
    r = bo - L.apply_A(xg.reshape(bo.shape))
    rel = float(np.sqrt(L.wdot(r, r) / L.wdot(bo, bo)))
    assert info.converged and info.iters < 80, info.iters
    assert rel <= 1e-8, rel
    assert abs(rel - info.true_rel_res) <= 1e-3 * rel, (rel, info.true_rel_res)
