"""The FP32 RAS local solves in both kernel forms against the oracle: on the
matrix cores (v_mfma_f32_4x4x1 with a broadcast S operand, the default for
2 <= p <= 9) and on the vector pipe (SEM_FDM_MF32=0), for every degree the
matrix-core form takes, every boundary-condition mix, several right sides in
one launch, and the residual form r - rs formed as the box is read.  The
matrix-core form solves 1 or 2 consecutive elements per wavefront
(SEM_FDM_MF32_CHAIN), loading the next one's inputs ahead; the meshes leave
partly filled workgroups and wavefronts.  Inside the smoother the matrix-core
form also takes the x step, and then the y step, of the gather-scatter of A's
output as it reads (SEM_FDM_YSTEP=0: A's gather-scatter takes y and z,
SEM_FDM_XSTEP=0: A's output is assembled first).  Where its output is
assembled next and the elements come in whole groups of four along x, it sums
the x-faces inside each workgroup before the store (SEM_FDM_XFACES=0: the
gather-scatter's x pass covers every face)."""
import numpy as np
import pytest

from pairs import Pair, host, rel_err
from paper_2110_07663_amd import sem

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("mf32,chain,xfaces", [("1", "1", "1"), ("1", "2", "0"), ("1", "1", "0"),
                                               ("0", "1", "1")])
@pytest.mark.parametrize("p,shape,bc", [
    (2, (3, 2, 2), (1,) * 6), (3, (3, 3, 2), (1, 0, 1, 1, 0, 1)), (4, (2, 3, 2), (0,) * 6),
    (5, (3, 2, 3), (1, 1, 0, 1, 1, 0)), (6, (2, 2, 2), (1,) * 6), (7, (4, 3, 2), (0, 1, 1, 0, 1, 1)),
    (7, (1, 1, 1), (1,) * 6), (8, (2, 2, 3), (1,) * 6), (9, (3, 2, 2), (0, 0, 1, 1, 0, 1)),
    # whole groups of four elements along x: the x-faces inside each FDM
    # workgroup are summed before the store, the rest by the gather-scatter
    (3, (8, 2, 1), (1, 0, 0, 1, 1, 1)), (5, (4, 1, 2), (1,) * 6), (9, (4, 2, 1), (0, 1, 1, 1, 0, 0)),
    # zero 1D eigenvalues in x and z (one element, Neumann ends), none in y
    (5, (1, 2, 1), (0,) * 6),
    # a floating box (zero eigenvalue sum): handled by the vector kernel
    (4, (1, 1, 1), (0,) * 6)])
def test_ras_fp32_kernel_forms(monkeypatch, mf32, chain, xfaces, p, shape, bc):
    monkeypatch.setenv("SEM_FDM_MF32", mf32)
    monkeypatch.setenv("SEM_FDM_MF32_CHAIN", chain)
    monkeypatch.setenv("SEM_FDM_XFACES", xfaces)
    t = __import__("torch")
    P = Pair(shape, p, mesh="sin", schedule=(p, 1), smoother="ras", bc=bc,
             smoother_prec=sem.F32, lambda_override=[2.0])
    g, o = P.random_local(41)
    zg = host(P.gpu.apply_S(g.to(t.float32)))
    zo = P.ora.levels[0].apply_S(o).reshape(-1)
    assert rel_err(zg, zo) < 1e-5
    assert np.abs(zg - zo).max() < 1e-5 * np.abs(zo).max()


@pytest.mark.parametrize("p,shape,bc", [
    (3, (3, 2, 2), (1,) * 6), (7, (3, 2, 2), (1,) * 6), (7, (3, 2, 2), (0, 1, 1, 0, 0, 1)),
    (5, (3, 2, 2), (1, 0, 0, 1, 1, 0)), (2, (3, 2, 2), (0,) * 6),
    # interior y-faces on both sides of the middle row, Neumann and Dirichlet y ends
    (7, (2, 3, 3), (1, 1, 0, 1, 1, 0)), (3, (2, 4, 2), (0, 1, 1, 0, 1, 1)),
    # groups of four elements along x (x-face sums inside the FDM workgroups)
    (7, (4, 3, 2), (1, 0, 1, 1, 0, 1)), (3, (8, 2, 2), (0, 1, 0, 1, 1, 0))])
def test_ras_fp32_forms_agree_in_the_smoother(monkeypatch, p, shape, bc):
    """Cheby-RAS smoothing (post-smoothing residual formed as the box is read)
    with each kernel form against the oracle, the matrix-core form taking the
    x and y steps of A's gather-scatter in the FDM, the x step only, or
    neither; Dirichlet and Neumann faces."""
    t = __import__("torch")
    for mf32, chain, xstep, ystep, xfaces in (
            ("1", "1", "1", "1", "1"), ("1", "2", "1", "1", "0"), ("1", "1", "1", "0", "1"),
            ("1", "1", "0", "1", "1"), ("1", "1", "1", "1", "0"), ("0", "1", "1", "1", "1")):
        monkeypatch.setenv("SEM_FDM_MF32", mf32)
        monkeypatch.setenv("SEM_FDM_MF32_CHAIN", chain)
        monkeypatch.setenv("SEM_FDM_XSTEP", xstep)
        monkeypatch.setenv("SEM_FDM_YSTEP", ystep)
        monkeypatch.setenv("SEM_FDM_XFACES", xfaces)
        P = Pair(shape, p, mesh="sin", schedule=(p, 1), smoother="ras", cheb_order=2,
                 smoother_prec=sem.F32, lambda_override=[1.8], bc=bc)
        b, bo = P.random_local(42)
        x, xo = P.random_local(43)
        b, x = b.to(t.float32), x.to(t.float32)
        P.gpu.smooth(b, x, level=0)
        tag = (mf32, chain, xstep, ystep, xfaces)
        assert rel_err(host(x), P.ora.smooth(bo, xo, level=0)) < 1e-5, tag


@pytest.mark.parametrize("fdm_prec,tol", [(sem.F16, 5e-3), (sem.BF16, 4e-2)])
@pytest.mark.parametrize("mf16,xfaces", [("1", "1"), ("1", "0"), ("0", "1")])
@pytest.mark.parametrize("p,shape,bc", [
    (2, (3, 2, 2), (1,) * 6), (3, (8, 2, 1), (1, 0, 0, 1, 1, 1)), (5, (3, 2, 3), (1, 1, 0, 1, 1, 0)),
    (7, (4, 3, 2), (0, 1, 1, 0, 1, 1)), (7, (1, 1, 1), (1,) * 6), (9, (4, 2, 1), (0, 1, 1, 1, 0, 0)),
    (5, (1, 2, 1), (0,) * 6)])
def test_ras_16bit_kernel_forms(monkeypatch, fdm_prec, tol, mf16, xfaces, p, shape, bc):
    """FP16 / BF16 operands with FP32 accumulation: the matrix-core line kernel
    in its 4x4x4 form (the default; the box and the eigenvalue-scaled tensor
    brought into [0.5, 1) by powers of two) and the 16x16x16 tile kernel
    (SEM_FDM_MF16=0), against the oracle, norm-wise and entry by entry
    relative to the largest entry."""
    monkeypatch.setenv("SEM_FDM_MF16", mf16)
    monkeypatch.setenv("SEM_FDM_XFACES", xfaces)
    t = __import__("torch")
    P = Pair(shape, p, mesh="sin", schedule=(p, 1), smoother="ras", bc=bc,
             smoother_prec=sem.F32, fdm_prec=fdm_prec, lambda_override=[2.0])
    g, o = P.random_local(41)
    zg = host(P.gpu.apply_S(g.to(t.float32)))
    zo = P.ora.levels[0].apply_S(o).reshape(-1)
    assert rel_err(zg, zo) < tol
    assert np.abs(zg - zo).max() < 2 * tol * np.abs(zo).max()


@pytest.mark.parametrize("fdm_prec,tol", [(sem.F16, 5e-3), (sem.BF16, 4e-2)])
@pytest.mark.parametrize("p,shape,bc", [
    (3, (3, 2, 2), (1,) * 6), (7, (2, 3, 3), (1, 1, 0, 1, 1, 0)), (7, (4, 3, 2), (1, 0, 1, 1, 0, 1))])
def test_ras_16bit_forms_agree_in_the_smoother(monkeypatch, fdm_prec, tol, p, shape, bc):
    """Cheby-RAS smoothing with 16-bit FDM operands: the line kernel taking the
    x and y steps of A's gather-scatter (or the x step only, or neither) and
    forming the post-smoothing residual as it reads, and the tile kernel,
    against the oracle."""
    t = __import__("torch")
    for mf16, xstep, ystep, xfaces in (("1", "1", "1", "1"), ("1", "1", "0", "0"),
                                       ("1", "0", "1", "1"), ("0", "1", "1", "1")):
        monkeypatch.setenv("SEM_FDM_MF16", mf16)
        monkeypatch.setenv("SEM_FDM_XSTEP", xstep)
        monkeypatch.setenv("SEM_FDM_YSTEP", ystep)
        monkeypatch.setenv("SEM_FDM_XFACES", xfaces)
        P = Pair(shape, p, mesh="sin", schedule=(p, 1), smoother="ras", cheb_order=2,
                 smoother_prec=sem.F32, fdm_prec=fdm_prec, lambda_override=[1.8], bc=bc)
        b, bo = P.random_local(42)
        x, xo = P.random_local(43)
        b, x = b.to(t.float32), x.to(t.float32)
        P.gpu.smooth(b, x, level=0)
        tag = (mf16, xstep, ystep, xfaces)
        assert rel_err(host(x), P.ora.smooth(bo, xo, level=0)) < tol, tag
