"""Edge cases of the GPU path against the oracle: a single element, meshes one
element thick (missing Schwarz neighbours, 2-node coarse planes), the highest
supported degree, and element counts that leave the matrix-core FDM's last
4-element block partly empty."""
import numpy as np
import pytest

from pairs import Pair, host, rel_err
from paper_2110_07663_amd import sem

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    return torch


@pytest.mark.parametrize("p", [3, 7])
def test_single_element(p):
    """One element, all faces Dirichlet: the p = 1 level has no free node."""
    P = Pair((1, 1, 1), p, mesh="sin", schedule=(p, 1), smoother="ras", lambda_override=[1.5],
             coarse="dense")
    g, o = P.random_local(61)
    assert rel_err(host(P.gpu.apply_A(g)), P.ora.levels[0].apply_A(o)) < 1e-12
    assert rel_err(host(P.gpu.apply_S(g)), P.ora.levels[0].apply_S(o)) < 1e-12
    assert rel_err(host(P.gpu.vcycle(g)), P.ora.vcycle(o)) < 1e-12


@pytest.mark.parametrize("shape,bc", [((1, 4, 3), (1,) * 6), ((4, 1, 2), (1, 0, 1, 1, 0, 1)),
                                      ((3, 2, 1), (0, 1, 1, 0, 1, 1))])
def test_thin_meshes(shape, bc):
    """One element thick in some direction: Schwarz boxes miss neighbours, the
    exact coarse solve sees planes of 2 nodes or a single plane pair."""
    P = Pair(shape, 5, mesh="sin", schedule=(5, 3, 1), smoother="ras", bc=bc,
             lambda_override=[1.6, 1.8], coarse="dense")
    for seed in (62, 63):
        g, o = P.random_local(seed)
        assert rel_err(host(P.gpu.vcycle(g)), P.ora.vcycle(o)) < 1e-12


def test_highest_degree_fdm():
    """p = 10 (pbar = 13): FP64 and FP32 line kernels, FP16 matrix cores."""
    t = _torch()
    P = Pair((2, 2, 2), 10, mesh="sin", schedule=(10, 1), smoother="ras", lambda_override=[1.5])
    g, o = P.random_local(64)
    ref = P.ora.levels[0].apply_S(o)
    assert rel_err(host(P.gpu.apply_S(g)), ref) < 1e-12
    P32 = Pair((2, 2, 2), 10, mesh="sin", schedule=(10, 1), smoother="ras", lambda_override=[1.5],
               smoother_prec=sem.F32, oracle=False)
    assert rel_err(host(P32.gpu.apply_S(g.to(t.float32))), ref) < 1e-5
    P16 = Pair((2, 2, 2), 10, mesh="sin", schedule=(10, 1), smoother="ras", lambda_override=[1.5],
               smoother_prec=sem.F32, fdm_prec=sem.F16, oracle=False)
    assert rel_err(host(P16.gpu.apply_S(g.to(t.float32))), ref) < 5e-3


@pytest.mark.parametrize("shape", [(5, 2, 1), (3, 3, 1)])
def test_mfma_fdm_partial_block(shape):
    """E = 10 and 9: the last block of four elements is partly empty."""
    t = _torch()
    P = Pair(shape, 7, mesh="sin", schedule=(7, 1), smoother="ras", lambda_override=[1.5],
             smoother_prec=sem.F32, fdm_prec=sem.BF16)
    g, o = P.random_local(65)
    ref = P.ora.levels[0].apply_S(o)
    assert rel_err(host(P.gpu.apply_S(g.to(t.float32))), ref) < 4e-2
    assert np.all(np.isfinite(host(P.gpu.apply_S(g.to(t.float32)))))
