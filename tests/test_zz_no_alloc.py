"""sem_solve_static (reduction scratch in the library's static device array,
for callers that cannot allocate) against sem_solve through the C ABI: the
same iterates bit for bit, on two calls in a row, the second on a smaller
problem, in each Krylov form; and the element limit of the static array."""
import ctypes

import numpy as np
import pytest

from pairs import Pair, host
from paper_2110_07663_amd import sem
from paper_2110_07663_amd import workloads as wl

pytestmark = pytest.mark.gpu


def _rhs(P):
    import torch
    f, _ = wl.sinusoid(1, 2, 1)
    X = host(P.gpu.coords(0))
    return P.gpu.rhs(torch.as_tensor(f(X[0], X[1], X[2])).cuda())


@pytest.mark.parametrize("krylov,smoother,prec", [
    (sem.KRYLOV_FCG, "ras", sem.F32), (sem.KRYLOV_PCG, "jacobi", sem.F64),
    (sem.KRYLOV_FGMRES, "ras", sem.F64)])
def test_static_scratch_solve_equals_solve(krylov, smoother, prec):
    import torch
    big = Pair((4, 3, 3), 7, mesh="sin", schedule=(7, 3, 1), smoother=smoother, krylov=krylov,
               smoother_prec=prec, coarse="dense", oracle=False)
    small = Pair((2, 2, 2), 5, mesh="sin", schedule=(5, 3, 1), smoother=smoother, krylov=krylov,
                 smoother_prec=prec, coarse="pcg", oracle=False)
    for P in (big, small):  # two calls in a row, the second on the smaller problem
        b = _rhs(P)
        x_ref, i_ref = P.gpu.solve(b, rtol=1e-10, maxit=100)
        x_st, i_st = P.gpu.solve(b, rtol=1e-10, maxit=100, static_scratch=True)
        torch.cuda.synchronize()
        assert i_st.iters == i_ref.iters and i_st.converged == i_ref.converged == 1
        np.testing.assert_array_equal(host(x_st), host(x_ref))
        assert i_st.true_rel_res == i_ref.true_rel_res <= 1e-10


def test_static_scratch_keeps_the_context_scratch_untouched():
    """The context's own reduction scratch is restored after the call: a plain
    solve after a static one, and a static one with a bad argument, behave as
    before."""
    P = Pair((3, 2, 2), 7, mesh="sin", schedule=(7, 3, 1), smoother="ras", coarse="dense",
             oracle=False)
    b = _rhs(P)
    x0, i0 = P.gpu.solve(b, rtol=1e-9, maxit=100)
    P.gpu.solve(b, rtol=1e-9, maxit=100, static_scratch=True)
    with pytest.raises(sem.SemError):
        P.gpu.solve(b, rtol=-1.0, maxit=100, static_scratch=True)
    x1, i1 = P.gpu.solve(b, rtol=1e-9, maxit=100)
    np.testing.assert_array_equal(host(x0), host(x1))
    assert i0.iters == i1.iters


def test_static_scratch_rejects_meshes_beyond_its_limit():
    """39^3 = 59319 elements exceed the 56832 the array holds: SEM_EINVAL,
    with a message that says so, and nothing launched."""
    import torch
    P = Pair(39, 2, mesh="shift", schedule=(2, 1), smoother="jacobi", oracle=False)
    b = torch.zeros(P.gpu.levels[0].nlocal, dtype=torch.float64, device="cuda")
    x = torch.zeros_like(b)
    info = sem.SolveInfo()
    st = sem.lib().sem_solve_static(P.gpu.ctx, ctypes.c_void_p(b.data_ptr()),
                                    ctypes.c_void_p(x.data_ptr()), 1e-8, 10, ctypes.byref(info),
                                    ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == sem.SEM_EINVAL
    assert b"static scratch" in sem.lib().sem_last_error()
