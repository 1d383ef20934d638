"""The C-ABI library loads and exports every function include/sem.h declares (CPU only)."""
import ctypes
import os
import re

import pytest

from paper_2110_07663_amd import sem

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "sem.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:sem_status|void|const char \*)\s*(sem_\w+)\s*\(", text, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_paper_calls():
    names = declared_functions()
    for required in ("sem_setup", "sem_apply_A", "sem_smooth", "sem_vcycle", "sem_solve"):
        assert required in names


@pytest.mark.skipif(not os.path.exists(sem.LIB_PATH), reason="libsem.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(sem.LIB_PATH)
    for name in declared_functions():
        assert hasattr(lib, name), name
    assert sorted(declared_functions()) == sorted(sem.EXPORTS)


@pytest.mark.skipif(not os.path.exists(sem.LIB_PATH), reason="libsem.so not built")
def test_host_side_validation_without_gpu():
    """Planning is host-only: bad inputs are rejected with status codes, no GPU needed."""
    import numpy as np
    from paper_2110_07663_amd import workloads as wl
    L = sem.lib()
    xyz = np.ascontiguousarray(wl.box_vertices(2, 2, 2))
    mesh = sem.Mesh(2, 2, 2, 1, xyz.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    bc = (ctypes.c_int8 * 6)(1, 1, 1, 1, 1, 1)
    n = ctypes.c_size_t(0)
    o = sem.make_opts(schedule=(7, 3, 1))
    assert L.sem_plan(ctypes.byref(mesh), 7, bc, ctypes.byref(o), ctypes.byref(n)) == sem.SEM_OK
    assert n.value > 0
    o_bad = sem.make_opts(schedule=(7, 5, 6))
    assert L.sem_plan(ctypes.byref(mesh), 7, bc, ctypes.byref(o_bad), ctypes.byref(n)) == sem.SEM_EINVAL
    assert b"decreasing" in L.sem_last_error()
    o_hi = sem.make_opts(schedule=(12, 3, 1))
    assert L.sem_plan(ctypes.byref(mesh), 12, bc, ctypes.byref(o_hi), ctypes.byref(n)) == sem.SEM_EUNSUPPORTED
    o_p0 = sem.make_opts(schedule=(5, 3, 1))
    assert L.sem_plan(ctypes.byref(mesh), 7, bc, ctypes.byref(o_p0), ctypes.byref(n)) == sem.SEM_EINVAL
    o_proj = sem.make_opts(schedule=(7, 3, 1), proj_max=33)
    assert L.sem_plan(ctypes.byref(mesh), 7, bc, ctypes.byref(o_proj), ctypes.byref(n)) == sem.SEM_EINVAL
    assert b"proj_max" in L.sem_last_error()
    o_proj.proj_max = 10  # room for 10 prior solutions and their products with A
    n_proj = ctypes.c_size_t(0)
    assert L.sem_plan(ctypes.byref(mesh), 7, bc, ctypes.byref(o_proj), ctypes.byref(n_proj)) == sem.SEM_OK
    n_plain = ctypes.c_size_t(0)
    assert L.sem_plan(ctypes.byref(mesh), 7, bc, ctypes.byref(o), ctypes.byref(n_plain)) == sem.SEM_OK
    assert n_proj.value >= n_plain.value + 20 * 8 * 8 ** 3 * 8  # 20 vectors of E (p+1)^3 doubles
    # FP16 geometric factors: only under the FP32 smoother; 12 more bytes per p = 7 point
    o_g16 = sem.make_opts(schedule=(7, 3, 1), smoother_prec=sem.F64, geom_prec=sem.F16)
    assert L.sem_plan(ctypes.byref(mesh), 7, bc, ctypes.byref(o_g16), ctypes.byref(n)) == sem.SEM_EINVAL
    assert b"geom" in L.sem_last_error().lower()
    o_g16.geom_prec = 7
    assert L.sem_plan(ctypes.byref(mesh), 7, bc, ctypes.byref(o_g16), ctypes.byref(n)) == sem.SEM_EINVAL
    o_f32 = sem.make_opts(schedule=(7, 3, 1), smoother_prec=sem.F32)
    o_g16 = sem.make_opts(schedule=(7, 3, 1), smoother_prec=sem.F32, geom_prec=sem.F16)
    n_f32, n_g16 = ctypes.c_size_t(0), ctypes.c_size_t(0)
    assert L.sem_plan(ctypes.byref(mesh), 7, bc, ctypes.byref(o_f32), ctypes.byref(n_f32)) == sem.SEM_OK
    assert L.sem_plan(ctypes.byref(mesh), 7, bc, ctypes.byref(o_g16), ctypes.byref(n_g16)) == sem.SEM_OK
    assert n_g16.value >= n_f32.value + 8 * 8 ** 3 * 12
    bad_bc = (ctypes.c_int8 * 6)(1, 1, 2, 1, 1, 1)
    assert L.sem_plan(ctypes.byref(mesh), 7, bad_bc, ctypes.byref(o), ctypes.byref(n)) == sem.SEM_EINVAL
    # plan grows with the problem
    n2 = ctypes.c_size_t(0)
    xyz3 = np.ascontiguousarray(wl.box_vertices(4, 4, 4))
    mesh3 = sem.Mesh(4, 4, 4, 1, xyz3.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    assert L.sem_plan(ctypes.byref(mesh3), 7, bc, ctypes.byref(o), ctypes.byref(n2)) == sem.SEM_OK
    assert n2.value > n.value


@pytest.mark.skipif(not os.path.exists(sem.LIB_PATH), reason="libsem.so not built")
def test_tune_space_follows_the_papers_table():
    """Sec. 5 table: p=7 -> Cheby-ASM/RAS (7,3,1), Cheby-Jac (7,5,3,1); p=9 -> (9,5,1), (9,7,5,1)."""
    L = sem.lib()
    for p, short, long_ in ((7, [7, 3, 1], [7, 5, 3, 1]), (9, [9, 5, 1], [9, 7, 5, 1])):
        req = sem.TuneRequest()
        base = sem.make_opts(schedule=(p,))
        assert L.sem_tune_space(p, ctypes.byref(base), ctypes.byref(req)) == sem.SEM_OK
        seen = set()
        for k in range(req.ncand):
            o = req.cand[k]
            sched = [o.p_levels[l] for l in range(o.nlevels)]
            if o.smoother == sem.SMOOTH_JACOBI:
                assert sched == long_
                assert o.fdm_prec != sem.F16
            else:
                assert sched == short
            if o.geom_prec == sem.F16:  # FP16 factors: FP32 smoother; one-wavefront Ax at p = 7
                assert o.smoother_prec == sem.F32 and (p != 7 or o.ax_variant >= 1)
            seen.add((o.smoother, o.cheb_order, o.smoother_prec, o.fdm_prec, o.ax_variant,
                      o.geom_prec))
        assert len(seen) == req.ncand  # no duplicates
        orders = {s[1] for s in seen}
        assert orders == {1, 2, 3}
        assert {s[0] for s in seen} == {sem.SMOOTH_ASM, sem.SMOOTH_RAS, sem.SMOOTH_JACOBI}
        assert req.ncand == (90 if p == 7 else 33)
    # plan covers the largest candidate
    import numpy as np
    from paper_2110_07663_amd import workloads as wl
    xyz = np.ascontiguousarray(wl.box_vertices(2, 2, 2))
    mesh = sem.Mesh(2, 2, 2, 1, xyz.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    bc = (ctypes.c_int8 * 6)(1, 1, 1, 1, 1, 1)
    req = sem.TuneRequest()
    base = sem.make_opts(schedule=(7,))
    L.sem_tune_space(7, ctypes.byref(base), ctypes.byref(req))
    big = ctypes.c_size_t(0)
    assert L.sem_tune_plan(ctypes.byref(mesh), 7, bc, ctypes.byref(req), ctypes.byref(big)) == 0
    for k in range(req.ncand):
        n = ctypes.c_size_t(0)
        assert L.sem_plan(ctypes.byref(mesh), 7, bc, ctypes.byref(req.cand[k]), ctypes.byref(n)) == 0
        assert n.value <= big.value
