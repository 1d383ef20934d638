"""ctypes binding of libsem.so (C ABI in include/sem.h).

Argument marshalling only: device buffers are torch CUDA tensors whose data
pointers are handed to the library, together with torch's current HIP stream.
Every computation happens inside the library's kernels.  If the library is
missing, lib() raises; there is no other implementation to fall back to.
"""
import atexit
import ctypes
import os
import weakref

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libsem.so")

SEM_OK, SEM_EINVAL, SEM_EWORKSPACE, SEM_EHIP, SEM_ENOCONV, SEM_ENAN, SEM_EUNSUPPORTED, SEM_EGEOM = \
    0, -1, -2, -3, -4, -5, -6, -7
F64, F32, BF16, F16 = 0, 1, 2, 3
SMOOTH_JACOBI, SMOOTH_RAS, SMOOTH_ASM = 0, 1, 2
KRYLOV_PCG, KRYLOV_FCG, KRYLOV_FGMRES = 0, 1, 2
PRECOND_PMG, PRECOND_JACOBI = 0, 1
COARSE_AUTO, COARSE_PCG, COARSE_DIRECT = -1, 0, 1

_STATUS_NAMES = {0: "SEM_OK", -1: "SEM_EINVAL", -2: "SEM_EWORKSPACE", -3: "SEM_EHIP",
                 -4: "SEM_ENOCONV", -5: "SEM_ENAN", -6: "SEM_EUNSUPPORTED", -7: "SEM_EGEOM"}

EXPORTS = ("sem_default_opts", "sem_last_error", "sem_plan", "sem_setup", "sem_destroy",
           "sem_level_info", "sem_gll", "sem_coords", "sem_gather", "sem_rhs", "sem_apply_A",
           "sem_apply_S", "sem_smooth", "sem_prolong", "sem_restrict", "sem_vcycle", "sem_solve",
           "sem_profile", "sem_profile_read", "sem_tune_space", "sem_tune_plan", "sem_tune",
           "sem_batch_solve", "sem_projection_reset", "sem_solve_static")
TUNE_MAX = 96
PROF_NAMES = ("ax64", "ax32", "fdm", "gs64", "gs32", "coarse", "vcycle")


class Mesh(ctypes.Structure):
    _fields_ = [("nex", ctypes.c_int32), ("ney", ctypes.c_int32), ("nez", ctypes.c_int32),
                ("p_geom", ctypes.c_int32), ("xyz", ctypes.POINTER(ctypes.c_double))]


class Opts(ctypes.Structure):
    _fields_ = [("nlevels", ctypes.c_int32), ("p_levels", ctypes.c_int32 * 8),
                ("precond", ctypes.c_int32), ("smoother", ctypes.c_int32),
                ("cheb_order", ctypes.c_int32), ("lmin_fac", ctypes.c_double),
                ("lmax_fac", ctypes.c_double), ("arnoldi_steps", ctypes.c_int32),
                ("seed", ctypes.c_uint64), ("lambda_override", ctypes.c_double * 8),
                ("smoother_prec", ctypes.c_int32), ("fdm_prec", ctypes.c_int32),
                ("krylov", ctypes.c_int32), ("gmres_restart", ctypes.c_int32),
                ("coarse_tol", ctypes.c_double), ("coarse_maxit", ctypes.c_int32),
                ("ax_variant", ctypes.c_int32), ("batch_rhs", ctypes.c_int32),
                ("coarse_solver", ctypes.c_int32), ("proj_max", ctypes.c_int32),
                ("geom_prec", ctypes.c_int32)]


class SolveInfo(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("converged", ctypes.c_int32),
                ("rel_res", ctypes.c_double), ("true_rel_res", ctypes.c_double),
                ("r0_norm", ctypes.c_double), ("coarse_iters", ctypes.c_int32),
                ("lambda_tilde", ctypes.c_double * 8)]


class LevelDesc(ctypes.Structure):
    _fields_ = [("p", ctypes.c_int32), ("N", ctypes.c_int32), ("E", ctypes.c_int64),
                ("nlocal", ctypes.c_int64), ("nglobal", ctypes.c_int64),
                ("nshared", ctypes.c_int64), ("lmin", ctypes.c_double), ("lmax", ctypes.c_double),
                ("nmembers", ctypes.c_int64)]


class TuneRequest(ctypes.Structure):
    _fields_ = [("ncand", ctypes.c_int32), ("cand", Opts * TUNE_MAX), ("repeats", ctypes.c_int32),
                ("rtol", ctypes.c_double), ("maxit", ctypes.c_int32)]


class TuneResult(ctypes.Structure):
    _fields_ = [("best", ctypes.c_int32), ("ms", ctypes.c_double * TUNE_MAX),
                ("setup_ms", ctypes.c_double * TUNE_MAX), ("iters", ctypes.c_int32 * TUNE_MAX),
                ("status", ctypes.c_int32 * TUNE_MAX)]


class SemError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{_STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


_lib = None
_live = weakref.WeakSet()  # contexts not closed yet


@atexit.register
def _close_all():
    """Destroy every context still open while the interpreter (and with it the
    HIP runtime) is intact, instead of from object finalisers at teardown."""
    for s in list(_live):
        try:
            s.close()
        except Exception:
            pass


def lib():
    """Load libsem.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_2110_07663_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, dp = ctypes.c_void_p, ctypes.c_int32, ctypes.c_double
        L.sem_default_opts.argtypes = [ctypes.POINTER(Opts)]
        L.sem_default_opts.restype = None
        L.sem_last_error.restype = ctypes.c_char_p
        L.sem_plan.argtypes = [ctypes.POINTER(Mesh), i32, ctypes.POINTER(ctypes.c_int8),
                               ctypes.POINTER(Opts), ctypes.POINTER(ctypes.c_size_t)]
        L.sem_setup.argtypes = [ctypes.POINTER(Mesh), i32, ctypes.POINTER(ctypes.c_int8),
                                ctypes.POINTER(Opts), vp, ctypes.c_size_t, vp, ctypes.POINTER(vp)]
        L.sem_destroy.argtypes = [vp]
        L.sem_level_info.argtypes = [vp, i32, ctypes.POINTER(LevelDesc)]
        L.sem_gll.argtypes = [i32, vp, vp, vp]
        L.sem_coords.argtypes = [vp, i32, vp, vp]
        L.sem_gather.argtypes = [vp, i32, vp, vp, vp]
        L.sem_rhs.argtypes = [vp, vp, vp, vp]
        for name in ("sem_apply_A", "sem_apply_S", "sem_smooth", "sem_prolong", "sem_restrict"):
            getattr(L, name).argtypes = [vp, i32, i32, vp, vp, vp]
        L.sem_vcycle.argtypes = [vp, vp, vp, vp]
        L.sem_solve.argtypes = [vp, vp, vp, dp, i32, ctypes.POINTER(SolveInfo), vp]
        L.sem_solve_static.argtypes = [vp, vp, vp, dp, i32, ctypes.POINTER(SolveInfo), vp]
        L.sem_tune_space.argtypes = [i32, ctypes.POINTER(Opts), ctypes.POINTER(TuneRequest)]
        L.sem_tune_plan.argtypes = [ctypes.POINTER(Mesh), i32, ctypes.POINTER(ctypes.c_int8),
                                    ctypes.POINTER(TuneRequest), ctypes.POINTER(ctypes.c_size_t)]
        L.sem_tune.argtypes = [ctypes.POINTER(Mesh), i32, ctypes.POINTER(ctypes.c_int8),
                               ctypes.POINTER(TuneRequest), vp, vp, vp, ctypes.c_size_t, vp,
                               ctypes.POINTER(TuneResult)]
        L.sem_batch_solve.argtypes = [i32, ctypes.POINTER(vp), i32, ctypes.POINTER(vp),
                                      ctypes.POINTER(vp), dp, i32, i32, ctypes.POINTER(SolveInfo), vp]
        L.sem_profile.argtypes = [vp, i32]
        L.sem_projection_reset.argtypes = [vp]
        L.sem_profile_read.argtypes = [vp, ctypes.POINTER(ctypes.c_double),
                                       ctypes.POINTER(ctypes.c_int64)]
        for name in EXPORTS:
            if name not in ("sem_default_opts", "sem_last_error"):
                getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def check(status, allow=()):
    if status != SEM_OK and status not in allow:
        raise SemError(status, lib().sem_last_error().decode())
    return status


def default_opts():
    o = Opts()
    lib().sem_default_opts(ctypes.byref(o))
    return o


def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def gll_nodes(p):
    """GLL nodes (and weights) of degree p computed by the library, as numpy arrays."""
    import torch
    buf = torch.empty(2 * (p + 1), dtype=torch.float64, device="cuda")
    check(lib().sem_gll(p, _ptr(buf), ctypes.c_void_p(buf.data_ptr() + 8 * (p + 1)), _stream()))
    h = buf.cpu().numpy()
    return h[:p + 1].copy(), h[p + 1:].copy()


def tune(nex, ney, nez, xyz, p_geom, p, b, bc=(1, 1, 1, 1, 1, 1), base=None, request=None,
         repeats=3, rtol=1e-8, maxit=200):
    """Exhaustive search (library side) over the pMG space; returns (best Opts, result, request).

    b is the FP64 right side on the finest level (an E-vector shared by all candidates).
    """
    import torch
    L = lib()
    xyz = np.ascontiguousarray(xyz, dtype=np.float64)
    mesh = Mesh(nex, ney, nez, p_geom, xyz.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    bcs = (ctypes.c_int8 * 6)(*[int(v) for v in bc])
    if request is None:
        request = TuneRequest()
        base = base if base is not None else make_opts(schedule=(p,))
        check(L.sem_tune_space(p, ctypes.byref(base), ctypes.byref(request)))
    request.repeats, request.rtol, request.maxit = repeats, rtol, maxit
    nbytes = ctypes.c_size_t(0)
    check(L.sem_tune_plan(ctypes.byref(mesh), p, bcs, ctypes.byref(request), ctypes.byref(nbytes)))
    ws = torch.empty(nbytes.value, dtype=torch.uint8, device="cuda")
    x = torch.empty_like(b)
    res = TuneResult()
    check(L.sem_tune(ctypes.byref(mesh), p, bcs, ctypes.byref(request), _ptr(b), _ptr(x), _ptr(ws),
                     nbytes, _stream(), ctypes.byref(res)))
    best = Opts()
    ctypes.pointer(best)[0] = request.cand[res.best]
    return best, res, request


def batch_solve(solvers, bs, xs, rtol=1e-8, maxit=200, iters_per_launch=4, allow_noconv=False):
    """Solve every (solver i, right side k) pair together: bs[i][k] -> xs[i][k] (in place).

    Returns the list of SolveInfo (problem-major).  Each solver must have been
    set up with batch_rhs >= the number of right sides.
    """
    nctx = len(solvers)
    nrhs = len(bs[0])
    ctxs = (ctypes.c_void_p * nctx)(*[s.ctx for s in solvers])
    bp = (ctypes.c_void_p * (nctx * nrhs))(*[b.data_ptr() for row in bs for b in row])
    xp = (ctypes.c_void_p * (nctx * nrhs))(*[x.data_ptr() for row in xs for x in row])
    infos = (SolveInfo * (nctx * nrhs))()
    st = lib().sem_batch_solve(nctx, ctxs, nrhs, bp, xp, rtol, maxit, iters_per_launch, infos,
                               _stream())
    check(st, allow=(SEM_ENOCONV,) if allow_noconv else ())
    return list(infos)


def make_opts(schedule=(7, 3, 1), smoother=SMOOTH_JACOBI, cheb_order=2, lmin_fac=0.1,
              lmax_fac=1.1, arnoldi_steps=10, seed=0, lambda_override=None, smoother_prec=F64,
              fdm_prec=F64, krylov=KRYLOV_FCG, gmres_restart=20, coarse_tol=1e-10,
              coarse_maxit=2000, precond=PRECOND_PMG, ax_variant=-1, batch_rhs=0,
              coarse_solver=-1, proj_max=0, geom_prec=F32):
    o = default_opts()
    o.nlevels = len(schedule)
    for l, p in enumerate(schedule):
        o.p_levels[l] = p
    o.precond, o.smoother, o.cheb_order = precond, smoother, cheb_order
    o.lmin_fac, o.lmax_fac, o.arnoldi_steps, o.seed = lmin_fac, lmax_fac, arnoldi_steps, seed
    for l in range(8):
        o.lambda_override[l] = 0.0
    if lambda_override is not None:
        for l, v in enumerate(lambda_override):
            o.lambda_override[l] = float(v)
    o.smoother_prec, o.fdm_prec, o.krylov = smoother_prec, fdm_prec, krylov
    o.gmres_restart, o.coarse_tol, o.coarse_maxit = gmres_restart, coarse_tol, coarse_maxit
    o.ax_variant = ax_variant
    o.batch_rhs = batch_rhs
    o.coarse_solver = coarse_solver
    o.proj_max = proj_max
    o.geom_prec = geom_prec
    return o


class Solver:
    """One set-up problem: owns the torch workspace and the library context."""

    def __init__(self, nex, ney, nez, xyz, p_geom, p, bc=(1, 1, 1, 1, 1, 1), opts=None):
        import torch
        self._torch = torch
        L = lib()
        xyz = np.ascontiguousarray(xyz, dtype=np.float64)
        E = nex * ney * nez
        if xyz.shape != (E, (p_geom + 1) ** 3, 3):
            raise ValueError(f"xyz must have shape {(E, (p_geom + 1) ** 3, 3)}, got {xyz.shape}")
        self._xyz = xyz
        self.mesh = Mesh(nex, ney, nez, p_geom, xyz.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
        self.bc = (ctypes.c_int8 * 6)(*[int(b) for b in bc])
        self.opts = opts if opts is not None else make_opts(schedule=(p,))
        self.p = p
        nbytes = ctypes.c_size_t(0)
        check(L.sem_plan(ctypes.byref(self.mesh), p, self.bc, ctypes.byref(self.opts),
                         ctypes.byref(nbytes)))
        self.workspace_bytes = nbytes.value
        self.workspace = torch.empty(nbytes.value, dtype=torch.uint8, device="cuda")
        ctx = ctypes.c_void_p(0)
        check(L.sem_setup(ctypes.byref(self.mesh), p, self.bc, ctypes.byref(self.opts),
                          _ptr(self.workspace), nbytes, _stream(), ctypes.byref(ctx)))
        self.ctx = ctx
        _live.add(self)
        self.levels = [self.level_info(l) for l in range(self.nlevels)]

    @property
    def nlevels(self):
        return 1 if self.opts.precond == PRECOND_JACOBI else self.opts.nlevels

    def close(self):
        """Release the library context (synchronises the device first, so that
        no enqueued work still uses its workspace)."""
        if self.ctx:
            self._torch.cuda.synchronize()
            check(lib().sem_destroy(self.ctx))
            self.ctx = None
            _live.discard(self)

    def projection_reset(self):
        """Forget the prior solutions kept for opts.proj_max."""
        check(lib().sem_projection_reset(self.ctx))

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def level_info(self, level):
        d = LevelDesc()
        check(lib().sem_level_info(self.ctx, level, ctypes.byref(d)))
        return d

    def _vec(self, level=0, dtype=None):
        torch = self._torch
        return torch.empty(self.levels[level].nlocal, dtype=dtype or torch.float64, device="cuda")

    def coords(self, level=0):
        out = self._torch.empty(3, self.levels[level].nlocal, dtype=self._torch.float64, device="cuda")
        check(lib().sem_coords(self.ctx, level, _ptr(out), _stream()))
        return out

    def gather(self, u_global, level=0):
        out = self._vec(level)
        check(lib().sem_gather(self.ctx, level, _ptr(u_global), _ptr(out), _stream()))
        return out

    def rhs(self, f_local):
        out = self._vec(0)
        check(lib().sem_rhs(self.ctx, _ptr(f_local), _ptr(out), _stream()))
        return out

    def _prec_of(self, t):
        return F64 if t.dtype == self._torch.float64 else F32

    def apply_A(self, u, level=0, out=None):
        out = self._torch.empty_like(u) if out is None else out
        check(lib().sem_apply_A(self.ctx, level, self._prec_of(u), _ptr(u), _ptr(out), _stream()))
        return out

    def apply_S(self, r, level=0, out=None):
        out = self._torch.empty_like(r) if out is None else out
        check(lib().sem_apply_S(self.ctx, level, self._prec_of(r), _ptr(r), _ptr(out), _stream()))
        return out

    def smooth(self, b, x, level=0):
        """In place: x <- x + Cheb(b - A x)."""
        check(lib().sem_smooth(self.ctx, level, self._prec_of(b), _ptr(b), _ptr(x), _stream()))
        return x

    def prolong(self, xc, xf, level=0):
        check(lib().sem_prolong(self.ctx, level, self._prec_of(xc), _ptr(xc), _ptr(xf), _stream()))
        return xf

    def restrict(self, rf, level=0, out=None):
        out = self._vec(level + 1, rf.dtype) if out is None else out
        check(lib().sem_restrict(self.ctx, level, self._prec_of(rf), _ptr(rf), _ptr(out), _stream()))
        return out

    def vcycle(self, r, out=None):
        out = self._torch.empty_like(r) if out is None else out
        check(lib().sem_vcycle(self.ctx, _ptr(r), _ptr(out), _stream()))
        return out

    def profile(self, enable=True, kinds=None):
        """Event timing of the finest level's kernel classes; kinds: names of
        PROF_NAMES to record (None: all)."""
        if not enable:
            mask = 0
        elif kinds is None:
            mask = 1
        else:
            mask = sum(2 << PROF_NAMES.index(k) for k in kinds)
        check(lib().sem_profile(self.ctx, mask))

    def profile_read(self):
        """{kernel class: (total ms, launches)} of the finest level since profile(True)."""
        ms = (ctypes.c_double * len(PROF_NAMES))()
        n = (ctypes.c_int64 * len(PROF_NAMES))()
        check(lib().sem_profile_read(self.ctx, ms, n))
        return {k: (ms[i], n[i]) for i, k in enumerate(PROF_NAMES)}

    def solve(self, b, x=None, rtol=1e-8, maxit=500, allow_noconv=False, static_scratch=False):
        """Returns (x, SolveInfo); x is updated in place when given.
        static_scratch: call sem_solve_static (reduction scratch in the
        library's static device array) instead of sem_solve."""
        x = self._torch.zeros_like(b) if x is None else x
        info = SolveInfo()
        fn = lib().sem_solve_static if static_scratch else lib().sem_solve
        st = fn(self.ctx, _ptr(b), _ptr(x), rtol, maxit, ctypes.byref(info), _stream())
        check(st, allow=(SEM_ENOCONV,) if allow_noconv else ())
        return x, info
