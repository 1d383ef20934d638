"""Builds the same seeded problem on the HIP library and on the oracle.

The two sides share only the inputs from paper_2110_07663_amd.workloads.
Meshes given by vertices (p_geom = 1) are passed identically; meshes given by
a map sampled at GLL points use each side's own GLL nodes.
"""
import numpy as np

from oracle import gll as ogll
from oracle.hierarchy import Solver as OSolver
from paper_2110_07663_amd import sem
from paper_2110_07663_amd import workloads as wl


def torch():
    import torch as t
    return t


def dev(a, dtype=None):
    t = torch()
    return t.as_tensor(np.ascontiguousarray(a), dtype=dtype or t.float64).cuda()


def host(t):
    return t.detach().cpu().numpy().astype(np.float64)


class Pair:
    """GPU solver + oracle solver for one mesh and option set."""

    def __init__(self, n, p, mesh="sin", schedule=None, bc=(1,) * 6, smoother="jacobi",
                 cheb_order=2, lambda_override=None, smoother_prec=sem.F64, fdm_prec=sem.F64,
                 krylov=sem.KRYLOV_FCG, coarse_tol=1e-10, coarse_maxit=2000, seed=0,
                 precond=sem.PRECOND_PMG, oracle=True, lmin_fac=0.1, lmax_fac=1.1,
                 gmres_restart=20, coarse="pcg", proj_max=0, geom_prec=sem.F32):
        nex, ney, nez = (n, n, n) if np.isscalar(n) else n
        self.shape = (nex, ney, nez)
        schedule = tuple(schedule) if schedule else (p,)
        if mesh == "box":
            xyz_g = xyz_o = wl.box_vertices(nex, ney, nez)
            pg = 1
        elif mesh == "shift":
            assert nex == ney == nez
            xyz_g = xyz_o = wl.layer_shift_vertices(nex, seed=3)
            pg = 1
        elif mesh == "sin":
            pg = p
            xyz_g = wl.sampled_mesh(nex, ney, nez, sem.gll_nodes(p)[0], wl.sin_map(0.05))
            xyz_o = wl.sampled_mesh(nex, ney, nez, ogll.gll_nodes_weights(p)[0], wl.sin_map(0.05))
        else:
            raise ValueError(mesh)
        sm = {"jacobi": sem.SMOOTH_JACOBI, "ras": sem.SMOOTH_RAS, "asm": sem.SMOOTH_ASM}[smoother]
        opts = sem.make_opts(schedule=schedule, smoother=sm, cheb_order=cheb_order,
                             lambda_override=lambda_override, smoother_prec=smoother_prec,
                             fdm_prec=fdm_prec, krylov=krylov, coarse_tol=coarse_tol,
                             coarse_maxit=coarse_maxit, seed=seed, precond=precond,
                             lmin_fac=lmin_fac, lmax_fac=lmax_fac, gmres_restart=gmres_restart,
                             coarse_solver={"pcg": sem.COARSE_PCG, "dense": sem.COARSE_DIRECT}[coarse],
                             proj_max=proj_max, geom_prec=geom_prec)
        self.gpu = sem.Solver(nex, ney, nez, xyz_g, pg, p, bc=bc, opts=opts)
        self.ora = None
        if oracle:
            osched = schedule if precond == sem.PRECOND_PMG else (p,)
            lam = None
            if lambda_override is not None:
                lam = list(lambda_override) + [0] * 8
            self.ora = OSolver(nex, ney, nez, xyz_o, pg, osched, bc=bc, smoother=smoother,
                               cheb_order=cheb_order, lmin_fac=lmin_fac, lmax_fac=lmax_fac,
                               seed=seed, lambda_override=lam, coarse_tol=coarse_tol,
                               coarse_maxit=coarse_maxit, coarse=coarse)

    def random_local(self, seed, level=0, masked=True):
        """The same consistent random E-vector on both sides: (gpu tensor, oracle array)."""
        L = self.gpu.levels[level]
        ug = wl.random_global(L.nglobal, seed)
        if masked:
            ug = ug * global_mask(*self.shape, L.p, self.gpu_bc())
        g = self.gpu.gather(dev(ug), level)
        o = None
        if self.ora is not None:
            o = self.ora.levels[level].num.Q(ug)
        return g, o

    def gpu_bc(self):
        return tuple(int(b) for b in self.gpu.bc)

    def oracle_nodes(self, level=0):
        X = self.ora.levels[level].X
        return X.reshape(3, -1)


def global_mask(nex, ney, nez, p, bc):
    """1 on free global nodes, 0 on Dirichlet faces (index arithmetic only)."""
    nx, ny, nz = nex * p + 1, ney * p + 1, nez * p + 1
    m = np.ones((nz, ny, nx))
    if bc[0]:
        m[:, :, 0] = 0
    if bc[1]:
        m[:, :, -1] = 0
    if bc[2]:
        m[:, 0, :] = 0
    if bc[3]:
        m[:, -1, :] = 0
    if bc[4]:
        m[0] = 0
    if bc[5]:
        m[-1] = 0
    return m.reshape(-1)


def rel_err(a, b):
    a = np.asarray(a, dtype=np.float64).reshape(-1)
    b = np.asarray(b, dtype=np.float64).reshape(-1)
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)
