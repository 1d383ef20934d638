"""Structured hex mesh numbering and the Boolean gather Q (oracle, test-only).

Follows Sec. 2.1: nodes shared by adjacent elements carry one global value;
the map from global to element-local values is a Boolean matrix Q with
u_L = Q u, and the assembled operators are Q^T A_L Q and Q^T B_L Q.

Conventions (the paper fixes none; these are this project's readings):
  * elements of an nex x ney x nez grid, e = (ez*ney + ey)*nex + ex;
  * local node (i, j, k) of an element, i fastest: local index (k*N + j)*N + i
    with N = p + 1; E-vectors are arrays of shape [E, N, N, N] indexed
    [e, k, j, i];
  * global node grid of (nex*p+1) x (ney*p+1) x (nez*p+1) points,
    gid = ((ez*p + k)*(ny) + (ey*p + j))*(nx) + (ex*p + i);
  * bc is a tuple of 6 flags for the faces (x-, x+, y-, y+, z-, z+),
    1 = Dirichlet (u = 0), 0 = Neumann.
"""
import numpy as np

from . import gll as _gll


class Numbering:
    """Global numbering, mask and multiplicity of one level."""

    def __init__(self, nex, ney, nez, p, bc=(1, 1, 1, 1, 1, 1)):
        self.nex, self.ney, self.nez, self.p = nex, ney, nez, p
        self.N = p + 1
        self.E = nex * ney * nez
        self.bc = tuple(int(b) for b in bc)
        self.nx, self.ny, self.nz = nex * p + 1, ney * p + 1, nez * p + 1
        self.n = self.nx * self.ny * self.nz
        N = self.N
        ex, ey, ez = self.element_coords()
        r = np.arange(N)
        gx = ex[:, None, None, None] * p + r[None, None, None, :]
        gy = ey[:, None, None, None] * p + r[None, None, :, None]
        gz = ez[:, None, None, None] * p + r[None, :, None, None]
        self.gx = np.broadcast_to(gx, (self.E, N, N, N))
        self.gy = np.broadcast_to(gy, (self.E, N, N, N))
        self.gz = np.broadcast_to(gz, (self.E, N, N, N))
        self.gid = (gz * self.ny + gy) * self.nx + gx  # [E, N, N, N]
        self.mult = self.Qt(np.ones((self.E, N, N, N)))
        self.mask_global = self._dirichlet_mask_global()
        self.mask = self.Q(self.mask_global)

    def element_coords(self):
        e = np.arange(self.E)
        return e % self.nex, (e // self.nex) % self.ney, e // (self.nex * self.ney)

    def _dirichlet_mask_global(self):
        m = np.ones((self.nz, self.ny, self.nx))
        if self.bc[0]:
            m[:, :, 0] = 0
        if self.bc[1]:
            m[:, :, -1] = 0
        if self.bc[2]:
            m[:, 0, :] = 0
        if self.bc[3]:
            m[:, -1, :] = 0
        if self.bc[4]:
            m[0, :, :] = 0
        if self.bc[5]:
            m[-1, :, :] = 0
        return m.reshape(-1)

    # --- Q and Q^T -------------------------------------------------------
    def Q(self, u_global):
        """u_L = Q u: copy each global value to every local node holding it."""
        return np.asarray(u_global)[self.gid]

    def Qt(self, v_local):
        """Q^T v_L: sum local values into their global node."""
        return np.bincount(self.gid.reshape(-1), weights=np.asarray(v_local).reshape(-1),
                           minlength=self.n)

    def QQt(self, v_local):
        """Direct stiffness summation QQ^T on an E-vector."""
        return self.Q(self.Qt(v_local))

    def to_global(self, u_local):
        """Pick the global value of a consistent E-vector (any copy)."""
        u = np.zeros(self.n)
        u[self.gid.reshape(-1)] = np.asarray(u_local).reshape(-1)
        return u

    def dot_weight(self):
        """mask / mult: E-vector dot weight that counts each unique free dof once."""
        return self.mask / self.Q(self.mult)

    def wdot(self, a, b):
        return float(np.sum(self.dot_weight() * a * b))


def level_coordinates(xyz, p_geom, p):
    """Node coordinates at the level's GLL points from the input coordinates.

    xyz: [E, (p_geom+1)^3, 3] at the GLL(p_geom) nodes, i fastest.  The
    isoparametric interpolant of degree p_geom (Sec. 2.1) is evaluated at the
    GLL(p) nodes; for p_geom = 1 this is trilinear interpolation of the
    element vertices.  Returns X [3, E, N, N, N].
    """
    E = xyz.shape[0]
    Ng = p_geom + 1
    J = _gll.interpolation(p_geom, p)  # [N, Ng]
    X = np.empty((3, E, p + 1, p + 1, p + 1))
    for a in range(3):
        xa = xyz[:, :, a].reshape(E, Ng, Ng, Ng)  # [e, k, j, i]
        X[a] = np.einsum('kc,jb,ia,ecba->ekji', J, J, J, xa)
    return X
