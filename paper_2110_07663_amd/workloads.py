"""Seeded synthetic inputs for the SE Poisson solver: meshes and right-hand sides.

This module only *defines* inputs (coordinates of mesh nodes, source terms,
random vectors).  It contains none of the solver's arithmetic: no GLL rule,
no numbering, no operator.  Where node coordinates at reference points are
needed, the caller passes the 1D reference points in (the library exports its
own GLL nodes for that purpose).

Meshes are structured nex x ney x nez hexahedral grids on the unit cube
[0,1]^3; every map below keeps the unit cube (each face stays on its plane),
so u = sin(a pi x) sin(b pi y) sin(c pi z) vanishes on the whole boundary and
is an exact manufactured solution of -lap u = f with homogeneous Dirichlet
conditions.

Coordinate arrays have shape [E, Ng^3, 3]: element e = (ez*ney + ey)*nex + ex,
node (i, j, k) of the element at local index (k*Ng + j)*Ng + i.  Ng = 2 means
the 8 element vertices (the element is the trilinear image of the reference
cube); Ng = p+1 means the map sampled at the given reference points.

Workloads (stand-ins for the paper's Kershaw family, which needs a map not
given in the paper):
  * unit cube, undeformed: box_vertices;
  * smooth sinusoidal deformation x' = x + 0.05 s, y' = y + 0.05 s,
    z' = z + 0.05 s with s = sin(2 pi x) sin(2 pi y) sin(2 pi z): sin_map;
  * anisotropic "layer-shift" box with element aspect ratios up to 10:1:
    layer_shift_vertices.
"""
import math

import numpy as np


def _element_origin(nex, ney, nez):
    e = np.arange(nex * ney * nez)
    return e % nex, (e // nex) % ney, e // (nex * ney)


def box_vertices(nex, ney, nez):
    """Vertices [E, 8, 3] of the undeformed nex x ney x nez grid of [0,1]^3."""
    ex, ey, ez = _element_origin(nex, ney, nez)
    out = np.empty((len(ex), 8, 3))
    for k in range(2):
        for j in range(2):
            for i in range(2):
                v = (k * 2 + j) * 2 + i
                out[:, v, 0] = (ex + i) / nex
                out[:, v, 1] = (ey + j) / ney
                out[:, v, 2] = (ez + k) / nez
    return out


def sin_map(amp=0.05):
    """The smooth deformation x' = x + amp*s (same in y, z), s = prod sin(2 pi x_d)."""
    def f(x, y, z):
        s = np.sin(2 * np.pi * x) * np.sin(2 * np.pi * y) * np.sin(2 * np.pi * z)
        return x + amp * s, y + amp * s, z + amp * s
    return f


def sampled_mesh(nex, ney, nez, ref_points, mapping=None):
    """Node coordinates [E, Ng^3, 3] of `mapping` sampled at the tensor points.

    ref_points: 1D reference coordinates in [-1, 1] (Ng of them), e.g. GLL nodes.
    The undeformed position of reference point r in element ex is
    (ex + (r+1)/2)/nex; `mapping` (x, y, z) -> (x', y', z') is applied to it.
    """
    r = (np.asarray(ref_points, dtype=np.float64) + 1.0) / 2.0
    Ng = len(r)
    ex, ey, ez = _element_origin(nex, ney, nez)
    x = (ex[:, None, None, None] + r[None, None, None, :]) / nex
    y = (ey[:, None, None, None] + r[None, None, :, None]) / ney
    z = (ez[:, None, None, None] + r[None, :, None, None]) / nez
    E = len(ex)
    shape = (E, Ng, Ng, Ng)
    x, y, z = np.broadcast_to(x, shape), np.broadcast_to(y, shape), np.broadcast_to(z, shape)
    if mapping is not None:
        x, y, z = mapping(x, y, z)
    out = np.empty((E, Ng ** 3, 3))
    out[:, :, 0] = np.asarray(x).reshape(E, -1)
    out[:, :, 1] = np.asarray(y).reshape(E, -1)
    out[:, :, 2] = np.asarray(z).reshape(E, -1)
    return out


def _phi(a, t):
    """Piecewise-linear map of [0,1] onto itself sending 1/2 to a."""
    return np.where(t <= 0.5, 2.0 * a * t, a + 2.0 * (1.0 - a) * (t - 0.5))


def layer_shift_vertices(n, seed=3, slabs=4, amin=0.05, amax=0.95):
    """Vertices [E, 8, 3] of the anisotropic n^3 "layer-shift" box.

    Vertex grid i/n.  The x-range is cut into `slabs` slabs; at each slab
    boundary a ~ U[amin, amax] (the first forced to amin) and a is linearly
    interpolated to every x-plane; y' = phi_a(y).  Likewise c is drawn on the
    (slabs+1)^2 grid of (x, y) slab boundaries (c[0,0] forced to amin),
    bilinearly interpolated to every (x, y) vertex line, and z' = phi_c(z).
    phi_a sends [0,1/2] to [0,a] and [1/2,1] to [a,1], so element heights are
    2a/n and 2(1-a)/n and aspect ratios reach (1-amin)/amin-ish extremes
    (10:1 for amin = 0.05 against the x-width 1/n).
    """
    rng = np.random.default_rng(seed)
    a_b = rng.uniform(amin, amax, slabs + 1)
    a_b[0] = amin
    c_b = rng.uniform(amin, amax, (slabs + 1, slabs + 1))
    c_b[0, 0] = amin
    t = np.arange(n + 1) / n
    knots = np.linspace(0.0, 1.0, slabs + 1)
    a = np.interp(t, knots, a_b)  # per x-plane
    # bilinear interpolation of c to the (x, y) vertex lines (index [ix, iy])
    cx = np.stack([np.interp(t, knots, c_b[:, m]) for m in range(slabs + 1)], axis=1)
    c = np.stack([np.interp(t, knots, cx[ix]) for ix in range(n + 1)], axis=0)
    ix, iy, iz = np.meshgrid(np.arange(n + 1), np.arange(n + 1), np.arange(n + 1), indexing='ij')
    X = ix / n
    Y = _phi(a[ix], iy / n)
    Z = _phi(c[ix, iy], iz / n)
    ex, ey, ez = _element_origin(n, n, n)
    out = np.empty((n ** 3, 8, 3))
    for k in range(2):
        for j in range(2):
            for i in range(2):
                v = (k * 2 + j) * 2 + i
                out[:, v, 0] = X[ex + i, ey + j, ez + k]
                out[:, v, 1] = Y[ex + i, ey + j, ez + k]
                out[:, v, 2] = Z[ex + i, ey + j, ez + k]
    return out


def sinusoid(a=1, b=1, c=1):
    """(f, u) with u = sin(a pi x) sin(b pi y) sin(c pi z) and f = -lap u."""
    k2 = (a * a + b * b + c * c) * math.pi ** 2

    def u(x, y, z):
        return np.sin(a * np.pi * x) * np.sin(b * np.pi * y) * np.sin(c * np.pi * z)

    def f(x, y, z):
        return k2 * u(x, y, z)

    return f, u


def random_global(n, seed):
    """n samples of U(-1, 1) from numpy's default generator."""
    return np.random.default_rng(seed).uniform(-1.0, 1.0, n)


def batch_spec(nprob=64, seed=5, sides=(8, 12, 16, 24), degrees=(5, 7, 9), nrhs=4):
    """Problem list of the batched workload: [(side, p, [(a,b,c) x nrhs]), ...]."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(nprob):
        side = int(rng.choice(sides))
        p = int(rng.choice(degrees))
        freqs = [tuple(int(v) for v in rng.integers(1, 5, 3)) for _ in range(nrhs)]
        out.append((side, p, freqs))
    return out
