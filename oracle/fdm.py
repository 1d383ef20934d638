"""Overlapping Schwarz smoother by the fast diagonalisation method (oracle, test-only).

Sec. 2.2.2.  The ASM smoother (eq. 4) is s = sum_e W_e R_e^T Abar_e^{-1} R_e r.
Each deformed element is approximated by a box, the box is extended by one
node in each direction, giving pbar^3 = (p+3)^3 unknowns, and the separable
extended-box operator (eq. 5)

    Abar = B_z (x) B_y (x) A_x + B_z (x) A_y (x) B_x + A_z (x) B_y (x) B_x

is inverted through the generalised eigenproblems A_* s = lambda B_* s (eq. 6),
S_*^T A_* S_* = Lambda_*, S_*^T B_* S_* = I (eq. 7), so that (eqs. 8-9)

    Abar^{-1} = (S_z (x) S_y (x) S_x) D^{-1} (S_z^T (x) S_y^T (x) S_x^T),
    D = I (x) I (x) Lambda_x + I (x) Lambda_y (x) I + Lambda_z (x) I (x) I.

RAS drops the overlap values after the local solve ("formally, changing W_e").

Readings where the paper gives no formula:
  * box length L_r of an element = mean of its 4 vertex-to-vertex edge
    lengths parallel to r (likewise s, t);
  * the 1D extended grid is the left neighbour's node p-1, the element's
    nodes 0..p and the right neighbour's node 1.  A_* and B_* are the 1D
    stiffness (2/L) Dhat^T W Dhat and mass (L/2) W assembled over the
    (left, element, right) triple with each element's own L, restricted to
    those p+3 nodes (homogeneous Dirichlet beyond them);
  * where the element touches the domain boundary there is no neighbour: the
    missing extension node is decoupled; on a Dirichlet face the element's
    boundary node is decoupled too.  A decoupled node is excluded from the
    local solve (its output is zero), represented by an identity column of
    S and lambda = +inf;
  * a 1D eigenvalue below 1e-12 of the largest one is set to 0; a zero
    eigenvalue sum (the constant mode of a box floating on Neumann faces in
    all three directions) is dropped from the local solve;
  * ASM weight W(node) = 1 / (number of extended boxes containing the node);
    RAS weight on an element's own nodes = 1 / (number of elements owning
    the node), zero on the overlap shell.
"""
import numpy as np

from . import gll as _gll


def box_lengths(X):
    """L[E, 3]: mean edge length along r, s, t from the element corner nodes."""
    c = X[:, :, [0, -1]][:, :, :, [0, -1]][:, :, :, :, [0, -1]]  # [3, E, 2(k), 2(j), 2(i)]
    Lr = np.sqrt(np.sum((c[:, :, :, :, 1] - c[:, :, :, :, 0]) ** 2, axis=0)).mean(axis=(1, 2))
    Ls = np.sqrt(np.sum((c[:, :, :, 1, :] - c[:, :, :, 0, :]) ** 2, axis=0)).mean(axis=(1, 2))
    Lt = np.sqrt(np.sum((c[:, :, 1, :, :] - c[:, :, 0, :, :]) ** 2, axis=0)).mean(axis=(1, 2))
    return np.stack([Lr, Ls, Lt], axis=1)


_REF_CACHE = {}


def _reference_1d(p):
    """GLL weights and the reference 1D stiffness Ahat = Dhat^T W Dhat."""
    if p not in _REF_CACHE:
        _, w, D = _gll.gll(p)
        _REF_CACHE[p] = (w, D.T @ np.diag(w) @ D)
    return _REF_CACHE[p]


def extended_1d(p, Lm, L, Lp, has_left, has_right, dir_left, dir_right):
    """Extended 1D pair (K, M), shape (p+3, p+3), and the coupled index list.

    Lm / Lp are the neighbours' lengths (ignored when the neighbour is absent).
    """
    w, Ahat = _reference_1d(p)
    n = 3 * p + 1
    K = np.zeros((n, n))
    M = np.zeros((n, n))
    for t, (Le, present) in enumerate(((Lm, has_left), (L, True), (Lp, has_right))):
        if not present:
            continue
        s = slice(t * p, t * p + p + 1)
        K[s, s] += (2.0 / Le) * Ahat
        M[s, s] += (Le / 2.0) * np.diag(w)
    ext = np.arange(p - 1, 2 * p + 2)  # chain indices of the p+3 extended nodes
    K = K[np.ix_(ext, ext)]
    M = M[np.ix_(ext, ext)]
    coupled = np.ones(p + 3, dtype=bool)
    if not has_left:
        coupled[0] = False
        if dir_left:
            coupled[1] = False
    if not has_right:
        coupled[p + 2] = False
        if dir_right:
            coupled[p + 1] = False
    return K, M, coupled


def generalized_eig(K, M, coupled):
    """S, lam with S^T K S = diag(lam), S^T M S = I on the coupled nodes.

    M is diagonal (GLL mass), so with Mh = M^{-1/2}: eigh(Mh K Mh) = V diag(lam) V^T
    and S = Mh V.  Decoupled nodes get identity columns and lam = +inf.
    """
    pb = K.shape[0]
    c = np.nonzero(coupled)[0]
    d = np.nonzero(~coupled)[0]
    S = np.zeros((pb, pb))
    lam = np.full(pb, np.inf)
    Kc = K[np.ix_(c, c)]
    mh = 1.0 / np.sqrt(np.diag(M)[c])
    lc, V = np.linalg.eigh(mh[:, None] * Kc * mh[None, :])
    # the constant mode of a line floating on Neumann ends has eigenvalue 0
    # (up to rounding): make it exactly 0 so that the local solve can drop it
    lc = np.where(np.abs(lc) <= 1e-12 * np.abs(lc).max(), 0.0, lc)
    S[np.ix_(c, np.arange(len(c)))] = mh[:, None] * V
    lam[:len(c)] = lc
    for t, i in enumerate(d):
        S[i, len(c) + t] = 1.0
    return S, lam


class FDM:
    """Per-element FDM data of one level: S[E,3,pb,pb], lam[E,3,pb]."""

    def __init__(self, num, X):
        p = num.p
        self.num = num
        self.p, self.pb = p, p + 3
        E = num.E
        L = box_lengths(X)
        ex, ey, ez = num.element_coords()
        counts = (num.nex, num.ney, num.nez)
        pos = (ex, ey, ez)
        strides = (1, num.nex, num.nex * num.ney)
        self.S = np.zeros((E, 3, self.pb, self.pb))
        self.lam = np.zeros((E, 3, self.pb))
        for e in range(E):
            for d in range(3):
                has_l = pos[d][e] > 0
                has_r = pos[d][e] < counts[d] - 1
                Lm = L[e - strides[d], d] if has_l else 0.0
                Lp = L[e + strides[d], d] if has_r else 0.0
                K, M, cpl = extended_1d(p, Lm, L[e, d], Lp, has_l, has_r,
                                        num.bc[2 * d], num.bc[2 * d + 1])
                self.S[e, d], self.lam[e, d] = generalized_eig(K, M, cpl)
        self._box_index()

    def _box_index(self):
        """Global index of every extended-box node, -1 outside the domain."""
        num, p, pb = self.num, self.p, self.pb
        ex, ey, ez = num.element_coords()
        r = np.arange(pb) - 1
        gx = ex[:, None] * p + r[None, :]
        gy = ey[:, None] * p + r[None, :]
        gz = ez[:, None] * p + r[None, :]
        ok = ((gx >= 0) & (gx < num.nx))[:, None, None, :] & \
             ((gy >= 0) & (gy < num.ny))[:, None, :, None] & \
             ((gz >= 0) & (gz < num.nz))[:, :, None, None]
        g = (gz[:, :, None, None] * num.ny + gy[:, None, :, None]) * num.nx + gx[:, None, None, :]
        self.box_gid = np.where(ok, g, -1)

    def gather(self, r_local):
        """R_e r for every element: [E, pb, pb, pb] (zero outside the domain)."""
        rg = self.num.to_global(r_local)
        ok = self.box_gid >= 0
        return np.where(ok, rg[np.where(ok, self.box_gid, 0)], 0.0)

    def local_solve(self, rb):
        """Abar_e^{-1} applied to box vectors rb[E, pb, pb, pb] (eq. 8)."""
        Sx, Sy, Sz = self.S[:, 0], self.S[:, 1], self.S[:, 2]
        t = np.einsum('eia,ekji->ekja', Sx, rb)
        t = np.einsum('ejb,ekja->ekba', Sy, t)
        t = np.einsum('ekc,ekba->ecba', Sz, t)
        Dm = (self.lam[:, 2][:, :, None, None] + self.lam[:, 1][:, None, :, None]
              + self.lam[:, 0][:, None, None, :])
        # a box floating on Neumann faces in all three directions has a zero
        # eigenvalue sum (its constant mode); that mode is dropped
        keep = Dm > 0.0
        t = np.where(keep, t / np.where(keep, Dm, 1.0), 0.0)
        t = np.einsum('eia,ecba->ecbi', Sx, t)
        t = np.einsum('ejb,ecbi->ecji', Sy, t)
        t = np.einsum('ekc,ecji->ekji', Sz, t)
        return t

    def apply_ras(self, r_local):
        """RAS: keep each element's own nodes, weight by 1/mult, assemble, mask."""
        num, p = self.num, self.p
        y = self.local_solve(self.gather(r_local))[:, 1:p + 2, 1:p + 2, 1:p + 2]
        W = 1.0 / num.Q(num.mult)
        return num.mask * num.QQt(W * y)

    def apply_asm(self, r_local):
        """ASM (eq. 4): sum all box outputs into the global vector, times 1/#boxes."""
        num = self.num
        y = self.local_solve(self.gather(r_local))
        ok = self.box_gid >= 0
        s = np.bincount(self.box_gid[ok], weights=y[ok], minlength=num.n)
        nbox = np.bincount(self.box_gid[ok], minlength=num.n)
        s = s / np.maximum(nbox, 1)
        return num.mask * num.Q(s)
