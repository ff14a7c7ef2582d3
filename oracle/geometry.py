"""Oracle: RWG basis functions, FMM-FFT grouping and the spherical angular grid.

Test infrastructure (see the package docstring).  Plain NumPy, float64.

RWG basis (Section II.A, eq. (2); the basis of ref. [20]).  Every edge shared by
two triangles carries one basis function b_n.  With l_n the edge length, T+ and
T- the two triangles, A+- their areas and p+- their vertices opposite the edge:

    b_n(r) = l_n / (2 A+) (r - p+)   on T+,
    b_n(r) = l_n / (2 A-) (p- - r)   on T-.

Reading (the paper is silent on orientation): triangles are oriented
counter-clockwise seen from outside; for an edge with end vertices a < b (global
indices) T+ is the triangle that traverses the edge from a to b.  Basis functions
are numbered by the edge key (a, b) in lexicographic order.

Grouping (Section II.A): the domain is split into a cubic box grid; non-empty
boxes are the groups.  Reading: a basis function belongs to the box containing
its edge midpoint; box edge ``box``; the grid is anchored at ``origin`` with
``K`` boxes per axis; a point on a box face goes to the higher box, and indices
are clamped to [0, K-1].  Box v = (ix, iy, iz) has linear index
(ix * K + iy) * K + iz and centre origin + (i + 1/2) * box.  Groups are the
non-empty boxes in increasing linear index; inside a group the basis functions
keep their global order.

Angular grid (Section II.A): L + 1 points in theta and 2L + 1 in phi.  Reading:
theta nodes are Gauss-Legendre nodes in cos(theta), ordered by increasing theta;
phi_j = 2 pi j / n_phi.  Direction index i = i_theta * n_phi + i_phi.
"""
import math
import numpy as np


# --------------------------------------------------------------------------- RWG

def rwg(verts, tris):
    """Build the RWG basis (ref. [20]) of a consistently oriented triangle mesh.

    An edge shared by two triangles that traverse it in opposite directions carries
    one basis function.  An edge of a single triangle lies on the rim of an open
    surface (the plates of the trihedral example, Section III.A) and carries none:
    no current crosses a free edge.

    Returns a dict of arrays, one row per basis function in (a, b) order:
      ``edge`` [N,2] end vertices (a < b), ``tri_p``/``tri_m`` [N] triangle indices
      (T+ traverses a -> b), ``free_p``/``free_m`` [N] opposite vertices, ``length``
      [N] edge length.
    Raises ``ValueError`` for an edge of more than two triangles or of two triangles
    traversing it the same way.
    """
    tris = np.asarray(tris, dtype=np.int64)
    nt = tris.shape[0]
    # directed edges (u -> w) of each triangle and the vertex opposite to them
    u = np.concatenate([tris[:, 0], tris[:, 1], tris[:, 2]])
    w = np.concatenate([tris[:, 1], tris[:, 2], tris[:, 0]])
    opp = np.concatenate([tris[:, 2], tris[:, 0], tris[:, 1]])
    tri_id = np.concatenate([np.arange(nt)] * 3)
    lo = np.minimum(u, w)
    hi = np.maximum(u, w)
    forward = u < w
    order = np.lexsort((~forward, hi, lo))      # by (lo, hi), forward first
    lo, hi, forward, opp, tri_id = lo[order], hi[order], forward[order], opp[order], tri_id[order]
    key = lo * (int(hi.max()) + 1) + hi
    first = np.flatnonzero(np.concatenate([[True], np.diff(key) != 0]))
    count = np.diff(np.concatenate([first, [key.size]]))
    if np.any(count > 2):
        raise ValueError("an edge is shared by more than two triangles")
    a = first[count == 2]                       # forward half of each shared edge
    b = a + 1
    if not (np.all(forward[a]) and not np.any(forward[b])):
        raise ValueError("triangles are not consistently oriented")
    verts = np.asarray(verts, dtype=np.float64)
    return {
        "edge": np.stack([lo[a], hi[a]], axis=1),
        "tri_p": tri_id[a], "tri_m": tri_id[b],
        "free_p": opp[a], "free_m": opp[b],
        "length": np.linalg.norm(verts[hi[a]] - verts[lo[a]], axis=1),
    }


def triangle_areas(verts, tris):
    v = np.asarray(verts, dtype=np.float64)
    t = np.asarray(tris, dtype=np.int64)
    return 0.5 * np.linalg.norm(np.cross(v[t[:, 1]] - v[t[:, 0]], v[t[:, 2]] - v[t[:, 0]]), axis=1)


# ---------------------------------------------------------------------- grouping

def group_basis(verts, edges, origin, box, K):
    """Assign basis functions to boxes (Section II.A).

    Returns ``(perm, offsets, box_index, centers)``: ``perm`` [N] lists global basis
    indices in group order, ``offsets`` [G+1] is the CSR split of ``perm`` into
    groups, ``box_index`` [G, 3] the integer box coordinates and ``centers`` [G, 3]
    the box centres r_v (the phase centres of eq. (4)).
    """
    v = np.asarray(verts, dtype=np.float64)
    e = np.asarray(edges, dtype=np.int64)
    mid = 0.5 * (v[e[:, 0]] + v[e[:, 1]])
    o = np.asarray(origin, dtype=np.float64)
    idx = np.floor((mid - o[None, :]) / box).astype(np.int64)
    idx = np.clip(idx, 0, K - 1)
    lin = (idx[:, 0] * K + idx[:, 1]) * K + idx[:, 2]
    perm = np.argsort(lin, kind="stable")
    boxes, counts = np.unique(lin[perm], return_counts=True)
    offsets = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    bidx = np.stack([boxes // (K * K), (boxes // K) % K, boxes % K], axis=1)
    centers = o[None, :] + (bidx + 0.5) * box
    return perm, offsets, bidx, centers


# ------------------------------------------------------------------ angular grid

def grid_order(box, digits):
    """Size L of the angular grid for a box of edge ``box`` (wavelengths).

    Section II.A gives L = 2 k R^s + (2 k R^s)^(1/3) * 1.8 * (log10(1/Gamma))^(2/3)
    with R^s the radius of the smallest sphere enclosing a box.  Reading: R^s is
    half the box diagonal, log10(1/Gamma) is the number of accurate digits, and
    L is that value rounded to the nearest integer plus one.  This reproduces the
    L = 16, 24, 31, 37 that Table IV lists for boxes of 0.5, 1, 1.5 and 2
    wavelengths at 5 digits.
    """
    k = 2.0 * math.pi
    rs = math.sqrt(3.0) * box / 2.0
    x = 2.0 * k * rs + (2.0 * k * rs) ** (1.0 / 3.0) * 1.8 * digits ** (2.0 / 3.0)
    return int(round(x)) + 1


def angular_grid(n_theta, n_phi):
    """Directions of the spherical grid (Section II.A).

    Returns ``(theta [n_theta], phi [n_phi], khat, that, phat)`` where the last
    three are [n_theta * n_phi, 3] unit vectors in direction order
    i = i_theta * n_phi + i_phi.
    """
    x, _ = np.polynomial.legendre.leggauss(n_theta)
    theta = np.arccos(x[::-1])          # increasing theta
    phi = 2.0 * np.pi * np.arange(n_phi) / n_phi
    th = np.repeat(theta, n_phi)
    ph = np.tile(phi, n_theta)
    st, ct, sp, cp = np.sin(th), np.cos(th), np.sin(ph), np.cos(ph)
    khat = np.stack([st * cp, st * sp, ct], axis=1)
    that = np.stack([ct * cp, ct * sp, -st], axis=1)
    phat = np.stack([-sp, cp, np.zeros_like(sp)], axis=1)
    return theta, phi, khat, that, phat


def gauss_legendre_weights(n_theta):
    """Gauss-Legendre weights matching :func:`angular_grid`'s theta order."""
    _, w = np.polynomial.legendre.leggauss(n_theta)
    return w[::-1]


# ----------------------------------------------------------- a complete problem

class Problem:
    """Mesh + RWG + groups + grid of one workload, in group order.

    ``rwg`` arrays are permuted to group order (row n of every per-basis array is
    the n-th basis function of the concatenated groups).
    """

    def __init__(self, verts, tris, origin, box, K, n_theta, n_phi, k=2.0 * math.pi):
        self.verts = np.asarray(verts, dtype=np.float64)
        self.tris = np.asarray(tris, dtype=np.int64)
        self.k = float(k)
        basis = rwg(self.verts, self.tris)
        perm, offsets, bidx, centers = group_basis(self.verts, basis["edge"], origin, box, K)
        self.perm = perm
        self.rwg = {key: val[perm] for key, val in basis.items()}
        self.offsets = offsets
        self.box_index = bidx
        self.centers = centers
        self.n_theta, self.n_phi = int(n_theta), int(n_phi)
        self.areas = triangle_areas(self.verts, self.tris)
        (self.theta, self.phi, self.khat, self.that, self.phat) = angular_grid(n_theta, n_phi)

    @property
    def n_groups(self):
        return self.offsets.size - 1

    @property
    def n_basis(self):
        return int(self.offsets[-1])

    @property
    def n_dir(self):
        return self.n_theta * self.n_phi

    def group_sizes(self):
        return np.diff(self.offsets)

    def group_of_basis(self):
        return np.repeat(np.arange(self.n_groups), self.group_sizes())
