"""Oracle: plane-wave excitation vectors, the right-hand side V of eq. (2).

Test infrastructure (see the package docstring).  Plain NumPy, complex128.

Eq. (2) tests the incident field with every RWG basis function (Galerkin testing):
V_m = < b_m, n x n x E^i >.  The basis functions are tangential to the surface, so
b_m . (n x n x E) = b_m . (n (n . E) - E) = -b_m . E and

    V_m = - int_{S_m} b_m(r) . E^i(r) dr.

For the workloads with many right-hand sides the incident fields are unit plane
waves E^i(r) = e_hat exp(-j k k_hat . r) travelling along k_hat with polarisation
e_hat (the paper's own excitations are plane waves, Section III).  Readings (the
paper gives no formula for V beyond eq. (2)): the inner product is the plain
(unconjugated) integral of the Galerkin method; positions are absolute (the phase
reference is the origin); each triangle is integrated with the same symmetric
3-point rule as the far-fields of eq. (4).  The aggregation stage takes these
vectors as its input I_v (eq. (3)), one column per incident wave.

``planewave_highorder`` integrates the same integrand of one basis function with
the collapsed Gauss rule of :mod:`oracle.farfield`; it is used only to check the
3-point rule's convergence.
"""
import numpy as np

from .farfield import integrate_triangle

# barycentric coordinates of the symmetric 3-point rule (weights A/3 each)
_NODES = ((2.0 / 3.0, 1.0 / 6.0, 1.0 / 6.0),
          (1.0 / 6.0, 2.0 / 3.0, 1.0 / 6.0),
          (1.0 / 6.0, 1.0 / 6.0, 2.0 / 3.0))


def planewave_excitation(problem, khat, epol, rows=None):
    """V of eq. (2) for plane waves: [N, R] complex128, rows in group order (or only
    the group-order rows ``rows``, [len(rows), R]).

    ``khat`` [R, 3] unit propagation directions, ``epol`` [R, 3] polarisations.
    Column r is V_m = -int b_m . e_r exp(-j k k_r . r) dr over T+ and T-.
    """
    b = problem.rwg
    v, t = problem.verts, problem.tris
    khat = np.atleast_2d(np.asarray(khat, dtype=np.float64))
    epol = np.atleast_2d(np.asarray(epol, dtype=np.float64))
    rows = np.arange(problem.n_basis) if rows is None else np.asarray(rows)
    out = np.zeros((rows.size, khat.shape[0]), dtype=np.complex128)
    for tri_key, free_key, sign in (("tri_p", "free_p", +1.0), ("tri_m", "free_m", -1.0)):
        tri = t[b[tri_key][rows]]                           # [n, 3] corner indices
        corners = v[tri]                                    # [n, 3, 3]
        area = 0.5 * np.linalg.norm(np.cross(corners[:, 1] - corners[:, 0],
                                             corners[:, 2] - corners[:, 0]), axis=1)
        free = v[b[free_key][rows]]                         # [n, 3]
        scale = sign * b["length"][rows] / (2.0 * area)     # b_n = scale (r - p)
        for lam in _NODES:
            r = lam[0] * corners[:, 0] + lam[1] * corners[:, 1] + lam[2] * corners[:, 2]   # [N, 3]
            bn = scale[:, None] * (r - free)                # RWG value at the node
            w = area / 3.0                                  # rule weight
            field = np.exp(-1j * problem.k * (r @ khat.T))  # [N, R]
            out -= (w[:, None] * (bn @ epol.T)) * field
    return out


def planewave_highorder(problem, row, khat, epol, n=20):
    """V_row of :func:`planewave_excitation` by an n x n collapsed Gauss rule per
    triangle, the RWG function evaluated pointwise.  Returns [R] complex128."""
    b = problem.rwg
    v, t = problem.verts, problem.tris
    khat = np.atleast_2d(np.asarray(khat, dtype=np.float64))
    epol = np.atleast_2d(np.asarray(epol, dtype=np.float64))
    ln = b["length"][row]
    out = np.zeros(khat.shape[0], dtype=np.complex128)
    for tri, free, orient in ((b["tri_p"][row], b["free_p"][row], +1.0),
                              (b["tri_m"][row], b["free_m"][row], -1.0)):
        c0, c1, c2 = v[t[tri, 0]], v[t[tri, 1]], v[t[tri, 2]]
        area = 0.5 * np.linalg.norm(np.cross(c1 - c0, c2 - c0))
        p = v[free]

        def integrand(r, p=p, area=area, orient=orient):
            bn = orient * ln / (2.0 * area) * (r - p[None, :])               # [m, 3]
            return -(bn @ epol.T) * np.exp(-1j * problem.k * (r @ khat.T))   # [m, R]

        out += integrate_triangle(c0, c1, c2, integrand, n)
    return out
