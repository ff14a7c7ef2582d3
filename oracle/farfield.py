"""Oracle: far-field signatures of RWG basis functions, eq. (4).

Test infrastructure (see the package docstring).  Plain NumPy, complex128.

Eq. (4) defines, for basis n of group v, direction i and polarisation alpha in
{theta, phi},

    P^{alpha,+-}_{n,i} = alpha_hat_i . int_{S_n} (I - k_i k_i) b_n(r) exp(+-j k k_i.(r - r_v)) dr.

Because alpha_hat is orthogonal to k_i, alpha_hat . (I - k_i k_i) = alpha_hat, so the
projector drops out.  The paper does not name its quadrature; the reading here is
the symmetric 3-point rule on each triangle (points with barycentric coordinates
(2/3, 1/6, 1/6) and permutations, weights A/3), which integrates polynomials of
degree 2 exactly.  With it the contribution of each triangle of the support is
l_n / 6 times a sum over three points.

``farfield_highorder`` integrates the same integrand with a collapsed (Duffy)
tensor Gauss-Legendre rule of n x n points per triangle; it is used only to check
the 3-point rule's convergence.

Layout of the dense far-field: ``[N][2][n_theta][n_phi]`` complex128, rows in
group order, polarisation index 0 = theta, 1 = phi.
"""
import numpy as np

_BARY3 = np.array([[2.0 / 3.0, 1.0 / 6.0, 1.0 / 6.0],
                   [1.0 / 6.0, 2.0 / 3.0, 1.0 / 6.0],
                   [1.0 / 6.0, 1.0 / 6.0, 2.0 / 3.0]])


def _triangle_points(verts, tris, tri_idx):
    """3-point rule nodes of the triangles ``tri_idx``: [n, 3 points, 3 coords]."""
    t = tris[tri_idx]                                   # [n, 3]
    corners = verts[t]                                  # [n, 3 corners, 3]
    return np.einsum("qc,ncx->nqx", _BARY3, corners)


def farfield_rows(problem, rows, khat, that, phat, centers_of_rows, sign=+1):
    """P^{alpha,sign} for the basis functions ``rows`` (group-order indices).

    ``khat``, ``that``, ``phat``: [D, 3] direction and polarisation unit vectors.
    ``centers_of_rows``: [len(rows), 3] phase centre r_v of each row's group.
    Returns [len(rows), 2, D] complex128.
    """
    b = problem.rwg
    v, t = problem.verts, problem.tris
    rows = np.asarray(rows)
    ln = b["length"][rows]
    pts_p = _triangle_points(v, t, b["tri_p"][rows])    # [n, 3, 3]
    pts_m = _triangle_points(v, t, b["tri_m"][rows])
    fp = v[b["free_p"][rows]]                           # [n, 3]
    fm = v[b["free_m"][rows]]
    rho = np.concatenate([pts_p - fp[:, None, :], fm[:, None, :] - pts_m], axis=1)  # [n, 6, 3]
    pts = np.concatenate([pts_p, pts_m], axis=1)                                  # [n, 6, 3]
    rel = pts - centers_of_rows[:, None, :]
    phase = np.exp(sign * 1j * problem.k * np.einsum("nqx,dx->nqd", rel, khat))  # [n, 6, D]
    a_th = np.einsum("nqx,dx->nqd", rho, that)
    a_ph = np.einsum("nqx,dx->nqd", rho, phat)
    out = np.empty((rows.size, 2, khat.shape[0]), dtype=np.complex128)
    out[:, 0, :] = np.sum(a_th * phase, axis=1)
    out[:, 1, :] = np.sum(a_ph * phase, axis=1)
    out *= (ln / 6.0)[:, None, None]
    return out


def farfield_group(problem, g, sign=+1):
    """Dense far-field of group ``g``: [n_beta, 2, n_theta, n_phi] complex128."""
    lo, hi = int(problem.offsets[g]), int(problem.offsets[g + 1])
    rows = np.arange(lo, hi)
    c = np.repeat(problem.centers[g][None, :], rows.size, axis=0)
    out = np.empty((rows.size, 2, problem.n_dir), dtype=np.complex128)
    step = 256
    for s in range(0, rows.size, step):
        out[s:s + step] = farfield_rows(problem, rows[s:s + step], problem.khat,
                                        problem.that, problem.phat, c[s:s + step], sign)
    return out.reshape(rows.size, 2, problem.n_theta, problem.n_phi)


def farfield_all(problem, sign=+1):
    """Dense far-fields of every group, [N, 2, n_theta, n_phi] complex128."""
    return np.concatenate([farfield_group(problem, g, sign) for g in range(problem.n_groups)], axis=0)


# ----------------------------------------------------------- high-order reference

def _collapsed_rule(n):
    """Nodes (barycentric-free form) and weights of the n x n collapsed Gauss rule
    on the reference triangle {(s, t): 0 <= t <= s <= 1} scaled to unit area."""
    x, w = np.polynomial.legendre.leggauss(n)
    x = 0.5 * (x + 1.0)
    w = 0.5 * w
    s, tt = np.meshgrid(x, x, indexing="ij")
    ws, wt = np.meshgrid(w, w, indexing="ij")
    # map (s, tt) in [0,1]^2 to the triangle: point = c0 + s (c1 - c0) + s tt (c2 - c1)
    # area element = 2 A s ds dtt, and the integral of 1 over [0,1]^2 of s is 1/2.
    return s.ravel(), tt.ravel(), (ws * wt * s * 2.0).ravel()


def integrate_triangle(c0, c1, c2, f, n=20):
    """Integral of ``f(points [m,3]) -> [m, ...]`` over the triangle (c0, c1, c2)."""
    s, tt, w = _collapsed_rule(n)
    pts = c0[None, :] + s[:, None] * (c1 - c0)[None, :] + (s * tt)[:, None] * (c2 - c1)[None, :]
    area = 0.5 * np.linalg.norm(np.cross(c1 - c0, c2 - c0))
    vals = f(pts)
    return area * np.tensordot(w, vals, axes=(0, 0))


def farfield_highorder(problem, row, khat, that, phat, center, n=20, sign=+1):
    """P^{alpha,sign} of one basis function by an n x n collapsed Gauss rule.

    Returns [2, D] complex128.  Written independently of the 3-point routine: the
    basis function is evaluated pointwise from its definition.
    """
    b = problem.rwg
    v, t = problem.verts, problem.tris
    ln = b["length"][row]
    out = np.zeros((2, khat.shape[0]), dtype=np.complex128)
    for tri, free, orient in ((b["tri_p"][row], b["free_p"][row], +1.0),
                              (b["tri_m"][row], b["free_m"][row], -1.0)):
        c0, c1, c2 = v[t[tri, 0]], v[t[tri, 1]], v[t[tri, 2]]
        area = 0.5 * np.linalg.norm(np.cross(c1 - c0, c2 - c0))
        p = v[free]

        def integrand(r, p=p, area=area, orient=orient):
            bn = orient * ln / (2.0 * area) * (r - p[None, :])                 # [m, 3]
            ph = np.exp(sign * 1j * problem.k * ((r - center[None, :]) @ khat.T))  # [m, D]
            return np.stack([(bn @ that.T) * ph, (bn @ phat.T) * ph], axis=1)  # [m, 2, D]

        out += integrate_triangle(c0, c1, c2, integrand, n)
    return out
