"""Geodesic sphere meshes (class-I subdivision of the icosahedron).

The paper's sphere meshes are not available; a geodesic icosphere of frequency
``f`` stands in for them.  It has ``10 f^2 + 2`` vertices, ``30 f^2`` edges and
``20 f^2`` triangles, all triangles oriented counter-clockwise seen from outside.
``f = 8`` gives the 1280-triangle, 1920-edge mesh of the small workload and
``f = 177`` gives 939,870 edges for the 30-wavelength sphere (the paper meshes that
sphere with 940,308 basis functions).

Every vertex is computed once from an integer key, so a point shared by two
icosahedron faces has bit-identical coordinates in both.
"""
import numpy as np

_PHI = (1.0 + 5.0 ** 0.5) / 2.0


def _icosahedron():
    v = np.array([
        [-1, _PHI, 0], [1, _PHI, 0], [-1, -_PHI, 0], [1, -_PHI, 0],
        [0, -1, _PHI], [0, 1, _PHI], [0, -1, -_PHI], [0, 1, -_PHI],
        [_PHI, 0, -1], [_PHI, 0, 1], [-_PHI, 0, -1], [-_PHI, 0, 1],
    ], dtype=np.float64)
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    f = np.array([
        [0, 11, 5], [0, 5, 1], [0, 1, 7], [0, 7, 10], [0, 10, 11],
        [1, 5, 9], [5, 11, 4], [11, 10, 2], [10, 7, 6], [7, 1, 8],
        [3, 9, 4], [3, 4, 2], [3, 2, 6], [3, 6, 8], [3, 8, 9],
        [4, 9, 5], [2, 4, 11], [6, 2, 10], [8, 6, 7], [9, 8, 1],
    ], dtype=np.int64)
    # orient every face outward (normal along the centroid)
    a, b, c = v[f[:, 0]], v[f[:, 1]], v[f[:, 2]]
    n = np.cross(b - a, c - a)
    flip = np.einsum("ij,ij->i", n, a + b + c) < 0
    f[flip] = f[flip][:, [0, 2, 1]]
    return v, f


def icosphere(freq, radius=1.0, center=(0.0, 0.0, 0.0)):
    """Return ``(vertices [V,3] float64, triangles [F,3] int32)``.

    Class-I geodesic subdivision: each icosahedron face (A, B, C) is split into
    ``freq^2`` triangles whose vertices are ``(a B + b C + (freq-a-b) A) / freq``
    projected onto the sphere.
    """
    fq = int(freq)
    if fq < 1:
        raise ValueError("freq must be >= 1")
    v0, faces = _icosahedron()

    # global edge table of the icosahedron (p < q)
    e = np.sort(np.concatenate([faces[:, [0, 1]], faces[:, [1, 2]], faces[:, [2, 0]]]), axis=1)
    edges = np.unique(e, axis=0)
    edge_id = {(int(p), int(q)): k for k, (p, q) in enumerate(edges)}

    n_edge_pts = fq - 1
    n_face_pts = (fq - 1) * (fq - 2) // 2
    nv = 12 + 30 * n_edge_pts + 20 * n_face_pts
    verts = np.empty((nv, 3), dtype=np.float64)
    verts[:12] = v0
    # edge points: t = 1..fq-1 steps from p toward q
    if n_edge_pts > 0:
        t = np.arange(1, fq, dtype=np.float64)[None, :, None]
        p = v0[edges[:, 0]][:, None, :]
        q = v0[edges[:, 1]][:, None, :]
        pts = ((fq - t) * p + t * q) / fq
        pts /= np.linalg.norm(pts, axis=2, keepdims=True)
        verts[12:12 + 30 * n_edge_pts] = pts.reshape(-1, 3)
    face_base = 12 + 30 * n_edge_pts

    # local (a, b) lattice of one face: a steps toward B, b steps toward C
    aa, bb = np.meshgrid(np.arange(fq + 1), np.arange(fq + 1), indexing="ij")
    keep = aa + bb <= fq
    la, lb = aa[keep], bb[keep]
    local_index = -np.ones((fq + 1, fq + 1), dtype=np.int64)
    local_index[la, lb] = np.arange(la.size)
    interior = (la > 0) & (lb > 0) & (la + lb < fq)

    tris = []
    for fi, (A, B, C) in enumerate(faces):
        gid = np.empty(la.size, dtype=np.int64)
        wa = fq - la - lb
        # corners
        gid[(la == 0) & (lb == 0)] = A
        gid[(la == fq)] = B
        gid[(lb == fq)] = C

        def on_edge(u, w_u, v_):
            # points on the face edge u--v_, w_u = steps from u toward v_
            p, q = (u, v_) if u < v_ else (v_, u)
            steps = w_u if u < v_ else fq - w_u
            return 12 + edge_id[(int(p), int(q))] * n_edge_pts + (steps - 1)

        m = (lb == 0) & (la > 0) & (la < fq)          # A--B edge, la steps from A
        gid[m] = on_edge(A, la[m], B)
        m = (la == 0) & (lb > 0) & (lb < fq)          # A--C edge, lb steps from A
        gid[m] = on_edge(A, lb[m], C)
        m = (wa == 0) & (la > 0) & (lb > 0)           # B--C edge, lb steps from B
        gid[m] = on_edge(B, lb[m], C)
        if n_face_pts > 0:
            ia, ib = la[interior], lb[interior]
            pts = (ia[:, None] * v0[B] + ib[:, None] * v0[C] + (fq - ia - ib)[:, None] * v0[A]) / fq
            pts /= np.linalg.norm(pts, axis=1, keepdims=True)
            base = face_base + fi * n_face_pts
            verts[base:base + n_face_pts] = pts
            gid[interior] = base + np.arange(n_face_pts)

        # up triangles (a,b),(a+1,b),(a,b+1); down triangles (a+1,b),(a+1,b+1),(a,b+1)
        ua, ub = np.nonzero(keep[:fq, :fq] & ((aa[:fq, :fq] + bb[:fq, :fq]) <= fq - 1))
        up = np.stack([local_index[ua, ub], local_index[ua + 1, ub], local_index[ua, ub + 1]], axis=1)
        da, db = np.nonzero((aa[:fq, :fq] + bb[:fq, :fq]) <= fq - 2)
        dn = np.stack([local_index[da + 1, db], local_index[da + 1, db + 1], local_index[da, db + 1]], axis=1)
        tris.append(gid[np.concatenate([up, dn])])

    tri = np.concatenate(tris).astype(np.int32)
    r = float(radius)
    verts = verts * r + np.asarray(center, dtype=np.float64)[None, :]
    return verts, tri


def trihedral(edge, n):
    """Trihedral corner reflector: three mutually perpendicular square plates of side
    ``edge`` in the planes x = 0, y = 0 and z = 0, meeting at the origin and spanning
    the first octant.  Each plate is an ``n x n`` grid of squares, each square split
    into two triangles along its (0,0)-(1,1) diagonal.  Points on the three shared
    axes are one vertex each, so the plates are joined along the axes.

    Triangles are oriented with normals -x, -y, -z (away from the octant), which
    traverses every shared edge in opposite directions from its two triangles.  The
    mesh has 3 n (n + 1) + 1 vertices, 6 n^2 triangles and 9 n^2 - 3 n edges with two
    triangles (the plates' outer rims, 6 n edges, have one).

    Returns ``(vertices [V,3] float64, triangles [F,3] int32)``.
    """
    n = int(n)
    if n < 1:
        raise ValueError("n must be >= 1")
    h = float(edge) / n
    key = {}
    verts = []

    def vid(i, j, k):
        if (i, j, k) not in key:
            key[(i, j, k)] = len(verts)
            verts.append((i * h, j * h, k * h))
        return key[(i, j, k)]

    tris = []
    # plate axis pairs (u, v) and the normal each plate gets
    plates = [((0, 1), np.array([0.0, 0.0, -1.0])),   # z = 0: u = x, v = y
              ((0, 2), np.array([0.0, -1.0, 0.0])),   # y = 0: u = x, v = z
              ((1, 2), np.array([-1.0, 0.0, 0.0]))]   # x = 0: u = y, v = z
    for (au, av), normal in plates:
        eu = np.zeros(3)
        ev = np.zeros(3)
        eu[au] = 1.0
        ev[av] = 1.0
        flip = np.dot(np.cross(eu, ev), normal) < 0
        for a in range(n):
            for b in range(n):
                def p(da, db):
                    c = [0, 0, 0]
                    c[au], c[av] = a + da, b + db
                    return vid(*c)
                p00, p10, p11, p01 = p(0, 0), p(1, 0), p(1, 1), p(0, 1)
                for t in ((p00, p10, p11), (p00, p11, p01)):
                    tris.append((t[0], t[2], t[1]) if flip else t)
    return np.array(verts, dtype=np.float64), np.array(tris, dtype=np.int32)
