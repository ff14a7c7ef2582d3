"""Oracle: aggregation and disaggregation, dense and in Tucker format.

Test infrastructure (see the package docstring).  Plain NumPy, complex128.

Per group and polarisation alpha the aggregation matrix A^alpha (N_dir x n_beta) has
entries A^alpha[i, n] = P^{alpha,+}_{n,i} of eq. (4).

* Dense aggregation, eq. (3) and Fig. 2(a):       F^alpha = A^alpha x.
* Dense disaggregation, eq. (5) and Fig. 3(a):   V = sum_alpha (A^alpha)* G^alpha,
  using P^- = (P^+)* (conjugate transpose) from the end of Section II.A.
* Tucker aggregation, Section II.C / Fig. 2(b), and Tucker disaggregation,
  Section II.C / Fig. 3(b), follow the paper's steps in order (see the functions).

Shapes: a group's dense rows are [n_beta, 2, n_theta, n_phi]; x and V are [n_beta]
or [n_beta, R]; F and G are [2, N_dir] or [2, N_dir, R] with direction index
i = i_theta * n_phi + i_phi.  Tucker factors use the paper's shapes: core
[r_theta, r_phi, r_beta], U^theta [n_theta, r_theta], U^phi [n_phi, r_phi],
U^beta [n_beta, r_beta].
"""
import numpy as np


def _as_matrix(v):
    """[n] -> [n, 1]; [n, R] unchanged.  Returns (matrix, was_vector)."""
    v = np.asarray(v)
    return (v[:, None], True) if v.ndim == 1 else (v, False)


# ------------------------------------------------------------------------ dense

def dense_aggregate(dense_group, x):
    """F^alpha = A^alpha x for alpha = theta, phi (eq. (3)).  Returns [2, N_dir(, R)]."""
    xm, vec = _as_matrix(x)
    nb = dense_group.shape[0]
    out = []
    for alpha in range(2):
        a = dense_group[:, alpha].reshape(nb, -1).T          # [N_dir, n_beta]
        out.append(a @ xm)
    f = np.stack(out)                                         # [2, N_dir, R]
    return f[..., 0] if vec else f


def dense_disaggregate(dense_group, g):
    """V = sum_alpha (A^alpha)* G^alpha (eq. (5)).  Returns [n_beta(, R)]."""
    g = np.asarray(g)
    vec = g.ndim == 2
    gm = g[..., None] if vec else g                           # [2, N_dir, R]
    nb = dense_group.shape[0]
    v = 0
    for alpha in range(2):
        a = dense_group[:, alpha].reshape(nb, -1).T          # [N_dir, n_beta]
        v = v + a.conj().T @ gm[alpha]
    return v[:, 0] if vec else v


# ----------------------------------------------------------------------- Tucker

def tucker_aggregate_one(core, factors, x):
    """Fig. 2(b): aggregation of one polarisation in Tucker format.

    Step 1: the product of U^beta^T with the current vector (no conjugation) gives a
            length-r_beta vector, which multiplies the core matricised as
            r_beta x (r_theta r_phi)  [the paper prints r_theta x r_theta r_phi; the
            inner dimension must be r_beta].
    Step 2: the resulting r_theta r_phi values, arranged as an r_phi x r_theta matrix,
            are multiplied by U^phi from the left (n_phi x r_theta).
    Step 3: the transpose of that (r_theta x n_phi) is multiplied by U^theta from the
            left (n_theta x n_phi).
    Step 4: the n_theta x n_phi result, vectorised, is the group's pattern.
    Returns [N_dir(, R)].
    """
    ut, up, ub = factors
    rt, rp, rb = core.shape
    xm, vec = _as_matrix(x)
    R = xm.shape[1]
    out = np.empty((ut.shape[0] * up.shape[0], R), dtype=np.complex128)
    cmat = np.transpose(core, (2, 0, 1)).reshape(rb, rt * rp)      # [r_beta, (theta', phi')]
    for r in range(R):
        y = ub.T @ xm[:, r]                                         # step 1a: [r_beta]
        t = y @ cmat                                                # step 1b: [r_t r_p]
        m = t.reshape(rt, rp).T                                     # step 2: [r_phi, r_theta]
        m = up @ m                                                  #          [n_phi, r_theta]
        f = ut @ m.T                                                # step 3: [n_theta, n_phi]
        out[:, r] = f.reshape(-1)                                   # step 4
    return out[:, 0] if vec else out


def tucker_disaggregate_one(core, factors, g):
    """Fig. 3(b): disaggregation of one polarisation in Tucker format.

    Step 1: conj(g), arranged as n_theta x n_phi, is multiplied by U^theta^T from the
            left (r_theta x n_phi) and then by U^phi from the right (r_theta x r_phi).
    Step 2: that matrix, vectorised, multiplies the matricised core (r_beta values).
    Step 3: the result is multiplied by U^beta (n_beta values) and conjugated.
    Returns [n_beta(, R)].
    """
    ut, up, ub = factors
    rt, rp, rb = core.shape
    gm, vec = _as_matrix(g)
    R = gm.shape[1]
    out = np.empty((ub.shape[0], R), dtype=np.complex128)
    cmat = np.transpose(core, (2, 0, 1)).reshape(rb, rt * rp)      # [r_beta, (theta', phi')]
    for r in range(R):
        gg = gm[:, r].conj().reshape(ut.shape[0], up.shape[0])      # [n_theta, n_phi]
        s1 = ut.T @ gg                                              # step 1: [r_theta, n_phi]
        s2 = s1 @ up                                                #         [r_theta, r_phi]
        s3 = cmat @ s2.reshape(-1)                                  # step 2: [r_beta]
        out[:, r] = (ub @ s3).conj()                                # step 3
    return out[:, 0] if vec else out


def svd_aggregate_one(w, ub, x):
    """Truncated-SVD aggregation: F = W (U^beta^T x)."""
    return w @ (ub.T @ x)


def svd_disaggregate_one(w, ub, g):
    """Truncated-SVD disaggregation: (W U^beta^T)* g = conj(U^beta) (W^H g)."""
    return ub.conj() @ (w.conj().T @ g)


def tucker_aggregate(tucker_group, x):
    """Both polarisations: ``tucker_group = [(core, factors)] * 2``.  [2, N_dir(, R)]."""
    return np.stack([tucker_aggregate_one(c, f, x) for c, f in tucker_group])


def tucker_disaggregate(tucker_group, g):
    """Sum over both polarisations (eq. (5)).  [n_beta(, R)]."""
    g = np.asarray(g)
    return sum(tucker_disaggregate_one(c, f, g[alpha]) for alpha, (c, f) in enumerate(tucker_group))


# ------------------------------------------------------- whole-problem helpers

def aggregate_all(kind, data, offsets, x):
    """Aggregation over all groups; ``kind`` is 'dense' (data = [N,2,n_t,n_p]),
    'tucker' (data = list of per-group Tucker pairs) or 'svd' (data = list of
    per-group (W, U^beta) pairs).  Returns [G, 2, N_dir(, R)]."""
    out = []
    for g in range(offsets.size - 1):
        xs = x[offsets[g]:offsets[g + 1]]
        if kind == "dense":
            out.append(dense_aggregate(data[offsets[g]:offsets[g + 1]], xs))
        elif kind == "svd":
            out.append(np.stack([svd_aggregate_one(w, ub, xs) for w, ub in data[g]]))
        else:
            out.append(tucker_aggregate(data[g], xs))
    return np.stack(out)


def disaggregate_all(kind, data, offsets, gin):
    """Disaggregation over all groups.  ``gin`` is [G, 2, N_dir(, R)]; returns
    [N(, R)] in group order."""
    out = []
    for g in range(offsets.size - 1):
        if kind == "dense":
            out.append(dense_disaggregate(data[offsets[g]:offsets[g + 1]], gin[g]))
        elif kind == "svd":
            out.append(sum(svd_disaggregate_one(w, ub, gin[g][alpha]) for alpha, (w, ub) in enumerate(data[g])))
        else:
            out.append(tucker_disaggregate(data[g], gin[g]))
    return np.concatenate(out, axis=0)


def rel_err(y, ref):
    """Relative L2 error ||y - ref|| / ||ref|| over all entries."""
    y = np.asarray(y, dtype=np.complex128)
    ref = np.asarray(ref, dtype=np.complex128)
    den = np.linalg.norm(ref)
    return float(np.linalg.norm(y - ref) / den) if den > 0 else float(np.linalg.norm(y))


# --------------------------------------------------------------- brute force

def brute_tucker_aggregate_one(core, factors, x):
    """Quadruple loop over the Tucker model, for tiny inputs only."""
    ut, up, ub = factors
    nt, npp, nb = ut.shape[0], up.shape[0], ub.shape[0]
    rt, rp, rb = core.shape
    out = np.zeros(nt * npp, dtype=np.complex128)
    for it in range(nt):
        for ip in range(npp):
            acc = 0j
            for n in range(nb):
                for a in range(rt):
                    for b in range(rp):
                        for c in range(rb):
                            acc += core[a, b, c] * ut[it, a] * up[ip, b] * ub[n, c] * x[n]
            out[it * npp + ip] = acc
    return out
