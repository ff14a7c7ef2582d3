"""Oracle: truncated higher-order SVD of an aggregation tensor (Section II.B, eq. (6)).

Test infrastructure (see the package docstring).  Plain NumPy, complex128.

The aggregation matrix of one group and polarisation (N_dir x n_beta) is viewed as
the tensor A of shape n_theta x n_phi x n_beta (Fig. 1(a)) and written as
A = C x_1 U^theta x_2 U^phi x_3 U^beta (eq. (6)).  Following Section II.B: the
factor of mode p is the leading part of the left singular vectors of the mode-p
unfolding of A; the core is C = A x_1 U^theta* x_2 U^phi* x_3 U^beta*, with *
the conjugate transpose.

Readings:
* Truncation (Section II.B names a tolerance gamma; Section III.A says the Tucker
  truncation uses gamma / sqrt(3)): in every mode keep the smallest rank r such that
  the discarded singular values satisfy sqrt(sum_{i >= r} s_i^2) <= gamma / sqrt(3) *
  ||A||_F.  By the HOSVD error bound this gives ||A - A_hat||_F <= gamma ||A||_F.
* gamma = 0 keeps every singular value (full multilinear rank).
* One decomposition per group and polarisation.
"""
import numpy as np


def tensorize(dense_group, alpha):
    """[n_beta, 2, n_theta, n_phi] far-field rows -> tensor A [n_theta, n_phi, n_beta]."""
    return np.transpose(dense_group[:, alpha], (1, 2, 0))


def unfold(a, mode):
    """Mode-``mode`` unfolding (0, 1, 2): the mode's index becomes the row index."""
    return np.moveaxis(a, mode, 0).reshape(a.shape[mode], -1)


def truncation_rank(s, threshold):
    """Smallest r with sqrt(sum_{i >= r} s_i^2) <= threshold (s sorted descending)."""
    if threshold <= 0.0:
        return int(s.size)
    tail = np.sqrt(np.cumsum((s ** 2)[::-1]))[::-1]   # tail[i] = sqrt(sum_{j >= i} s_j^2)
    ok = np.nonzero(tail <= threshold)[0]
    r = int(ok[0]) if ok.size else int(s.size)
    return max(r, 1)


def mode_product(a, m, mode):
    """Mode-``mode`` product a x_mode m, with m of shape [new, a.shape[mode]]."""
    moved = np.moveaxis(a, mode, 0)
    out = np.tensordot(m, moved, axes=(1, 0))
    return np.moveaxis(out, 0, mode)


def hosvd(a, gamma):
    """Truncated HOSVD of a 3-way tensor.

    Returns ``core [r_t, r_p, r_b], (U_t [n_t, r_t], U_p [n_p, r_p], U_b [n_b, r_b]),
    sigmas`` where ``sigmas`` holds the three full singular-value vectors.
    """
    norm = np.linalg.norm(a)
    thr = gamma / np.sqrt(3.0) * norm
    factors, sigmas = [], []
    for mode in range(3):
        u, s, _ = np.linalg.svd(unfold(a, mode), full_matrices=False)
        r = truncation_rank(s, thr)
        factors.append(u[:, :r])
        sigmas.append(s)
    core = a
    for mode in range(3):
        core = mode_product(core, factors[mode].conj().T, mode)
    return core, tuple(factors), sigmas


def truncated_svd(a, gamma):
    """The paper's comparison method (Section I; Section II.C, the truncated SVD of
    the aggregation matrix): only the basis mode is compressed.

    The aggregation matrix of one group and polarisation, A (N_dir x n_beta), is the
    transpose of the mode-3 unfolding of the tensor ``a``.  With U^beta the leading
    r_beta left singular vectors of that unfolding, A ~ W U^beta^T with
    W = A conj(U^beta) (N_dir x r_beta).  Reading (the paper gives no rule for the
    SVD rank): the smallest r_beta whose discarded tail satisfies
    sqrt(sum_{i >= r} s_i^2) <= gamma ||A||_F, so that ||A - W U^beta^T||_F <= gamma ||A||_F.

    Returns ``W [N_dir, r_beta], U_b [n_beta, r_beta], s`` (s: all singular values).
    """
    amat = unfold(a, 2)                               # [n_beta, N_dir]
    u, s, _ = np.linalg.svd(amat, full_matrices=False)
    r = truncation_rank(s, gamma * np.linalg.norm(a))
    ub = u[:, :r]
    w = amat.T @ ub.conj()                            # A conj(U^beta), [N_dir, r_beta]
    return w, ub, s


def svd_memory(n_beta, n_dir, r_beta, elem_bytes=16):
    """Stored bytes of the truncated-SVD method: U^beta and W."""
    return elem_bytes * (n_beta * r_beta + n_dir * r_beta)


def reconstruct(core, factors):
    """A_hat = C x_1 U^theta x_2 U^phi x_3 U^beta (eq. (6))."""
    out = core
    for mode in range(3):
        out = mode_product(out, factors[mode], mode)
    return out


def compress_all_svd(dense, offsets, gamma):
    """Truncated SVD of every (group, polarisation): a list over groups of
    ``[(W, U_b) for alpha in (0, 1)]``."""
    out = []
    for g in range(offsets.size - 1):
        blk = dense[offsets[g]:offsets[g + 1]]
        out.append([truncated_svd(tensorize(blk, alpha), gamma)[:2] for alpha in range(2)])
    return out


def compress_all(dense, offsets, gamma):
    """HOSVD of every (group, polarisation) of a dense far-field [N,2,n_t,n_p].

    Returns a list over groups of ``[(core, factors) for alpha in (0, 1)]``.
    """
    out = []
    for g in range(offsets.size - 1):
        blk = dense[offsets[g]:offsets[g + 1]]
        per_alpha = []
        for alpha in range(2):
            core, fac, _ = hosvd(tensorize(blk, alpha), gamma)
            per_alpha.append((core, fac))
        out.append(per_alpha)
    return out
