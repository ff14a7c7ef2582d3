"""Seeded random draws: complex Gaussian vectors, directions, random Tucker factors."""
import numpy as np


def rng(seed):
    """``numpy.random.default_rng(seed)`` (PCG64)."""
    return np.random.default_rng(seed)


def complex_normal(gen, shape, dtype=np.complex128):
    """Circular complex Gaussian CN(0, 1): ``(N(0,1) + j N(0,1)) / sqrt(2)``."""
    re = gen.standard_normal(shape)
    im = gen.standard_normal(shape)
    out = np.empty(shape, dtype=np.complex128)
    out.real = re
    out.imag = im
    out *= 2.0 ** -0.5
    return out.astype(dtype, copy=False)


def unit_vectors(gen, count):
    """Directions uniform on the unit sphere (normalised N(0, I_3) draws), [count, 3]."""
    v = gen.standard_normal((count, 3))
    return v / np.linalg.norm(v, axis=1, keepdims=True)


def planewaves(gen, count):
    """Incident plane waves for many right-hand sides: propagation directions uniform on
    the unit sphere (:func:`unit_vectors`) and polarisation theta_hat of each direction,
    (cos t cos p, cos t sin p, -sin t) with t, p the direction's polar angles.
    Returns ``(khat [count, 3], epol [count, 3])``."""
    k = unit_vectors(gen, count)
    t = np.arccos(np.clip(k[:, 2], -1.0, 1.0))
    p = np.arctan2(k[:, 1], k[:, 0])
    e = np.stack([np.cos(t) * np.cos(p), np.cos(t) * np.sin(p), -np.sin(t)], axis=1)
    return k, e


def synthetic_ranks(gen, nb, n_theta, n_phi):
    """Random multilinear ranks (r_theta, r_phi, r_beta) for one tensor of shape
    n_theta x n_phi x nb, each between 1 and its mode size."""
    rt = int(gen.integers(1, n_theta + 1))
    rp = int(gen.integers(1, n_phi + 1))
    rb = int(gen.integers(1, nb + 1))
    return rt, rp, rb


def synthetic_tucker(gen, n_theta, n_phi, nb, rt, rp, rb, decay=0.5):
    """Random core and factors with the shapes of one Tucker-compressed tensor.

    Returns ``(core [rt, rp, rb], Ut [n_theta, rt], Up [n_phi, rp], Ub [nb, rb])``,
    complex128.  Factor columns are CN(0, 1/n) so they have roughly unit norm; the
    core entries are CN(0, 1) scaled by ``exp(-decay * (i/rt + j/rp + k/rb) * 4)``
    so that, as in a compressed far-field, most of the energy sits in the leading
    slices.
    """
    ut = complex_normal(gen, (n_theta, rt)) / np.sqrt(n_theta)
    up = complex_normal(gen, (n_phi, rp)) / np.sqrt(n_phi)
    ub = complex_normal(gen, (nb, rb)) / np.sqrt(nb)
    core = complex_normal(gen, (rt, rp, rb))
    i = np.arange(rt)[:, None, None] / max(rt, 1)
    j = np.arange(rp)[None, :, None] / max(rp, 1)
    k = np.arange(rb)[None, None, :] / max(rb, 1)
    core *= np.exp(-decay * 4.0 * (i + j + k))
    return core, ut, up, ub
