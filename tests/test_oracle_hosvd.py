"""Pins of the oracle's truncated HOSVD, Section II.B (CPU only)."""
import json
import math
import os

import numpy as np
import pytest

import synth
from synth import workloads as W
from oracle import geometry as geo
from oracle import farfield as ff
from oracle import hosvd as H


@pytest.fixture(scope="module")
def small():
    w = W.SMALL
    v, t = synth.icosphere(w.freq, w.radius)
    P = geo.Problem(v, t, w.origin, w.box, w.boxes_per_axis, w.n_theta, w.n_phi)
    D = ff.farfield_all(P)
    return P, D


def _exact_low_rank(rng, shape, ranks):
    """A tensor with exact multilinear ranks built in the test from random parts."""
    core = synth.complex_normal(rng, ranks)
    fac = [np.linalg.qr(synth.complex_normal(rng, (n, r)))[0] for n, r in zip(shape, ranks)]
    a = core
    for m in range(3):
        a = np.moveaxis(np.tensordot(fac[m], np.moveaxis(a, m, 0), axes=(1, 0)), 0, m)
    return a


def test_recovers_exact_multilinear_ranks():
    rng = np.random.default_rng(7)
    a = _exact_low_rank(rng, (9, 13, 20), (3, 5, 7))
    core, fac, _ = H.hosvd(a, 1e-10)
    assert core.shape == (3, 5, 7)
    assert np.linalg.norm(H.reconstruct(core, fac) - a) / np.linalg.norm(a) < 1e-13


def test_full_rank_is_exact(small):
    P, D = small
    a = H.tensorize(D[P.offsets[0]:P.offsets[1]], 0)
    core, fac, sig = H.hosvd(a, 0.0)
    assert core.shape == (a.shape[0], a.shape[1], a.shape[2])
    assert np.linalg.norm(H.reconstruct(core, fac) - a) / np.linalg.norm(a) < 1e-13
    # all-orthogonality of the full core: C_(p) C_(p)^H = diag(sigma^(p)^2)
    nrm2 = np.linalg.norm(a) ** 2
    for m in range(3):
        cm = H.unfold(core, m)
        assert np.allclose(cm @ cm.conj().T, np.diag(sig[m] ** 2), atol=1e-12 * nrm2)


def test_tensorize_is_the_aggregation_matrix(small):
    P, D = small
    blk = D[P.offsets[2]:P.offsets[3]]
    a = H.tensorize(blk, 1)
    i_t, i_p, n = 4, 7, 11
    assert a[i_t, i_p, n] == blk[n, 1, i_t, i_p]
    # mode-3 unfolding rows are the basis functions' patterns
    u3 = H.unfold(a, 2)
    assert np.array_equal(u3[n], blk[n, 1].reshape(-1))


@pytest.mark.parametrize("gamma", [1e-3, 1e-4, 1e-6])
def test_invariants(small, gamma):
    P, D = small
    for g in (0, 5):
        for alpha in (0, 1):
            a = H.tensorize(D[P.offsets[g]:P.offsets[g + 1]], alpha)
            core, fac, sig = H.hosvd(a, gamma)
            nrm = np.linalg.norm(a)
            ahat = H.reconstruct(core, fac)
            # error bound of the truncated HOSVD
            assert np.linalg.norm(a - ahat) <= gamma * nrm * (1 + 1e-9)
            # orthonormal factors
            for u in fac:
                assert np.allclose(u.conj().T @ u, np.eye(u.shape[1]), atol=1e-13)
            # ||C|| = ||A_hat||; slice energies of the core never exceed sigma_i^2
            assert abs(np.linalg.norm(core) - np.linalg.norm(ahat)) < 1e-13 * nrm
            for m in range(3):
                cm = H.unfold(core, m)
                energy = np.sum(np.abs(cm) ** 2, axis=1)
                assert np.all(energy <= sig[m][:cm.shape[0]] ** 2 * (1 + 1e-12))
            # minimal ranks: one fewer column would break the per-mode threshold
            thr = gamma / math.sqrt(3) * nrm
            for m, s in enumerate(sig):
                r = fac[m].shape[1]
                assert math.sqrt(np.sum(s[r:] ** 2)) <= thr
                if r > 1:
                    assert math.sqrt(np.sum(s[r - 1:] ** 2)) > thr


def test_truncation_rank_edge_cases():
    s = np.array([3.0, 2.0, 1.0, 0.0])
    assert H.truncation_rank(s, 0.0) == 4           # gamma = 0 keeps everything
    assert H.truncation_rank(s, 1.0) == 2           # tail [1, 0] has norm 1 <= 1
    assert H.truncation_rank(s, 0.999) == 3
    assert H.truncation_rank(s, 100.0) == 1         # never below rank one


@pytest.mark.slow
def test_sphere_ranks_near_table_iv(golden_dir):
    """Ranks of a typical 2-lambda group of the 30-lambda sphere lie near Table IV.
    A sanity band only: the paper's mesh and quadrature differ."""
    ref = json.load(open(os.path.join(golden_dir, "paper_sphere_ranks.json")))
    rt, rp, rb = ref["box_lambda_to_ranks"]["2.0"]
    w = W.SPHERE30
    v, t = synth.icosphere(w.freq, w.radius)
    P = geo.Problem(v, t, w.origin, w.box, w.boxes_per_axis, w.n_theta, w.n_phi)
    nb = P.group_sizes()
    g = int(np.argmin(np.abs(nb - ref["box_lambda_to_nbeta"]["2.0"])))
    a = H.tensorize(ff.farfield_group(P, g), 0)
    core, _, _ = H.hosvd(a, ref["gamma"])
    got = core.shape
    assert abs(got[0] - rt) <= 0.2 * rt and abs(got[1] - rp) <= 0.2 * rp
    assert abs(got[2] - rb) <= 0.25 * rb, got


# ---------------------------------------------------------------- truncated SVD

def test_svd_full_rank_is_exact(small):
    P, D = small
    blk = D[P.offsets[2]:P.offsets[3]]
    a = H.tensorize(blk, 1)
    w, ub, s = H.truncated_svd(a, 0.0)
    amat = blk[:, 1].reshape(blk.shape[0], -1).T          # [N_dir, n_beta]
    assert ub.shape[1] == min(amat.shape)
    assert np.linalg.norm(w @ ub.T - amat) <= 1e-12 * np.linalg.norm(amat)


@pytest.mark.parametrize("gamma", [1e-2, 1e-4, 1e-6])
def test_svd_is_the_best_approximation_of_its_rank(small, gamma):
    """Eckart-Young: the error of W U^beta^T equals the discarded singular-value tail,
    it meets the gamma bound, and one rank less would not."""
    P, D = small
    blk = D[P.offsets[5]:P.offsets[6]]
    a = H.tensorize(blk, 0)
    amat = blk[:, 0].reshape(blk.shape[0], -1).T
    w, ub, s = H.truncated_svd(a, gamma)
    r = ub.shape[1]
    err = np.linalg.norm(w @ ub.T - amat)
    tail = np.sqrt(np.sum(s[r:] ** 2))
    assert abs(err - tail) <= 1e-10 * np.linalg.norm(amat)
    assert err <= gamma * np.linalg.norm(amat) * (1 + 1e-12)
    if r > 1:
        assert np.sqrt(np.sum(s[r - 1:] ** 2)) > gamma * np.linalg.norm(amat)
    # orthonormal basis factor
    assert np.allclose(ub.conj().T @ ub, np.eye(r), atol=1e-12)


def test_svd_memory_ratio_near_table_iii(golden_dir):
    """On a typical 2-lambda group of the 30-lambda sphere the SVD method stores about
    twice what Tucker stores at gamma = 1e-6, as in Table III.  A sanity band: the
    paper's totals are over its own mesh."""
    ref = json.load(open(os.path.join(golden_dir, "paper_sphere_svd_vs_tucker.json")))
    paper_ratio = ref["svd_mb"]["1e-6"] / ref["tucker_mb"]["1e-6"]
    w = W.SPHERE30
    v, t = synth.icosphere(w.freq, w.radius)
    P = geo.Problem(v, t, w.origin, w.box, w.boxes_per_axis, w.n_theta, w.n_phi)
    nb = P.group_sizes()
    g = int(np.argmin(np.abs(nb - 909)))
    a = H.tensorize(ff.farfield_group(P, g), 0)
    core, (ut, up, ubt), _ = H.hosvd(a, 1e-6)
    wm, ubs, _ = H.truncated_svd(a, 1e-6)
    tucker = core.size + ut.size + up.size + ubt.size
    svd = H.svd_memory(a.shape[2], a.shape[0] * a.shape[1], ubs.shape[1], 1)
    ratio = svd / tucker
    assert 0.7 * paper_ratio <= ratio <= 1.4 * paper_ratio, (ratio, paper_ratio)
