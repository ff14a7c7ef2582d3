"""Pins of the oracle's dense and Tucker aggregation / disaggregation (CPU only)."""
import numpy as np
import pytest

import synth
from synth import workloads as W
from oracle import geometry as geo
from oracle import farfield as ff
from oracle import hosvd as H
from oracle import products as pr


@pytest.fixture(scope="module")
def small():
    w = W.SMALL
    v, t = synth.icosphere(w.freq, w.radius)
    P = geo.Problem(v, t, w.origin, w.box, w.boxes_per_axis, w.n_theta, w.n_phi)
    D = ff.farfield_all(P)
    return P, D


def test_dense_against_loops():
    rng = np.random.default_rng(3)
    nb, nt, npp = 4, 3, 5
    blk = synth.complex_normal(rng, (nb, 2, nt, npp))
    x = synth.complex_normal(rng, nb)
    g = synth.complex_normal(rng, (2, nt * npp))
    f = pr.dense_aggregate(blk, x)
    v = pr.dense_disaggregate(blk, g)
    for a in range(2):
        for it in range(nt):
            for ip in range(npp):
                ref = sum(blk[n, a, it, ip] * x[n] for n in range(nb))
                assert abs(f[a, it * npp + ip] - ref) < 1e-14
    for n in range(nb):
        ref = sum(np.conj(blk[n, a, it, ip]) * g[a, it * npp + ip]
                  for a in range(2) for it in range(nt) for ip in range(npp))
        assert abs(v[n] - ref) < 1e-13


def test_tucker_against_brute_force():
    rng = np.random.default_rng(4)
    for (nt, npp, nb, rt, rp, rb) in [(3, 3, 5, 2, 3, 4), (2, 4, 6, 1, 2, 6), (3, 2, 1, 3, 2, 1)]:
        core, ut, up, ub = synth.synthetic_tucker(rng, nt, npp, nb, rt, rp, rb)
        x = synth.complex_normal(rng, nb)
        got = pr.tucker_aggregate_one(core, (ut, up, ub), x)
        ref = pr.brute_tucker_aggregate_one(core, (ut, up, ub), x)
        assert np.max(np.abs(got - ref)) < 1e-13
        # disaggregation against the conjugate transpose of the brute-force matrix
        amat = np.stack([pr.brute_tucker_aggregate_one(core, (ut, up, ub), e)
                         for e in np.eye(nb)], axis=1)                     # [N_dir, nb]
        g = synth.complex_normal(rng, nt * npp)
        assert np.max(np.abs(pr.tucker_disaggregate_one(core, (ut, up, ub), g)
                             - amat.conj().T @ g)) < 1e-13


def test_full_rank_tucker_equals_dense(small):
    """gamma = 0: the Tucker chain reproduces the plain products with A itself."""
    P, D = small
    rng = synth.rng(0)
    for g in (0, 7):
        blk = D[P.offsets[g]:P.offsets[g + 1]]
        tg = [(c, f) for c, f, _ in (H.hosvd(H.tensorize(blk, a), 0.0) for a in range(2))]
        x = synth.complex_normal(rng, blk.shape[0])
        gin = synth.complex_normal(rng, (2, P.n_dir))
        assert pr.rel_err(pr.tucker_aggregate(tg, x), pr.dense_aggregate(blk, x)) < 1e-13
        assert pr.rel_err(pr.tucker_disaggregate(tg, gin), pr.dense_disaggregate(blk, gin)) < 1e-13


def test_tucker_equals_dense_of_reconstruction_and_error_bound(small):
    P, D = small
    rng = synth.rng(1)
    for g in range(P.n_groups):
        blk = D[P.offsets[g]:P.offsets[g + 1]]
        parts = [H.hosvd(H.tensorize(blk, a), 1e-6) for a in range(2)]
        tg = [(c, f) for c, f, _ in parts]
        rec = np.stack([np.transpose(H.reconstruct(c, f), (2, 0, 1)) for c, f in tg], axis=1)
        x = synth.complex_normal(rng, blk.shape[0])
        f_t = pr.tucker_aggregate(tg, x)
        assert pr.rel_err(f_t, pr.dense_aggregate(rec, x)) < 1e-13
        # compression error: ||(A - A_hat) x|| <= gamma ||A||_F ||x||
        for a in range(2):
            err = np.linalg.norm(f_t[a] - pr.dense_aggregate(blk, x)[a])
            assert err <= 1e-6 * np.linalg.norm(blk[:, a]) * np.linalg.norm(x)


def test_adjoint_identity_and_round_trip(small):
    P, D = small
    rng = synth.rng(2)
    x = synth.complex_normal(rng, P.n_basis)
    gin = synth.complex_normal(rng, (P.n_groups, 2, P.n_dir))
    tuck = H.compress_all(D, P.offsets, 1e-6)
    for kind, data in (("dense", D), ("tucker", tuck)):
        f = pr.aggregate_all(kind, data, P.offsets, x)
        v = pr.disaggregate_all(kind, data, P.offsets, gin)
        lhs = np.vdot(gin, f)            # G^H (A x)
        rhs = np.vdot(v, x)              # (A^H G)^H x
        assert abs(lhs - rhs) < 1e-12 * abs(rhs)
        vv = pr.disaggregate_all(kind, data, P.offsets, f)
        rt = np.vdot(x, vv)
        assert abs(rt.imag) < 1e-12 * abs(rt.real)
        assert abs(rt.real - np.vdot(f, f).real) < 1e-12 * rt.real


def test_multi_rhs_is_columnwise(small):
    P, D = small
    rng = synth.rng(3)
    blk = D[P.offsets[1]:P.offsets[2]]
    tg = [(c, f) for c, f, _ in (H.hosvd(H.tensorize(blk, a), 1e-4) for a in range(2))]
    X = synth.complex_normal(rng, (blk.shape[0], 3))
    Gm = synth.complex_normal(rng, (2, P.n_dir, 3))
    F = pr.tucker_aggregate(tg, X)
    V = pr.tucker_disaggregate(tg, Gm)
    for r in range(3):
        assert np.allclose(F[..., r], pr.tucker_aggregate(tg, X[:, r]), atol=1e-14)
        assert np.allclose(V[:, r], pr.tucker_disaggregate(tg, Gm[..., r]), atol=1e-14)
    assert np.allclose(pr.dense_aggregate(blk, X)[..., 2], pr.dense_aggregate(blk, X[:, 2]))


def test_identity_angular_factors_reduce_to_svd_method(small):
    """With U^theta = I and U^phi = I only the basis mode is compressed: the chain
    becomes the truncated-SVD product U^beta-projected (Section II.C, last paragraph)."""
    P, D = small
    blk = D[P.offsets[4]:P.offsets[5]]
    a = H.tensorize(blk, 0)
    u, s, _ = np.linalg.svd(H.unfold(a, 2), full_matrices=False)
    ub = u[:, :40]
    core = H.mode_product(a, ub.conj().T, 2)
    fac = (np.eye(P.n_theta), np.eye(P.n_phi), ub)
    x = synth.complex_normal(synth.rng(5), blk.shape[0])
    amat = blk[:, 0].reshape(blk.shape[0], -1).T                 # [N_dir, nb]
    svd_prod = (amat @ ub.conj()) @ (ub.T @ x)
    assert pr.rel_err(pr.tucker_aggregate_one(core, fac, x), svd_prod) < 1e-13


def test_svd_products_match_the_explicit_operator(small):
    """SVD-method aggregation / disaggregation equal the explicit W U^beta^T and its
    conjugate transpose, satisfy the adjoint identity, and agree with the dense
    products within gamma."""
    P, D = small
    gamma = 1e-4
    data = H.compress_all_svd(D, P.offsets, gamma)
    rng = synth.rng(21)
    x = synth.complex_normal(rng, P.n_basis)
    gin = synth.complex_normal(rng, (P.n_groups, 2, P.n_dir))
    f = pr.aggregate_all("svd", data, P.offsets, x)
    v = pr.disaggregate_all("svd", data, P.offsets, gin)
    for g in range(P.n_groups):
        lo, hi = P.offsets[g], P.offsets[g + 1]
        for alpha in range(2):
            w, ub = data[g][alpha]
            op = w @ ub.T
            assert pr.rel_err(f[g, alpha], op @ x[lo:hi]) < 1e-13
    # adjoint identity over the whole problem
    lhs = np.vdot(gin, f)
    rhs = np.vdot(v, x)
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)
    assert pr.rel_err(f, pr.aggregate_all("dense", D, P.offsets, x)) < 10 * gamma
    assert pr.rel_err(v, pr.disaggregate_all("dense", D, P.offsets, gin)) < 10 * gamma
