"""Pins of the oracle's far-field signatures, eq. (4) (CPU only)."""
import math

import numpy as np
import pytest

import synth
from synth import workloads as W
from oracle import geometry as geo
from oracle import farfield as ff


def _problem(freq, radius, k=2 * math.pi, box=None, n_theta=6, n_phi=11):
    v, t = synth.icosphere(freq, radius)
    box = box or 2.0 * radius
    return geo.Problem(v, t, (-radius,) * 3, box, 1, n_theta, n_phi, k=k)


def test_static_limit_closed_form():
    """k -> 0: the integral of b_n is l_n (r_c- - r_c+), the centroid difference
    (exact for the 3-point rule, which integrates linear functions exactly)."""
    P = _problem(4, 0.7, k=0.0)
    b = P.rwg
    rows = np.arange(P.n_basis)
    c = np.repeat(P.centers[:1], rows.size, axis=0)
    got = ff.farfield_rows(P, rows, P.khat, P.that, P.phat, c)
    cen = P.verts[P.tris].mean(axis=1)
    vec = b["length"][:, None] * (cen[b["tri_m"]] - cen[b["tri_p"]])      # [N, 3]
    exp_t = vec @ P.that.T
    exp_p = vec @ P.phat.T
    assert np.max(np.abs(got[:, 0] - exp_t)) < 1e-15 * 10
    assert np.max(np.abs(got[:, 1] - exp_p)) < 1e-15 * 10
    assert np.max(np.abs(got.imag)) == 0.0
    # same thing from the free vertices: l_n / 3 (p- - p+)
    vec2 = b["length"][:, None] / 3.0 * (P.verts[b["free_m"]] - P.verts[b["free_p"]])
    assert np.allclose(vec, vec2, atol=1e-15)


def test_phase_centre_shift():
    """Moving the phase centre by d multiplies P^{alpha,+} by exp(-j k k_i . d)."""
    P = _problem(3, 0.5)
    rows = np.arange(0, P.n_basis, 7)
    c0 = np.zeros((rows.size, 3))
    d = np.array([0.13, -0.21, 0.07])
    a = ff.farfield_rows(P, rows, P.khat, P.that, P.phat, c0)
    b = ff.farfield_rows(P, rows, P.khat, P.that, P.phat, c0 + d)
    ph = np.exp(-1j * P.k * (P.khat @ d))
    assert np.max(np.abs(b - a * ph[None, None, :])) < 1e-14 * np.max(np.abs(a))


def test_receive_pattern_is_conjugate():
    """P^{alpha,-} = conj(P^{alpha,+}) for real basis functions (end of Section II.A)."""
    P = _problem(3, 0.5)
    rows = np.arange(P.n_basis)
    c = np.repeat(P.centers[:1], rows.size, axis=0)
    p = ff.farfield_rows(P, rows, P.khat, P.that, P.phat, c, sign=+1)
    m = ff.farfield_rows(P, rows, P.khat, P.that, P.phat, c, sign=-1)
    assert np.max(np.abs(m - p.conj())) < 1e-15


def test_highorder_rule_is_converged():
    P = _problem(2, 0.5)
    for row in (0, 5, 17):
        a = ff.farfield_highorder(P, row, P.khat, P.that, P.phat, P.centers[0], n=16)
        b = ff.farfield_highorder(P, row, P.khat, P.that, P.phat, P.centers[0], n=24)
        assert np.max(np.abs(a - b)) < 1e-14 * np.max(np.abs(b))


def test_three_point_rule_converges_second_order():
    """Error of the degree-2 rule relative to the high-order rule falls ~4x per
    halving of the element size h.  The rule misses the cubic Taylor terms of
    rho * exp(j k k.r); since b_n = l_n/(2A) rho with |rho| ~ h, the leading missed
    term is (r - r0) (k s)^2 / 2, an O(h^4 k^2) error on an O(h^2) value: O((kh)^2)."""
    errs = []
    for f in (2, 4, 8):
        P = _problem(f, 0.5, n_theta=5, n_phi=9)
        rng = np.random.default_rng(f)
        rows = rng.choice(P.n_basis, size=12, replace=False)
        c = np.repeat(P.centers[:1], rows.size, axis=0)
        p3 = ff.farfield_rows(P, rows, P.khat, P.that, P.phat, c)
        e = []
        for j, row in enumerate(rows):
            ph = ff.farfield_highorder(P, row, P.khat, P.that, P.phat, P.centers[0], n=16)
            e.append(np.max(np.abs(p3[j] - ph)) / np.max(np.abs(ph)))
        errs.append(max(e))
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 3.5 < r1 < 5.5 and 3.5 < r2 < 5.0, errs


def test_small_workload_dense_shape_and_layout():
    w = W.SMALL
    v, t = synth.icosphere(w.freq, w.radius)
    P = geo.Problem(v, t, w.origin, w.box, w.boxes_per_axis, w.n_theta, w.n_phi)
    D = ff.farfield_group(P, 3)
    assert D.shape == (P.group_sizes()[3], 2, w.n_theta, w.n_phi)
    # direction (i_theta, i_phi) of the dense layout is row i_theta * n_phi + i_phi
    lo = P.offsets[3]
    rows = np.array([lo + 2])
    it, ip = 5, 9
    i = it * w.n_phi + ip
    one = ff.farfield_rows(P, rows, P.khat[i:i + 1], P.that[i:i + 1], P.phat[i:i + 1], P.centers[3:4])
    assert np.allclose(D[2, :, it, ip], one[0, :, 0], rtol=0, atol=1e-15)
