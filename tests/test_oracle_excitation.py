"""Pins of the oracle's plane-wave excitation vectors, eq. (2) (CPU only)."""
import math

import numpy as np

import synth
from oracle import geometry as geo
from oracle import farfield as ff
from oracle import excitation as ex


def _problem(freq, radius, k=2 * math.pi, n_theta=6, n_phi=11, box=None, K=1):
    v, t = synth.icosphere(freq, radius)
    box = box or 2.0 * radius
    return geo.Problem(v, t, (-radius,) * 3, box, K, n_theta, n_phi, k=k)


def test_static_limit_closed_form():
    """k -> 0: V_m = -e . int b_m = -e . l_m (r_c- - r_c+), the centroid difference,
    exactly for the 3-point rule (it integrates linear functions exactly)."""
    P = _problem(4, 0.7, k=0.0)
    b = P.rwg
    khat, epol = synth.planewaves(synth.rng(3), 5)
    got = ex.planewave_excitation(P, khat, epol)
    cen = P.verts[P.tris].mean(axis=1)
    vec = b["length"][:, None] * (cen[b["tri_m"]] - cen[b["tri_p"]])
    want = -(vec @ epol.T)
    assert np.max(np.abs(got - want)) < 1e-15 * 10
    assert np.max(np.abs(got.imag)) == 0.0


def test_reversed_grid_wave_is_the_far_field():
    """A wave travelling along -k_i with polarisation alpha_i (a direction and
    polarisation of the grid) gives V_m = -exp(j k k_i . r_v) P^{alpha,+}_{m,i} of
    eq. (4): the integrand of eq. (4) with the phase reference moved from the box
    centre r_v to the origin, and the sign of eq. (2)."""
    P = _problem(3, 0.5, n_theta=4, n_phi=7, box=0.5, K=2)
    g = int(np.argmax(P.group_sizes()))
    lo, hi = int(P.offsets[g]), int(P.offsets[g + 1])
    pf = ff.farfield_group(P, g).reshape(hi - lo, 2, P.n_dir)
    for i in (0, 5, P.n_dir - 1):
        phase = np.exp(1j * P.k * (P.khat[i] @ P.centers[g]))
        for a, pol in enumerate((P.that[i], P.phat[i])):
            got = ex.planewave_excitation(P, -P.khat[i][None, :], pol[None, :])[lo:hi, 0]
            want = -phase * pf[:, a, i]
            assert np.max(np.abs(got - want)) < 1e-14 * np.max(np.abs(want)), (i, a)


def test_columns_are_independent_waves():
    """Column r depends only on wave r (up to the rounding of the BLAS products), and
    the call is linear in the polarisation."""
    P = _problem(3, 0.5)
    khat, epol = synth.planewaves(synth.rng(5), 4)
    all4 = ex.planewave_excitation(P, khat, epol)
    for r in range(4):
        one = ex.planewave_excitation(P, khat[r], epol[r])
        assert np.max(np.abs(one[:, 0] - all4[:, r])) < 1e-15 * np.max(np.abs(all4[:, r]))
    e2 = np.cross(khat, epol)
    mix = ex.planewave_excitation(P, khat, 2.0 * epol - 3.0 * e2)
    sep = 2.0 * all4 - 3.0 * ex.planewave_excitation(P, khat, e2)
    assert np.max(np.abs(mix - sep)) < 1e-14 * np.max(np.abs(sep))


def test_three_point_rule_converges_second_order():
    """The 3-point rule against the high-order rule: the error relative to the value
    falls about 4x per halving of the element size (O((kh)^2), as for eq. (4))."""
    khat, epol = synth.planewaves(synth.rng(7), 3)
    errs = []
    for f in (4, 8, 16):      # (f = 2 is not yet in the asymptotic range)
        P = _problem(f, 0.5)
        rows = synth.rng(f).choice(P.n_basis, size=10, replace=False)
        v3 = ex.planewave_excitation(P, khat, epol)[rows]
        e = [np.max(np.abs(v3[j] - ex.planewave_highorder(P, row, khat, epol, n=16))) / np.max(np.abs(v3[j]))
             for j, row in enumerate(rows)]
        errs.append(max(e))
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 3.5 < r1 < 5.5 and 3.5 < r2 < 5.5, errs


def test_planewave_draws():
    """Directions are unit vectors and the polarisations theta_hat are unit and
    orthogonal to them (seeded, reproducible)."""
    k1, e1 = synth.planewaves(synth.rng(2), 64)
    k2, e2 = synth.planewaves(synth.rng(2), 64)
    assert np.array_equal(k1, k2) and np.array_equal(e1, e2)
    assert np.allclose(np.linalg.norm(k1, axis=1), 1.0, atol=1e-15)
    assert np.allclose(np.linalg.norm(e1, axis=1), 1.0, atol=1e-15)
    assert np.max(np.abs(np.sum(k1 * e1, axis=1))) < 1e-15
    # theta_hat points towards increasing theta: its z component is -sin(theta) <= 0
    assert np.all(e1[:, 2] <= 0.0)
