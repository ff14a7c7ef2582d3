"""Pins of the oracle's box-grid spectra (eq. (3), eq. (5); CPU only).

The placement is checked against the mesh itself: every basis function's edge
midpoint must lie in the box whose fibre holds its group's spectrum, with the box
found here by plain coordinate comparison; and against a row-major enumeration of
a non-cubic grid written as nested loops.
"""
import numpy as np
import pytest

import synth
from synth import workloads as W
from oracle import boxgrid as bg
from oracle import geometry as geo
from oracle import products as pr


def small_problem():
    w = W.SMALL
    v, t = synth.icosphere(w.freq, w.radius)
    return w, geo.Problem(v, t, w.origin, w.box, w.boxes_per_axis, w.n_theta, w.n_phi)


def cubic_boxes(P, K):
    ix, iy, iz = P.box_index.T
    return (ix * K + iy) * K + iz


def test_fibres_sit_in_the_box_of_their_basis_functions():
    w, P = small_problem()
    K = w.boxes_per_axis
    dims = (K, K, K)
    # group g's spectrum is the constant g + 1 (polarisation 0) and -(g + 1) (polarisation 1)
    f = np.zeros((P.n_groups, 2, 3), np.complex128)
    f[:, 0] = (np.arange(P.n_groups) + 1)[:, None]
    f[:, 1] = -f[:, 0]
    grid = bg.scatter(f, cubic_boxes(P, K), dims)
    assert grid.shape == (2, K, K, K, 3)
    mid = 0.5 * (P.verts[P.rwg["edge"][:, 0]] + P.verts[P.rwg["edge"][:, 1]])
    origin = np.asarray(w.origin)
    owner = P.group_of_basis()
    occupied = set()
    for n in range(P.n_basis):
        # the box [origin + v box, origin + (v + 1) box) on each axis that holds the midpoint
        v = [0, 0, 0]
        for c in range(3):
            lo = [origin[c] + j * w.box for j in range(K)]
            v[c] = max(j for j in range(K) if lo[j] <= mid[n, c] + 1e-12)
        occupied.add(tuple(v))
        assert np.all(grid[0][tuple(v)] == owner[n] + 1), n
        assert np.all(grid[1][tuple(v)] == -(owner[n] + 1)), n
    assert len(occupied) == P.n_groups
    for v in np.ndindex(K, K, K):
        if v not in occupied:
            assert not np.any(grid[:, v[0], v[1], v[2]])


def test_row_major_enumeration_of_a_noncubic_grid():
    dims = (3, 4, 5)
    rng = synth.rng(3)
    boxes = rng.choice(60, size=17, replace=False)
    f = synth.complex_normal(rng, (17, 2, 6, 2))
    grid = bg.scatter(f, boxes, dims)
    lin = 0
    where = {}
    for vx in range(3):
        for vy in range(4):
            for vz in range(5):
                where[lin] = (vx, vy, vz)
                lin += 1
    for g, b in enumerate(boxes):
        assert np.array_equal(grid[:, where[b][0], where[b][1], where[b][2]], f[g])
    assert np.count_nonzero(np.abs(grid).sum(axis=(0, 4, 5))) == 17


def test_gather_is_the_adjoint_of_scatter():
    dims = (2, 3, 4)
    rng = synth.rng(4)
    boxes = rng.choice(24, size=9, replace=False)
    f = synth.complex_normal(rng, (9, 2, 5))
    gg = synth.complex_normal(rng, (2,) + dims + (5,))
    assert np.array_equal(bg.gather(bg.scatter(f, boxes, dims), boxes, dims), f)
    lhs = np.vdot(bg.scatter(f, boxes, dims), gg)
    rhs = np.vdot(f, bg.gather(gg, boxes, dims))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_disaggregation_never_reads_empty_boxes():
    dims = (2, 2, 3)
    rng = synth.rng(5)
    lay_offsets = np.array([0, 3, 4, 9])
    boxes = np.array([7, 0, 11])
    dense = synth.complex_normal(rng, (9, 2, 2, 3))
    gg = synth.complex_normal(rng, (2,) + dims + (6,))
    junk = gg.copy()
    empty = [b for b in range(12) if b not in boxes]
    for b in empty:
        v = np.unravel_index(b, dims)
        junk[:, v[0], v[1], v[2]] = np.nan
    a = bg.disaggregate_grid("dense", dense, lay_offsets, gg, boxes, dims)
    b = bg.disaggregate_grid("dense", dense, lay_offsets, junk, boxes, dims)
    assert np.array_equal(a, b)
    # and the grid aggregation of a group equals its dense aggregation (eq. (3))
    x = synth.complex_normal(rng, 9)
    fgrid = bg.aggregate_grid("dense", dense, lay_offsets, x, boxes, dims)
    v = np.unravel_index(7, dims)
    assert np.allclose(fgrid[:, v[0], v[1], v[2]], pr.dense_aggregate(dense[0:3], x[0:3]))


@pytest.mark.parametrize("w", [W.SMALL, W.SPHERE6], ids=lambda w: w.name)
def test_box_multi_index_matches_the_grouping(w):
    v, t = synth.icosphere(w.freq, w.radius)
    P = geo.Problem(v, t, w.origin, w.box, w.boxes_per_axis, w.n_theta, w.n_phi)
    K = w.boxes_per_axis
    assert np.array_equal(bg.box_multi_index(cubic_boxes(P, K), (K, K, K)), P.box_index)
