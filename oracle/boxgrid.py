"""Oracle: spectra on the FMM-FFT box grid (Section II.A, eq. (3) and eq. (5)).

Test infrastructure (see the package docstring).  Plain NumPy, complex128.

The outgoing spectra of eq. (3) are indexed by u = (v_x, v_y, v_z, i): per
polarisation a tensor of K_x x K_y x K_z x N_dir entries.  The fibre of box v holds
the aggregated pattern of the group living in that box; boxes without basis
functions hold zero.  The disaggregation of eq. (5) reads the incoming spectra of
the receiving group's box.

Readings (silent in the paper):
* Polarisation outermost, then the box multi-index in row-major order, then the
  direction, then (for several right-hand sides) the right-hand side:
  [2][K_x][K_y][K_z][N_dir](R).  The linear box index is (v_x K_y + v_y) K_z + v_z,
  which for a cubic grid is the grouping's (ix K + iy) K + iz.
* Entries of the incoming spectra at empty boxes play no part in eq. (5).
"""
import numpy as np

from . import products


def box_multi_index(box_of_group, dims):
    """Linear box indices -> [G, 3] multi-indices (v_x, v_y, v_z) for a K_x x K_y x K_z grid."""
    kx, ky, kz = dims
    b = np.asarray(box_of_group, dtype=np.int64)
    return np.stack([b // (ky * kz), (b // kz) % ky, b % kz], axis=1)


def scatter(f_groups, box_of_group, dims):
    """Group-compact spectra [G, 2, N_dir(, R)] -> box-grid spectra
    [2, K_x, K_y, K_z, N_dir(, R)], zero on boxes holding no group (eq. (3))."""
    f_groups = np.asarray(f_groups)
    out = np.zeros((2,) + tuple(dims) + f_groups.shape[2:], dtype=np.complex128)
    for g, (vx, vy, vz) in enumerate(box_multi_index(box_of_group, dims)):
        for alpha in range(2):
            out[alpha, vx, vy, vz] = f_groups[g, alpha]
    return out


def gather(g_grid, box_of_group, dims):
    """Box-grid spectra [2, K_x, K_y, K_z, N_dir(, R)] -> the fibres of the groups'
    boxes, [G, 2, N_dir(, R)] (the input of eq. (5) for every group)."""
    g_grid = np.asarray(g_grid)
    idx = box_multi_index(box_of_group, dims)
    return np.stack([np.stack([g_grid[alpha, vx, vy, vz] for alpha in range(2)]) for vx, vy, vz in idx])


def aggregate_grid(kind, data, offsets, x, box_of_group, dims):
    """Aggregation of every group written onto the box grid (eq. (3))."""
    return scatter(products.aggregate_all(kind, data, offsets, x), box_of_group, dims)


def disaggregate_grid(kind, data, offsets, g_grid, box_of_group, dims):
    """Disaggregation (eq. (5)) of every group from the incoming spectra on the box grid."""
    return products.disaggregate_all(kind, data, offsets, gather(g_grid, box_of_group, dims))
