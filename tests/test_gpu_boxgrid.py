"""GPU parity of the box-grid spectra (eq. (3), eq. (5)): the Tucker aggregation
writes each group's fibre into its box of a K_x x K_y x K_z x N_dir tensor per
polarisation and zero on the empty boxes; the disaggregation reads the groups' boxes
only.  Outputs start as NaN so that an entry the kernels skip shows up, and the
incoming spectra hold NaN on the empty boxes so that a read of one shows up.

Tolerances as in the other parity tests: FP64 1e-11, FP32 and BF16x3 1e-5 (the
single-precision target), BF16x2 3e-5 (L2) / 1e-4 (max), its own bound below that
target, relative to the oracle.
"""
import numpy as np
import pytest

import synth
from synth import workloads as W
from oracle import boxgrid as bg
from oracle import geometry as geo
from gpu_util import dev, host, arena, max_rel, l2_rel, banner

pytestmark = pytest.mark.gpu

T = pytest.importorskip("paper_2103_05822_amd")

CDT = {T.FMM_C128: np.complex128, T.FMM_C64: np.complex64, T.FMM_BF16X2: np.complex64,
       T.FMM_BF16X3: np.complex64}
TOL = {T.FMM_C128: (1e-11, 1e-11), T.FMM_C64: (1e-5, 1e-5), T.FMM_BF16X2: (3e-5, 1e-4),
       T.FMM_BF16X3: (1e-5, 1e-5)}
DIMS = (3, 4, 5)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)


def ragged():
    sizes = [1, 2, 3, 64, 65, 130, 257]
    lay = T.Layout(5, 9, np.concatenate([[0], np.cumsum(sizes)]))
    rng = synth.rng(90)
    tuck = []
    for g in range(lay.n_groups):
        nb = sizes[g]
        pair = []
        for a in range(2):
            if g == 2:   # one group in truncated-SVD form
                rb = int(rng.integers(1, nb + 1))
                w = synth.complex_normal(rng, (lay.n_dir, rb))
                ub = synth.complex_normal(rng, (nb, rb)) / np.sqrt(nb)
                pair.append((w.reshape(5, 9, rb), (np.eye(5, dtype=complex), np.eye(9, dtype=complex), ub)))
                continue
            rt, rp, rb = synth.synthetic_ranks(rng, nb, 5, 9)
            core, ut, up, ub = synth.synthetic_tucker(rng, 5, 9, nb, rt, rp, rb)
            pair.append((core, (ut, up, ub)))
        tuck.append(pair)
    boxes = rng.choice(int(np.prod(DIMS)), size=lay.n_groups, replace=False)
    return lay, tuck, boxes


def grid_inputs(lay, boxes, nrhs, seed):
    rng = synth.rng(seed)
    shp = (nrhs,) if nrhs > 1 else ()
    x = synth.complex_normal(rng, (lay.n_basis,) + shp)
    gg = synth.complex_normal(rng, (2,) + DIMS + (lay.n_dir,) + shp)
    g_nan = gg.copy()
    used = set(int(b) for b in boxes)
    for b in range(int(np.prod(DIMS))):
        if b not in used:
            v = np.unravel_index(b, DIMS)
            g_nan[:, v[0], v[1], v[2]] = np.nan
    return x, gg, g_nan


class Handle:
    def __init__(self, lay, tuck, prec, boxes):
        self.h = T.fmm_tucker_create(lay)
        for g, pair in enumerate(tuck):
            for a, (core, (ut, up, ub)) in enumerate(pair):
                T.fmm_tucker_set_group(self.h, g, a, core, ut, up, ub)
        T.fmm_tucker_set_box_grid(self.h, DIMS, boxes)
        _, nbytes = T.fmm_tucker_storage_bytes(self.h, prec)
        self.arena = arena(nbytes)
        T.fmm_tucker_upload(self.h, prec, self.arena)

    def close(self):
        T.fmm_tucker_destroy(self.h)


def nan_buffer(shape, prec):
    return dev(np.full(shape, np.nan + 1j * np.nan), CDT[prec])


def check(prec, got, ref):
    tl2, tmax = TOL[prec]
    assert np.all(np.isfinite(got))
    e = (l2_rel(got, ref), max_rel(got, ref))
    print("  errors: l2 %.2e max %.2e" % e, flush=True)
    assert e[0] < tl2 and e[1] < tmax, e


@pytest.mark.parametrize("prec,nrhs", [(T.FMM_C128, 1), (T.FMM_C64, 1), (T.FMM_C128, 3), (T.FMM_C64, 3),
                                       (T.FMM_C64, 8), (T.FMM_BF16X2, 8), (T.FMM_BF16X3, 66)],
                         ids=["c128-1", "c64-1", "c128-3", "c64-3", "c64-8", "bf16x2-8", "bf16x3-66"])
def test_box_grid_stages(prec, nrhs):
    """Separate aggregation and disaggregation on a 3 x 4 x 5 grid (streaming kernels
    for nrhs 1 and 3, matrix-core products for 8 and 66)."""
    lay, tuck, boxes = ragged()
    banner("box grid stages prec=%d nrhs=%d" % (prec, nrhs))
    x, gg, g_nan = grid_inputs(lay, boxes, nrhs, 91)
    f_ref = bg.aggregate_grid("tucker", tuck, lay.offsets, x, boxes, DIMS)
    v_ref = bg.disaggregate_grid("tucker", tuck, lay.offsets, gg, boxes, DIMS)
    H = Handle(lay, tuck, prec, boxes)
    try:
        F = nan_buffer(f_ref.shape, prec)
        V = nan_buffer(v_ref.shape, prec)
        T.fmm_tucker_aggregate(H.h, prec, nrhs, dev(x, CDT[prec]), F)
        T.fmm_tucker_disaggregate(H.h, prec, nrhs, dev(g_nan, CDT[prec]), V)
        F, V = host(F), host(V)
    finally:
        H.close()
    empty = np.abs(f_ref).sum(axis=tuple(range(4, f_ref.ndim))) == 0
    assert np.all(F[np.broadcast_to(empty[(...,) + (None,) * (f_ref.ndim - 4)], F.shape)] == 0)
    check(prec, F, f_ref)
    check(prec, V, v_ref)


@pytest.mark.parametrize("prec,nrhs", [(T.FMM_C64, 1), (T.FMM_C64, 8), (T.FMM_BF16X2, 8)],
                         ids=["c64-1", "c64-8", "bf16x2-8"])
def test_box_grid_pass_and_graph(prec, nrhs):
    """The merged pass and its graph replays on the box grid equal the separate
    stages bit for bit."""
    import torch
    lay, tuck, boxes = ragged()
    banner("box grid pass+graph prec=%d nrhs=%d" % (prec, nrhs))
    x, gg, g_nan = grid_inputs(lay, boxes, nrhs, 92)
    f_ref = bg.aggregate_grid("tucker", tuck, lay.offsets, x, boxes, DIMS)
    v_ref = bg.disaggregate_grid("tucker", tuck, lay.offsets, gg, boxes, DIMS)
    H = Handle(lay, tuck, prec, boxes)
    try:
        xd, gd = dev(x, CDT[prec]), dev(g_nan, CDT[prec])
        F1, V1 = nan_buffer(f_ref.shape, prec), nan_buffer(v_ref.shape, prec)
        T.fmm_tucker_aggregate(H.h, prec, nrhs, xd, F1)
        T.fmm_tucker_disaggregate(H.h, prec, nrhs, gd, V1)
        F1, V1 = host(F1), host(V1)
        check(prec, F1, f_ref)
        check(prec, V1, v_ref)
        F, V = nan_buffer(f_ref.shape, prec), nan_buffer(v_ref.shape, prec)
        T.fmm_tucker_pass(H.h, prec, nrhs, xd, F, gd, V)
        assert np.array_equal(host(F), F1) and np.array_equal(host(V), V1)
        s = torch.cuda.Stream()
        F.fill_(float("nan"))
        with torch.cuda.stream(s):
            T.fmm_graph_capture(H.h, prec, nrhs, xd, F, gd, V, s)
        torch.cuda.synchronize()
        for _ in range(3):
            F.fill_(float("nan"))
            V.fill_(float("nan"))
            torch.cuda.synchronize()
            T.fmm_graph_launch(H.h, s)
            s.synchronize()
            assert np.array_equal(host(F), F1) and np.array_equal(host(V), V1)
    finally:
        H.close()


def test_box_grid_on_the_mesh_and_back():
    """Small sphere: compressed far-fields, the geometry's own box grid; then the grid
    is cleared and the group-compact results are the grid's fibres."""
    w = W.SMALL
    v, t = synth.icosphere(w.freq, w.radius)
    P = geo.Problem(v, t, w.origin, w.box, w.boxes_per_axis, w.n_theta, w.n_phi)
    lay = T.Layout(w.n_theta, w.n_phi, P.offsets)
    g = T.fmm_geometry_build(v, t, w.origin, w.box, w.boxes_per_axis, w.k, w.n_theta, w.n_phi)
    h = None
    try:
        banner("box grid small mesh")
        K, boxes = T.fmm_geometry_boxes(g)
        dims = (K, K, K)
        D = dev(np.zeros((P.n_basis, 2, w.n_theta, w.n_phi), np.complex128))
        T.fmm_farfield_fill(g, 0, P.n_groups, D)
        h = T.fmm_farfield_compress(lay, D, 0, P.n_groups, 1e-6)
        ranks = T.fmm_tucker_ranks(h, P.n_groups)
        tuck = []
        for gg_ in range(P.n_groups):
            nb = int(P.offsets[gg_ + 1] - P.offsets[gg_])
            pair = []
            for a in range(2):
                c, ut, up, ub = T.fmm_tucker_export(h, gg_, a, ranks[gg_, a], w.n_theta, w.n_phi, nb)
                pair.append((c, (ut, up, ub)))
            tuck.append(pair)
        x = synth.complex_normal(synth.rng(93), P.n_basis)
        T.fmm_tucker_set_box_grid(h, dims, boxes)
        _, nbytes = T.fmm_tucker_storage_bytes(h, T.FMM_C128)
        ar = arena(nbytes)
        T.fmm_tucker_upload(h, T.FMM_C128, ar)
        Fg = nan_buffer((2,) + dims + (P.n_dir,), T.FMM_C128)
        T.fmm_tucker_aggregate(h, T.FMM_C128, 1, dev(x), Fg)
        Fg = host(Fg)
        T.fmm_tucker_set_box_grid(h, None, None)
        T.fmm_tucker_upload(h, T.FMM_C128, ar)
        Fc = nan_buffer((P.n_groups, 2, P.n_dir), T.FMM_C128)
        T.fmm_tucker_aggregate(h, T.FMM_C128, 1, dev(x), Fc)
        Fc = host(Fc)
    finally:
        if h:
            T.fmm_tucker_destroy(h)
        T.fmm_geometry_destroy(g)
    ref = bg.aggregate_grid("tucker", tuck, P.offsets, x, boxes, dims)
    check(T.FMM_C128, Fg, ref)
    assert np.array_equal(bg.gather(Fg, boxes, dims), Fc)
    assert np.count_nonzero(np.abs(Fg).sum(axis=(0, 4))) == P.n_groups
