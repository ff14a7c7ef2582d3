"""The allocation-free pass, fmm_tucker_pass_noalloc, through the C ABI.

(This module's name makes pytest collect it last.)

It runs fmm_tucker_pass on the streaming kernels with the split items' partial sums
in a static device array.  The layout below has six (group, polarisation) items, far
fewer than 128, whose U^beta and core streams exceed the split size, so the items
run as row blocks whose partial sums go through that array.  Checked against the
allocating fmm_tucker_pass on the same inputs (same kernels, same block-order sums:
bit for bit) and against the oracle (FP64 1e-11, FP32 1e-5), on two calls in a row,
the second with fewer right-hand sides; then the host-side refusals (too many
right-hand sides for the array, a bf16 split precision) with buffers sized for the
call, so nothing is launched on a refused call.
"""
import numpy as np
import pytest

import synth
from oracle import products as pr
from gpu_util import dev, host, arena, max_rel, l2_rel, banner

pytestmark = pytest.mark.gpu

T = pytest.importorskip("paper_2103_05822_amd")

TOL = {T.FMM_C128: 1e-11, T.FMM_C64: 1e-5}
CDT = {T.FMM_C128: np.complex128, T.FMM_C64: np.complex64}


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)


def _noalloc(h, prec, nrhs, x, F, G, V):
    """Status of fmm_tucker_pass_noalloc through the binding (0 = FMM_OK)."""
    try:
        T.fmm_tucker_pass_noalloc(h, prec, nrhs, x, F, G, V)
    except T.FmmError as e:
        return e.status
    return 0


def _layout_and_factors(seed):
    lay = T.Layout(6, 11, np.array([0, 900, 1700, 1703]))
    rng = synth.rng(seed)
    tuck = []
    for g in range(lay.n_groups):
        nb = int(lay.offsets[g + 1] - lay.offsets[g])
        pair = []
        for _ in range(2):
            rb = min(nb, int(rng.integers(300, 420)))
            core, ut, up, ub = synth.synthetic_tucker(rng, 6, 11, nb, 5, 8, rb)
            pair.append((core, (ut, up, ub)))
        tuck.append(pair)
    return lay, tuck


@pytest.mark.parametrize("prec", [T.FMM_C128, T.FMM_C64], ids=["c128", "c64"])
def test_noalloc_pass_matches_allocating_pass(prec):
    import torch
    lay, tuck = _layout_and_factors(17)
    h = T.fmm_tucker_create(lay)
    try:
        for g, pair in enumerate(tuck):
            for a, (core, (ut, up, ub)) in enumerate(pair):
                T.fmm_tucker_set_group(h, g, a, core, ut, up, ub)
        _, nbytes = T.fmm_tucker_storage_bytes(h, prec)
        ar = arena(nbytes)
        T.fmm_tucker_upload(h, prec, ar)
        cd = CDT[prec]
        for nrhs in (3, 1):            # the second call is smaller
            banner("noalloc prec=%d nrhs=%d" % (prec, nrhs))
            rng = synth.rng(100 + nrhs)
            x = synth.complex_normal(rng, (lay.n_basis, nrhs))
            gin = synth.complex_normal(rng, (lay.n_groups, 2, lay.n_dir, nrhs))
            xd, gd = dev(x, cd), dev(gin, cd)
            F = dev(np.full(gin.shape, np.nan, cd))
            V = dev(np.full(x.shape, np.nan, cd))
            assert _noalloc(h, prec, nrhs, xd, F, gd, V) == 0, T.fmm_last_error()
            Fn, Vn = host(F), host(V)
            F2 = dev(np.zeros(gin.shape, cd))
            V2 = dev(np.zeros(x.shape, cd))
            T.fmm_tucker_pass(h, prec, nrhs, xd, F2, gd, V2)
            assert np.array_equal(Fn, host(F2)) and np.array_equal(Vn, host(V2))
            f_ref = pr.aggregate_all("tucker", tuck, lay.offsets, x)
            v_ref = pr.disaggregate_all("tucker", tuck, lay.offsets, gin)
            errs = (l2_rel(Fn, f_ref), max_rel(Fn, f_ref), l2_rel(Vn, v_ref), max_rel(Vn, v_ref))
            print("  errors vs oracle: F l2 %.2e max %.2e | V l2 %.2e max %.2e" % errs, flush=True)
            assert max(errs) < TOL[prec], errs
        # refusals on the host: too many right-hand sides for the static array (the
        # buffers are still sized for the call), and a bf16 split precision
        nrhs = 1000
        banner("noalloc refusal prec=%d nrhs=%d" % (prec, nrhs))
        xd = torch.zeros((lay.n_basis, nrhs), dtype=xd.dtype, device="cuda")
        gd = torch.zeros((lay.n_groups, 2, lay.n_dir, nrhs), dtype=xd.dtype, device="cuda")
        F = torch.zeros_like(gd)
        V = torch.zeros_like(xd)
        assert _noalloc(h, prec, nrhs, xd, F, gd, V) == -3
        assert "static scratch" in T.fmm_last_error()
        torch.cuda.synchronize()
    finally:
        T.fmm_tucker_destroy(h)


def test_noalloc_refuses_split_precisions():
    import torch
    lay, tuck = _layout_and_factors(18)
    h = T.fmm_tucker_create(lay)
    try:
        for g, pair in enumerate(tuck):
            for a, (core, (ut, up, ub)) in enumerate(pair):
                T.fmm_tucker_set_group(h, g, a, core, ut, up, ub)
        _, nbytes = T.fmm_tucker_storage_bytes(h, T.FMM_BF16X3)
        ar = arena(nbytes)
        T.fmm_tucker_upload(h, T.FMM_BF16X3, ar)
        x = torch.zeros((lay.n_basis, 2), dtype=torch.complex64, device="cuda")
        G = torch.zeros((lay.n_groups, 2, lay.n_dir, 2), dtype=torch.complex64, device="cuda")
        assert _noalloc(h, T.FMM_BF16X3, 2, x, torch.zeros_like(G), G, torch.zeros_like(x)) == -6
        assert _noalloc(None, T.FMM_C64, 2, x, torch.zeros_like(G), G, torch.zeros_like(x)) == -1
    finally:
        T.fmm_tucker_destroy(h)
