"""GPU parity of the plane-wave excitation vectors (eq. (2)) against the oracle.

The library evaluates the same 3-point rule in FP64 with the phase split at the box
centre, exp(-j k k.r) = exp(-j k k.r_v) exp(-j k k.(r - r_v)); the oracle uses the
absolute position.  Both are FP64 sums of six terms, so they agree to a few units of
rounding of the phase k k.r (|k r| up to ~30 rad here): bound 1e-12 relative to the
largest entry.  The complex64 output is the FP64 value rounded per part: bound 1e-7.
"""
import numpy as np
import pytest

import synth
from synth import workloads as W
from oracle import geometry as geo
from oracle import excitation as ex
from gpu_util import host, max_rel, banner

pytestmark = pytest.mark.gpu

T = pytest.importorskip("paper_2103_05822_amd")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)


@pytest.mark.parametrize("w", [W.SMALL, W.TRIHEDRAL_SMALL, W.SPHERE6], ids=lambda w: w.name)
@pytest.mark.parametrize("nrhs", [1, 3, 64])
def test_planewave_excitation_matches_oracle(w, nrhs):
    import torch
    v, t = w.mesh()
    P = geo.Problem(v, t, w.origin, w.box, w.boxes_per_axis, w.n_theta, w.n_phi)
    khat, epol = synth.planewaves(synth.rng(2 + nrhs), nrhs)
    ref = ex.planewave_excitation(P, khat, epol)
    geom = T.fmm_geometry_build(v, t, w.origin, w.box, w.boxes_per_axis, w.k, w.n_theta, w.n_phi)
    try:
        for prec, dt, tol in ((T.FMM_C128, torch.complex128, 1e-12), (T.FMM_C64, torch.complex64, 1e-7)):
            banner("planewave %s nrhs=%d prec=%d" % (w.name, nrhs, prec))
            x = torch.full((P.n_basis, nrhs), float("nan"), dtype=dt, device="cuda")
            T.fmm_planewave_excitation(geom, khat, epol, prec, x)
            got = host(x)
            err = max_rel(got, ref)
            print("  max rel err %.2e" % err, flush=True)
            assert np.all(np.isfinite(got)) and err < tol, err
    finally:
        T.fmm_geometry_destroy(geom)


def test_planewave_argument_errors():
    import torch
    w = W.SMALL
    v, t = w.mesh()
    geom = T.fmm_geometry_build(v, t, w.origin, w.box, w.boxes_per_axis, w.k, w.n_theta, w.n_phi)
    try:
        n, _ = T.fmm_geometry_info(geom)
        x = torch.zeros((n, 2), dtype=torch.complex64, device="cuda")
        k = np.array([[0.0, 0.0, 1.0], [0.0, 0.0, 2.0]])      # second direction not a unit vector
        e = np.array([[1.0, 0.0, 0.0], [1.0, 0.0, 0.0]])
        with pytest.raises(T.FmmError) as err:
            T.fmm_planewave_excitation(geom, k, e, T.FMM_C64, x)
        assert err.value.status == -1
        k[1, 2] = np.nan
        with pytest.raises(T.FmmError) as err:
            T.fmm_planewave_excitation(geom, k, e, T.FMM_C64, x)
        assert err.value.status == -5
    finally:
        T.fmm_geometry_destroy(geom)
