"""GPU parity: the HIP kernels against the FP64 oracle on the same seeded inputs.

Tolerances (relative to the largest reference entry, and relative L2 over all
outputs): FP64 paths 1e-11; FP32 paths 1e-5, the bound the method's target sets
for single precision (sums of up to ~2,000 FP32 terms with unit-roundoff 6e-8 stay
near 1e-6).
"""
import numpy as np
import pytest

import synth
from synth import workloads as W
from oracle import geometry as geo
from oracle import farfield as ff
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


# ---------------------------------------------------------------------------- helpers

def ragged_layout(n_theta=5, n_phi=9):
    """Groups of 1, 2, 3, 64, 65, 130, 257 basis functions (tails of every tile size)."""
    sizes = [1, 2, 3, 64, 65, 130, 257]
    return T.Layout(n_theta, n_phi, np.concatenate([[0], np.cumsum(sizes)]))


def small_problem(w=W.SMALL):
    v, t = w.mesh()
    return w, v, t, geo.Problem(v, t, w.origin, w.box, w.boxes_per_axis, w.n_theta, w.n_phi)


def random_tucker(lay, seed, rank_mode="random"):
    """Per (group, polarisation) synthetic factors; rank_mode picks edge cases."""
    rng = synth.rng(seed)
    out = []
    for g in range(lay.n_groups):
        nb = int(lay.offsets[g + 1] - lay.offsets[g])
        pair = []
        for a in range(2):
            if rank_mode == "full":
                rt, rp, rb = lay.n_theta, lay.n_phi, nb
            elif rank_mode == "one":
                rt, rp, rb = 1, 1, 1
            else:
                rt, rp, rb = synth.synthetic_ranks(rng, nb, lay.n_theta, lay.n_phi)
            core, ut, up, ub = synth.synthetic_tucker(rng, lay.n_theta, lay.n_phi, nb, rt, rp, rb)
            pair.append((core, (ut, up, ub)))
        out.append(pair)
    return out


def make_handle(lay, tuck):
    h = T.fmm_tucker_create(lay)
    for g, pair in enumerate(tuck):
        for a, (core, (ut, up, ub)) in enumerate(pair):
            T.fmm_tucker_set_group(h, g, a, core, ut, up, ub)
    return h


def run_tucker(lay, tuck, prec, x, gin, nrhs):
    h = make_handle(lay, tuck)
    try:
        _, nbytes = T.fmm_tucker_storage_bytes(h, prec)
        ar = arena(nbytes)
        T.fmm_tucker_upload(h, prec, ar)
        xd = dev(x, CDT[prec])
        gd = dev(gin, CDT[prec])
        F = dev(np.zeros((lay.n_groups, 2, lay.n_dir) + ((nrhs,) if nrhs > 1 else ()), CDT[prec]))
        V = dev(np.zeros(x.shape, CDT[prec]))
        T.fmm_tucker_aggregate(h, prec, nrhs, xd, F)
        T.fmm_tucker_disaggregate(h, prec, nrhs, gd, V)
        return host(F), host(V)
    finally:
        T.fmm_tucker_destroy(h)


def oracle_tucker(lay, tuck, x, gin):
    f = pr.aggregate_all("tucker", tuck, lay.offsets, x)
    v = pr.disaggregate_all("tucker", tuck, lay.offsets, gin)
    return f, v


# ------------------------------------------------------------------------------ Tucker

@pytest.mark.parametrize("prec", [T.FMM_C128, T.FMM_C64], ids=["c128", "c64"])
@pytest.mark.parametrize("rank_mode", ["random", "full", "one"])
@pytest.mark.parametrize("nrhs", [1, 3])
def test_tucker_ragged_layout(prec, rank_mode, nrhs):
    lay = ragged_layout()
    banner("tucker ragged prec=%d ranks=%s nrhs=%d" % (prec, rank_mode, nrhs))
    tuck = random_tucker(lay, 20 + nrhs, rank_mode)
    rng = synth.rng(5)
    shp = (nrhs,) if nrhs > 1 else ()
    x = synth.complex_normal(rng, (lay.n_basis,) + shp)
    gin = synth.complex_normal(rng, (lay.n_groups, 2, lay.n_dir) + shp)
    F, V = run_tucker(lay, tuck, prec, x, gin, nrhs)
    f_ref, v_ref = oracle_tucker(lay, tuck, x, gin)
    tol = TOL[prec]
    assert max_rel(F, f_ref) < tol and l2_rel(F, f_ref) < tol
    assert max_rel(V, v_ref) < tol and l2_rel(V, v_ref) < tol


@pytest.mark.parametrize("prec", [T.FMM_C128, T.FMM_C64], ids=["c128", "c64"])
def test_tucker_paper_grid_realistic_ranks(prec):
    """38 x 75 grid, group sizes of the 6-lambda sphere at box 2 lambda, ranks near
    Table IV's 2-lambda row (several column tiles, ragged tails)."""
    w = W.SPHERE6
    v, t = synth.icosphere(w.freq, w.radius)
    P = geo.Problem(v, t, w.origin, w.box, w.boxes_per_axis, w.n_theta, w.n_phi)
    lay = T.Layout(w.n_theta, w.n_phi, P.offsets)
    rng = synth.rng(31)
    tuck = []
    for g in range(lay.n_groups):
        nb = int(lay.offsets[g + 1] - lay.offsets[g])
        pair = []
        for a in range(2):
            rt = int(rng.integers(20, 29))
            rp = int(rng.integers(24, 34))
            rb = int(min(nb, rng.integers(150, 260)))
            core, ut, up, ub = synth.synthetic_tucker(rng, w.n_theta, w.n_phi, nb, rt, rp, rb)
            pair.append((core, (ut, up, ub)))
        tuck.append(pair)
    banner("tucker paper grid prec=%d groups=%d N=%d" % (prec, lay.n_groups, lay.n_basis))
    x = synth.complex_normal(rng, lay.n_basis)
    gin = synth.complex_normal(rng, (lay.n_groups, 2, lay.n_dir))
    F, V = run_tucker(lay, tuck, prec, x, gin, 1)
    f_ref, v_ref = oracle_tucker(lay, tuck, x, gin)
    tol = TOL[prec]
    assert max_rel(F, f_ref) < tol and l2_rel(F, f_ref) < tol
    assert max_rel(V, v_ref) < tol and l2_rel(V, v_ref) < tol


@pytest.mark.parametrize("prec", [T.FMM_C128, T.FMM_C64], ids=["c128", "c64"])
@pytest.mark.parametrize("nrhs", [1, 3])
def test_tucker_pass_equals_separate_stages(prec, nrhs):
    """The one-launch pass computes exactly what the two stage calls compute."""
    import torch
    lay = ragged_layout(6, 11)
    tuck = random_tucker(lay, 50 + nrhs)
    rng = synth.rng(8)
    shp = (nrhs,) if nrhs > 1 else ()
    x = synth.complex_normal(rng, (lay.n_basis,) + shp)
    gin = synth.complex_normal(rng, (lay.n_groups, 2, lay.n_dir) + shp)
    h = make_handle(lay, tuck)
    try:
        _, nbytes = T.fmm_tucker_storage_bytes(h, prec)
        ar = arena(nbytes)
        T.fmm_tucker_upload(h, prec, ar)
        xd, gd = dev(x, CDT[prec]), dev(gin, CDT[prec])
        F1, F2 = dev(np.zeros(gin.shape, CDT[prec])), dev(np.zeros(gin.shape, CDT[prec]))
        V1, V2 = dev(np.full(x.shape, 7.0, CDT[prec])), dev(np.full(x.shape, 7.0, CDT[prec]))
        banner("tucker pass vs stages prec=%d nrhs=%d" % (prec, nrhs))
        T.fmm_tucker_aggregate(h, prec, nrhs, xd, F1)
        T.fmm_tucker_disaggregate(h, prec, nrhs, gd, V1)
        T.fmm_tucker_pass(h, prec, nrhs, xd, F2, gd, V2)
        assert np.array_equal(host(F1), host(F2))
        assert np.array_equal(host(V1), host(V2))
        f_ref, v_ref = oracle_tucker(lay, tuck, x, gin)
        assert l2_rel(host(F2), f_ref) < TOL[prec] and l2_rel(host(V2), v_ref) < TOL[prec]
    finally:
        T.fmm_tucker_destroy(h)


def test_tucker_deterministic_and_graph_replays():
    import torch
    lay = ragged_layout(6, 11)
    tuck = random_tucker(lay, 41)
    rng = synth.rng(6)
    x = synth.complex_normal(rng, lay.n_basis)
    gin = synth.complex_normal(rng, (lay.n_groups, 2, lay.n_dir))
    h = make_handle(lay, tuck)
    try:
        prec = T.FMM_C64
        _, nbytes = T.fmm_tucker_storage_bytes(h, prec)
        ar = arena(nbytes)
        T.fmm_tucker_upload(h, prec, ar)
        xd, gd = dev(x, np.complex64), dev(gin, np.complex64)
        F = torch.zeros((lay.n_groups, 2, lay.n_dir), dtype=torch.complex64, device="cuda")
        V = torch.zeros(lay.n_basis, dtype=torch.complex64, device="cuda")
        banner("tucker eager x2")
        T.fmm_tucker_aggregate(h, prec, 1, xd, F)
        T.fmm_tucker_disaggregate(h, prec, 1, gd, V)
        F0, V0 = host(F).copy(), host(V).copy()
        T.fmm_tucker_aggregate(h, prec, 1, xd, F)
        T.fmm_tucker_disaggregate(h, prec, 1, gd, V)
        assert np.array_equal(host(F), F0) and np.array_equal(host(V), V0)
        banner("tucker graph capture + 3 replays")
        s = torch.cuda.Stream()
        with torch.cuda.stream(s):
            T.fmm_graph_capture(h, prec, 1, xd, F, gd, V, s)
        for rep in range(3):
            F.zero_()
            V.zero_()
            torch.cuda.synchronize()
            T.fmm_graph_launch(h, s)
            s.synchronize()
            assert np.array_equal(host(F), F0), rep
            assert np.array_equal(host(V), V0), rep
    finally:
        T.fmm_tucker_destroy(h)


# ------------------------------------------------------------------------------- dense

@pytest.mark.parametrize("prec", [T.FMM_C128, T.FMM_C64], ids=["c128", "c64"])
@pytest.mark.parametrize("nrhs", [1, 2, 3, 5, 8, 9, 66])
def test_dense_ragged_layout(prec, nrhs):
    """Dense products against the oracle: right-hand sides in blocks of 1, 2, 4 and 8
    per read of A, ragged blocks (3 = one block of 4 with 3 valid, 5 = one block of 8
    with 5 valid, 9 = a block of 8 and one with 1 valid, 66 = 8 blocks of 8 and one
    with 2 valid).  The disaggregation with 2 or more runs on row blocks of up to 16
    rows of one group: the groups of 1-3 rows leave wavefronts without rows, 65 and
    257 leave a one-row block."""
    lay = ragged_layout(7, 13)
    banner("dense ragged prec=%d nrhs=%d" % (prec, nrhs))
    rng = synth.rng(9)
    A = synth.complex_normal(rng, (lay.n_basis, 2, lay.n_theta, lay.n_phi))
    shp = (nrhs,) if nrhs > 1 else ()
    x = synth.complex_normal(rng, (lay.n_basis,) + shp)
    gin = synth.complex_normal(rng, (lay.n_groups, 2, lay.n_dir) + shp)
    d = T.fmm_dense_create(lay)
    try:
        Ad = dev(A, CDT[prec])
        F = dev(np.zeros(gin.shape, CDT[prec]))
        V = dev(np.zeros(x.shape, CDT[prec]))
        T.fmm_dense_aggregate(d, prec, Ad, nrhs, dev(x, CDT[prec]), F)
        T.fmm_dense_disaggregate(d, prec, Ad, nrhs, dev(gin, CDT[prec]), V)
        F, V = host(F), host(V)
    finally:
        T.fmm_dense_destroy(d)
    f_ref = pr.aggregate_all("dense", A, lay.offsets, x)
    v_ref = pr.disaggregate_all("dense", A, lay.offsets, gin)
    tol = TOL[prec]
    assert max_rel(F, f_ref) < tol and l2_rel(F, f_ref) < tol
    assert max_rel(V, v_ref) < tol and l2_rel(V, v_ref) < tol


# -------------------------------------------------------------------- far-field + compress

@pytest.mark.parametrize("w", [W.SMALL, W.TRIHEDRAL_SMALL], ids=["sphere", "trihedral"])
def test_farfield_fill_matches_oracle(w):
    w, v, t, P = small_problem(w)
    D_ref = ff.farfield_all(P)
    g = T.fmm_geometry_build(v, t, w.origin, w.box, w.boxes_per_axis, w.k, w.n_theta, w.n_phi)
    try:
        banner("farfield fill %s" % w.name)
        D = dev(np.zeros(D_ref.shape, np.complex128))
        T.fmm_farfield_fill(g, 0, P.n_groups, D)
        D = host(D)
        # a chunk of groups lands at the chunk's first row
        D2 = dev(np.zeros((int(P.offsets[5] - P.offsets[3]), 2, w.n_theta, w.n_phi), np.complex128))
        T.fmm_farfield_fill(g, 3, 2, D2)
        D2 = host(D2)
    finally:
        T.fmm_geometry_destroy(g)
    assert max_rel(D, D_ref) < 1e-13
    assert np.array_equal(D2, D[P.offsets[3]:P.offsets[5]])


@pytest.mark.parametrize("w", [W.SMALL, W.TRIHEDRAL_SMALL], ids=["sphere", "trihedral"])
@pytest.mark.parametrize("gamma", [1e-6, 1e-4, 0.0])
def test_compress_end_to_end(gamma, w):
    """GPU far-field -> GPU HOSVD -> GPU Tucker products against the oracle's dense
    products with its own far-field: the difference is the compression error,
    bounded by gamma ||A||_F ||x|| per tensor (plus rounding).  Closed (sphere) and
    open (trihedral plates) surfaces."""
    w, v, t, P = small_problem(w)
    D_ref = ff.farfield_all(P)
    lay = T.Layout(w.n_theta, w.n_phi, P.offsets)
    g = T.fmm_geometry_build(v, t, w.origin, w.box, w.boxes_per_axis, w.k, w.n_theta, w.n_phi)
    h = None
    try:
        banner("compress %s gamma=%g" % (w.name, gamma))
        D = dev(np.zeros(D_ref.shape, np.complex128))
        T.fmm_farfield_fill(g, 0, P.n_groups, D)
        h = T.fmm_farfield_compress(lay, D, 0, P.n_groups, gamma)
        ranks = T.fmm_tucker_ranks(h, P.n_groups)
        rng = synth.rng(w.seeds["x"])
        x = synth.complex_normal(rng, P.n_basis)
        _, nbytes = T.fmm_tucker_storage_bytes(h, T.FMM_C128)
        ar = arena(nbytes)
        T.fmm_tucker_upload(h, T.FMM_C128, ar)
        F = dev(np.zeros((P.n_groups, 2, P.n_dir), np.complex128))
        T.fmm_tucker_aggregate(h, T.FMM_C128, 1, dev(x), F)
        F = host(F)
        facs = [[T.fmm_tucker_export(h, gg, a, ranks[gg, a], w.n_theta, w.n_phi,
                                     int(P.offsets[gg + 1] - P.offsets[gg])) for a in range(2)]
                for gg in range(P.n_groups)]
    finally:
        if h:
            T.fmm_tucker_destroy(h)
        T.fmm_geometry_destroy(g)
    from oracle import hosvd as H
    for gg in range(P.n_groups):
        blk = D_ref[P.offsets[gg]:P.offsets[gg + 1]]
        xs = x[P.offsets[gg]:P.offsets[gg + 1]]
        f_dense = pr.dense_aggregate(blk, xs)
        for a in range(2):
            core, ut, up, ub = facs[gg][a]
            for u in (ut, up, ub):                     # orthonormal factors
                assert np.allclose(u.conj().T @ u, np.eye(u.shape[1]), atol=1e-12)
            bound = gamma * np.linalg.norm(blk[:, a]) * np.linalg.norm(xs)
            err = np.linalg.norm(F[gg, a] - f_dense[a])
            assert err <= bound * (1 + 1e-6) + 1e-12 * np.linalg.norm(f_dense[a]), (gg, a, err, bound)
            # ranks agree with the oracle's HOSVD up to ties at the threshold
            c_ref, _, _ = H.hosvd(H.tensorize(blk, a), gamma)
            assert np.all(np.abs(np.array(core.shape) - np.array(c_ref.shape)) <= 1), (core.shape, c_ref.shape)


@pytest.mark.parametrize("threads", [64, 128, 256, 512])
@pytest.mark.parametrize("prec", [T.FMM_C128, T.FMM_C64], ids=["c128", "c64"])
def test_tucker_workgroup_sizes(prec, threads, monkeypatch):
    """Every workgroup size of the streaming kernels (forced at upload) matches the
    oracle, for separate stages and the merged pass."""
    monkeypatch.setenv("TUCKFMM_STREAM_THREADS", str(threads))
    lay = ragged_layout(9, 17)
    banner("tucker workgroup size %d prec=%d" % (threads, prec))
    tuck = random_tucker(lay, 60 + threads)
    rng = synth.rng(11)
    x = synth.complex_normal(rng, lay.n_basis)
    gin = synth.complex_normal(rng, (lay.n_groups, 2, lay.n_dir))
    f_ref, v_ref = oracle_tucker(lay, tuck, x, gin)
    h = make_handle(lay, tuck)
    try:
        _, nbytes = T.fmm_tucker_storage_bytes(h, prec)
        ar = arena(nbytes)
        T.fmm_tucker_upload(h, prec, ar)
        xd, gd = dev(x, CDT[prec]), dev(gin, CDT[prec])
        F = dev(np.zeros(f_ref.shape, CDT[prec]))
        V = dev(np.zeros(v_ref.shape, CDT[prec]))
        T.fmm_tucker_pass(h, prec, 1, xd, F, gd, V)
        Fp, Vp = host(F), host(V)
        tol = TOL[prec]
        assert l2_rel(Fp, f_ref) < tol and l2_rel(Vp, v_ref) < tol
        T.fmm_tucker_aggregate(h, prec, 1, xd, F)
        T.fmm_tucker_disaggregate(h, prec, 1, gd, V)
        assert np.array_equal(host(F), Fp) and np.array_equal(host(V), Vp)
    finally:
        T.fmm_tucker_destroy(h)


def many_small_layout(n_groups=2500, seed=71):
    """Thousands of small groups, n_beta drawn from 1..80, on the 17 x 33 grid of the
    0.5-lambda boxes: the regime where a single item streams only a few kilobytes."""
    rng = synth.rng(seed)
    sizes = rng.integers(1, 81, size=n_groups)
    return T.Layout(17, 33, np.concatenate([[0], np.cumsum(sizes)]))


@pytest.mark.parametrize("threads", [0, 64, 128])
@pytest.mark.parametrize("prec", [T.FMM_C128, T.FMM_C64], ids=["c128", "c64"])
def test_tucker_many_small_items(prec, threads, monkeypatch):
    """5000 small items (no row-block splitting at this count) with random ranks: the
    merged pass and the separate stages against the oracle, for the workgroup size the
    layout picks (0) and forced sizes."""
    if threads:
        monkeypatch.setenv("TUCKFMM_STREAM_THREADS", str(threads))
    lay = many_small_layout()
    banner("tucker many small items prec=%d threads=%d groups=%d" % (prec, threads, lay.n_groups))
    tuck = random_tucker(lay, 72)
    rng = synth.rng(12)
    x = synth.complex_normal(rng, lay.n_basis)
    gin = synth.complex_normal(rng, (lay.n_groups, 2, lay.n_dir))
    f_ref, v_ref = oracle_tucker(lay, tuck, x, gin)
    h = make_handle(lay, tuck)
    try:
        _, nbytes = T.fmm_tucker_storage_bytes(h, prec)
        ar = arena(nbytes)
        T.fmm_tucker_upload(h, prec, ar)
        xd, gd = dev(x, CDT[prec]), dev(gin, CDT[prec])
        F = dev(np.zeros(f_ref.shape, CDT[prec]))
        V = dev(np.zeros(v_ref.shape, CDT[prec]))
        T.fmm_tucker_pass(h, prec, 1, xd, F, gd, V)
        Fp, Vp = host(F), host(V)
        tol = TOL[prec]
        res = (l2_rel(Fp, f_ref), max_rel(Fp, f_ref), l2_rel(Vp, v_ref), max_rel(Vp, v_ref))
        print("  errors: F l2 %.2e max %.2e | V l2 %.2e max %.2e" % res, flush=True)
        assert max(res) < tol, res
        T.fmm_tucker_aggregate(h, prec, 1, xd, F)
        T.fmm_tucker_disaggregate(h, prec, 1, gd, V)
        assert np.array_equal(host(F), Fp) and np.array_equal(host(V), Vp)
    finally:
        T.fmm_tucker_destroy(h)


# ------------------------------------------------------------ truncated SVD (comparison)

def random_svd(lay, seed, rank_mode="random"):
    """Per (group, polarisation) truncated-SVD factors ``(W [N_dir, r_b], U_b [nb, r_b])``."""
    rng = synth.rng(seed)
    out = []
    for g in range(lay.n_groups):
        nb = int(lay.offsets[g + 1] - lay.offsets[g])
        pair = []
        for a in range(2):
            rb = nb if rank_mode == "full" else (1 if rank_mode == "one" else int(rng.integers(1, nb + 1)))
            wmat = synth.complex_normal(rng, (lay.n_dir, rb))
            ub = synth.complex_normal(rng, (nb, rb)) / np.sqrt(nb)
            pair.append((wmat, ub))
        out.append(pair)
    return out


def svd_as_tucker(lay, svd):
    """The SVD model A = W U_b^T is the Tucker model with identity angular factors and
    core C[i, j, b] = W[i n_phi + j, b] (the direction index runs theta-major)."""
    eye_t = np.eye(lay.n_theta, dtype=np.complex128)
    eye_p = np.eye(lay.n_phi, dtype=np.complex128)
    return [[(wmat.reshape(lay.n_theta, lay.n_phi, -1), (eye_t, eye_p, ub)) for wmat, ub in pair]
            for pair in svd]


@pytest.mark.parametrize("prec", [T.FMM_C128, T.FMM_C64], ids=["c128", "c64"])
@pytest.mark.parametrize("rank_mode", ["random", "full", "one"])
@pytest.mark.parametrize("nrhs", [1, 3])
def test_svd_factors_match_oracle(prec, rank_mode, nrhs):
    """Identity angular factors select the SVD kernels' branch (no angular products);
    the result is the oracle's SVD aggregation / disaggregation, and the stored bytes
    are W and U_b only."""
    lay = ragged_layout()
    banner("svd ragged prec=%d ranks=%s nrhs=%d" % (prec, rank_mode, nrhs))
    svd = random_svd(lay, 40 + nrhs, rank_mode)
    rng = synth.rng(6)
    shp = (nrhs,) if nrhs > 1 else ()
    x = synth.complex_normal(rng, (lay.n_basis,) + shp)
    gin = synth.complex_normal(rng, (lay.n_groups, 2, lay.n_dir) + shp)
    tuck = svd_as_tucker(lay, svd)
    h = make_handle(lay, tuck)
    try:
        ranks = T.fmm_tucker_ranks(h, lay.n_groups)
        fbytes, _ = T.fmm_tucker_storage_bytes(h, prec)
    finally:
        T.fmm_tucker_destroy(h)
    from oracle import hosvd as H
    es = 16 if prec == T.FMM_C128 else 8
    want = sum(H.svd_memory(ub.shape[0], lay.n_dir, ub.shape[1], es) for pair in svd for _, ub in pair)
    assert fbytes == want
    assert np.all(ranks[:, :, 0] == lay.n_theta) and np.all(ranks[:, :, 1] == lay.n_phi)
    F, V = run_tucker(lay, tuck, prec, x, gin, nrhs)
    f_ref = pr.aggregate_all("svd", svd, lay.offsets, x)
    v_ref = pr.disaggregate_all("svd", svd, lay.offsets, gin)
    tol = TOL[prec]
    assert max_rel(F, f_ref) < tol and l2_rel(F, f_ref) < tol
    assert max_rel(V, v_ref) < tol and l2_rel(V, v_ref) < tol


@pytest.mark.parametrize("prec", [T.FMM_C128, T.FMM_C64], ids=["c128", "c64"])
def test_svd_and_tucker_groups_in_one_pass(prec):
    """Even groups in SVD form, odd groups in general Tucker form: one pass holds both
    item kinds and each matches its own oracle product."""
    lay = ragged_layout()
    banner("svd+tucker mixed prec=%d" % prec)
    svd = svd_as_tucker(lay, random_svd(lay, 51))
    gen = random_tucker(lay, 52)
    tuck = [svd[g] if g % 2 == 0 else gen[g] for g in range(lay.n_groups)]
    rng = synth.rng(7)
    x = synth.complex_normal(rng, lay.n_basis)
    gin = synth.complex_normal(rng, (lay.n_groups, 2, lay.n_dir))
    h = make_handle(lay, tuck)
    try:
        _, nbytes = T.fmm_tucker_storage_bytes(h, prec)
        ar = arena(nbytes)
        T.fmm_tucker_upload(h, prec, ar)
        F = dev(np.zeros((lay.n_groups, 2, lay.n_dir), CDT[prec]))
        V = dev(np.zeros(x.shape, CDT[prec]))
        T.fmm_tucker_pass(h, prec, 1, dev(x, CDT[prec]), F, dev(gin, CDT[prec]), V)
        F, V = host(F), host(V)
    finally:
        T.fmm_tucker_destroy(h)
    f_ref, v_ref = oracle_tucker(lay, tuck, x, gin)
    tol = TOL[prec]
    assert max_rel(F, f_ref) < tol and l2_rel(F, f_ref) < tol
    assert max_rel(V, v_ref) < tol and l2_rel(V, v_ref) < tol


@pytest.mark.parametrize("gamma", [1e-6, 1e-4, 0.0])
def test_compress_svd_end_to_end(gamma):
    """GPU far-field -> GPU truncated SVD -> GPU products against the oracle's dense
    products: the difference is bounded by gamma ||A||_F ||x|| per tensor; the basis
    rank agrees with the oracle's truncated SVD and the product W U_b^T with the
    oracle's (unique where the rank is)."""
    w, v, t, P = small_problem()
    D_ref = ff.farfield_all(P)
    lay = T.Layout(w.n_theta, w.n_phi, P.offsets)
    g = T.fmm_geometry_build(v, t, w.origin, w.box, w.boxes_per_axis, w.k, w.n_theta, w.n_phi)
    h = None
    try:
        banner("compress svd small gamma=%g" % gamma)
        D = dev(np.zeros(D_ref.shape, np.complex128))
        T.fmm_farfield_fill(g, 0, P.n_groups, D)
        h = T.fmm_farfield_compress_svd(lay, D, 0, P.n_groups, gamma)
        ranks = T.fmm_tucker_ranks(h, P.n_groups)
        rng = synth.rng(w.seeds["x"])
        x = synth.complex_normal(rng, P.n_basis)
        gin = synth.complex_normal(rng, (P.n_groups, 2, P.n_dir))
        _, nbytes = T.fmm_tucker_storage_bytes(h, T.FMM_C128)
        ar = arena(nbytes)
        T.fmm_tucker_upload(h, T.FMM_C128, ar)
        F = dev(np.zeros((P.n_groups, 2, P.n_dir), np.complex128))
        V = dev(np.zeros(x.shape, np.complex128))
        T.fmm_tucker_pass(h, T.FMM_C128, 1, dev(x), F, dev(gin), V)
        F, V = host(F), host(V)
        facs = [[T.fmm_tucker_export(h, gg, a, ranks[gg, a], w.n_theta, w.n_phi,
                                     int(P.offsets[gg + 1] - P.offsets[gg])) for a in range(2)]
                for gg in range(P.n_groups)]
    finally:
        if h:
            T.fmm_tucker_destroy(h)
        T.fmm_geometry_destroy(g)
    from oracle import hosvd as H
    assert np.all(ranks[:, :, 0] == w.n_theta) and np.all(ranks[:, :, 1] == w.n_phi)
    v_dense = pr.disaggregate_all("dense", D_ref, P.offsets, gin)
    for gg in range(P.n_groups):
        lo, hi = P.offsets[gg], P.offsets[gg + 1]
        blk = D_ref[lo:hi]
        xs = x[lo:hi]
        f_dense = pr.dense_aggregate(blk, xs)
        vbound = 0.0
        for a in range(2):
            core, ut, up, ub = facs[gg][a]
            assert np.array_equal(ut, np.eye(w.n_theta)) and np.array_equal(up, np.eye(w.n_phi))
            assert np.allclose(ub.conj().T @ ub, np.eye(ub.shape[1]), atol=1e-12)
            anorm = np.linalg.norm(blk[:, a])
            bound = gamma * anorm * np.linalg.norm(xs)
            err = np.linalg.norm(F[gg, a] - f_dense[a])
            assert err <= bound * (1 + 1e-6) + 1e-12 * np.linalg.norm(f_dense[a]), (gg, a, err, bound)
            vbound += gamma * anorm * np.linalg.norm(gin[gg, a])
            w_ref, ub_ref, s = H.truncated_svd(H.tensorize(blk, a), gamma)
            rb = ub.shape[1]
            assert abs(rb - ub_ref.shape[1]) <= 1, (rb, ub_ref.shape[1])
            if rb == ub_ref.shape[1] and (rb == s.size or s[rb - 1] - s[rb] > 1e-6 * s[0]):
                wmat = core.reshape(P.n_dir, rb)
                got, ref = wmat @ ub.T, w_ref @ ub_ref.T
                assert np.linalg.norm(got - ref) <= 1e-9 * anorm, (gg, a)
        err = np.linalg.norm(V[lo:hi] - v_dense[lo:hi])
        assert err <= vbound * (1 + 1e-6) + 1e-12 * np.linalg.norm(v_dense[lo:hi]), (gg, err, vbound)


def test_saved_handle_computes_the_same(tmp_path):
    """A handle written by fmm_tucker_save and read back runs the same pass bit for bit."""
    w, v, t, P = small_problem()
    lay = T.Layout(w.n_theta, w.n_phi, P.offsets)
    g = T.fmm_geometry_build(v, t, w.origin, w.box, w.boxes_per_axis, w.k, w.n_theta, w.n_phi)
    hs = []
    try:
        banner("save/load small")
        D = dev(np.zeros((P.n_basis, 2, w.n_theta, w.n_phi), np.complex128))
        T.fmm_farfield_fill(g, 0, P.n_groups, D)
        hs.append(T.fmm_farfield_compress(lay, D, 0, P.n_groups, 1e-6))
        path = str(tmp_path / "small.tuck")
        T.fmm_tucker_save(hs[0], path)
        hs.append(T.fmm_tucker_load(path))
        rng = synth.rng(14)
        x = dev(synth.complex_normal(rng, P.n_basis), np.complex64)
        gin = dev(synth.complex_normal(rng, (P.n_groups, 2, P.n_dir)), np.complex64)
        outs, ars = [], []
        for h in hs:
            _, nbytes = T.fmm_tucker_storage_bytes(h, T.FMM_C64)
            ars.append(arena(nbytes))
            T.fmm_tucker_upload(h, T.FMM_C64, ars[-1])
            F = dev(np.zeros((P.n_groups, 2, P.n_dir), np.complex64))
            V = dev(np.zeros(P.n_basis, np.complex64))
            T.fmm_tucker_pass(h, T.FMM_C64, 1, x, F, gin, V)
            outs.append((host(F), host(V)))
    finally:
        for h in hs:
            T.fmm_tucker_destroy(h)
        T.fmm_geometry_destroy(g)
    assert np.array_equal(outs[0][0], outs[1][0]) and np.array_equal(outs[0][1], outs[1][1])


@pytest.mark.parametrize("split", [1, 700, 5000])
@pytest.mark.parametrize("prec,nrhs", [(T.FMM_C128, 1), (T.FMM_C64, 1), (T.FMM_C128, 3), (T.FMM_C64, 3)],
                         ids=["c128-1", "c64-1", "c128-3", "c64-2"])
def test_split_items(prec, nrhs, split, monkeypatch):
    """Items split into row blocks over several workgroups (forced at upload with a
    small split size; 1 gives blocks of four rows) against the oracle; the pass equals
    the separate stages bit for bit, and graph replays repeat it.  Half the groups are
    in truncated-SVD form."""
    import torch
    monkeypatch.setenv("TUCKFMM_SPLIT_ELEMS", str(split))
    lay = ragged_layout()
    banner("split items prec=%d nrhs=%d split=%d" % (prec, nrhs, split))
    gen = random_tucker(lay, 80, "random")
    svd = svd_as_tucker(lay, random_svd(lay, 81, "full"))
    tuck = [gen[g] if g % 2 else svd[g] for g in range(lay.n_groups)]
    rng = synth.rng(82)
    shp = (nrhs,) if nrhs > 1 else ()
    x = synth.complex_normal(rng, (lay.n_basis,) + shp)
    gin = synth.complex_normal(rng, (lay.n_groups, 2, lay.n_dir) + shp)
    f_ref, v_ref = oracle_tucker(lay, tuck, x, gin)
    h = make_handle(lay, tuck)
    try:
        _, nbytes = T.fmm_tucker_storage_bytes(h, prec)
        ar = arena(nbytes)
        T.fmm_tucker_upload(h, prec, ar)
        xd, gd = dev(x, CDT[prec]), dev(gin, CDT[prec])
        F1 = dev(np.zeros(f_ref.shape, CDT[prec]))
        V1 = dev(np.zeros(v_ref.shape, CDT[prec]))
        T.fmm_tucker_aggregate(h, prec, nrhs, xd, F1)
        T.fmm_tucker_disaggregate(h, prec, nrhs, gd, V1)
        F1, V1 = host(F1), host(V1)
        tol = TOL[prec]
        assert max_rel(F1, f_ref) < tol and l2_rel(F1, f_ref) < tol
        assert max_rel(V1, v_ref) < tol and l2_rel(V1, v_ref) < tol
        F = dev(np.zeros(f_ref.shape, CDT[prec]))
        V = dev(np.zeros(v_ref.shape, CDT[prec]))
        T.fmm_tucker_pass(h, prec, nrhs, xd, F, gd, V)
        assert np.array_equal(host(F), F1) and np.array_equal(host(V), V1)
        s = torch.cuda.Stream()
        with torch.cuda.stream(s):
            T.fmm_graph_capture(h, prec, nrhs, xd, F, gd, V, s)
        torch.cuda.synchronize()
        for _ in range(2):
            F.zero_()
            V.zero_()
            torch.cuda.synchronize()
            T.fmm_graph_launch(h, s)
            s.synchronize()
            assert np.array_equal(host(F), F1) and np.array_equal(host(V), V1)
    finally:
        T.fmm_tucker_destroy(h)


def test_compress_plate_with_a_zero_pattern_row():
    """A flat box of the trihedral's y = 0 plate: its phi-polarised pattern is exactly
    zero at phi = 0 (phi_hat . J = J_y = 0 there), so the phi unfolding has a zero row.
    The divide-and-conquer eigensolver has returned non-finite eigenvectors for that
    Gram matrix; the compressor must detect it, recompute, and match the oracle's
    ranks with finite factors and the gamma bound."""
    w = W.TRIHEDRAL
    v, t = w.mesh()
    P = geo.Problem(v, t, w.origin, w.box, w.boxes_per_axis, w.n_theta, w.n_phi)
    g = int(np.nonzero((P.box_index == [1, 0, 1]).all(axis=1))[0][0])
    banner("compress trihedral plate group %d" % g)
    blk = ff.farfield_group(P, g)
    assert np.all(blk[:, 1, :, 0] == 0)
    nb = blk.shape[0]
    lay = T.Layout(w.n_theta, w.n_phi, [0, nb])
    gamma = 1e-6
    h = T.fmm_farfield_compress(lay, dev(blk), 0, 1, gamma)
    try:
        ranks = T.fmm_tucker_ranks(h, 1)
        facs = [T.fmm_tucker_export(h, 0, a, ranks[0, a], w.n_theta, w.n_phi, nb) for a in range(2)]
        x = synth.complex_normal(synth.rng(15), nb)
        _, nbytes = T.fmm_tucker_storage_bytes(h, T.FMM_C128)
        ar = arena(nbytes)
        T.fmm_tucker_upload(h, T.FMM_C128, ar)
        F = dev(np.zeros((1, 2, P.n_dir), np.complex128))
        T.fmm_tucker_aggregate(h, T.FMM_C128, 1, dev(x), F)
        F = host(F)
    finally:
        T.fmm_tucker_destroy(h)
    from oracle import hosvd as H
    f_dense = pr.dense_aggregate(blk, x)
    for a in range(2):
        assert all(np.all(np.isfinite(f)) for f in facs[a])
        c_ref, _, _ = H.hosvd(H.tensorize(blk, a), gamma)
        assert np.all(np.abs(np.array(facs[a][0].shape) - np.array(c_ref.shape)) <= 1), (facs[a][0].shape,
                                                                                         c_ref.shape)
        bound = gamma * np.linalg.norm(blk[:, a]) * np.linalg.norm(x)
        assert np.linalg.norm(F[0, a] - f_dense[a]) <= bound * (1 + 1e-6)


@pytest.mark.parametrize("bad", [np.nan, np.inf], ids=["nan", "inf"])
@pytest.mark.parametrize("svd", [False, True], ids=["hosvd", "svd"])
def test_compress_rejects_non_finite_farfield(bad, svd):
    """A NaN or Inf far-field entry is reported as FMM_ERR_NUMERIC before any
    eigensolver sees the data, and no handle is left behind."""
    lay = ragged_layout()
    banner("compress non-finite %s svd=%s" % (bad, svd))
    rng = synth.rng(16)
    D = synth.complex_normal(rng, (lay.n_basis, 2, lay.n_theta, lay.n_phi))
    D[70, 1, 2, 3] = bad
    fn = T.fmm_farfield_compress_svd if svd else T.fmm_farfield_compress
    with pytest.raises(T.FmmError) as err:
        fn(lay, dev(D), 0, lay.n_groups, 1e-6)
    assert err.value.status == -5 and "non-finite" in str(err.value)
