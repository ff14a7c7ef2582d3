"""Benchmark: aggregation + disaggregation pass, Tucker FP32 vs dense FP64, one GPU.

Workload (default): the 30-wavelength PEC sphere of Section III.B as a synthetic
stand-in -- geodesic sphere with 939,870 RWG basis functions, FMM box 2 lambda
(1034 groups), the paper's 38 x 75 angular grid (L = 37 at 5 digits), Tucker
tolerance 1e-6, one seeded complex-Gaussian right-hand side.  Setup (far-field
fill of eq. (4), truncated HOSVD, arena upload) runs on the GPU before timing and
is reported separately.

One step = one pass of every hot-path stage over the resident inputs:
Tucker FP32 aggregation, Tucker FP32 disaggregation, dense FP64 aggregation and
dense FP64 disaggregation.  ``value`` is the Tucker FP32 pass throughput in GB/s
of algorithmic bytes (factors read once per stage plus the x/F and G/V vectors);
per-stage times, dense throughput, the roofline fraction of the dominant kernel,
accuracy against the FP64 oracle on sampled groups and the oracle's own CPU
throughput are reported beside it.

Prints exactly one JSON line on stdout; progress goes to stderr.

``--sweep gamma|digits|box`` instead measures the trends of Figs. 5-7 (trihedral)
and 9-11 (sphere): memory and FP64 aggregation / disaggregation time of the Tucker
and truncated-SVD models against the dense far-fields while the tolerance, the FMM
accuracy (grid size) or the box size changes; it prints one JSON line of points.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
COPY_BYTES = 1 << 30
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic_sphere30.md")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    p = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=20)
    p.add_argument("--warmup", type=int, default=3)
    p.add_argument("--workload", default="sphere30",
                   choices=["sphere30", "sphere30g29", "sphere6", "small", "sphere20b0.5", "sphere20b1", "sphere20b2",
                            "sphere20b4", "sphere45", "trihedral", "trihedral_small"])
    p.add_argument("--sample-groups", type=int, default=6, help="groups checked against the oracle")
    p.add_argument("--cpu-seconds", type=float, default=12.0,
                   help="budget of the oracle CPU timing (0: no CPU baseline)")
    p.add_argument("--no-oracle", action="store_true", help="skip accuracy sampling and the CPU baseline")
    p.add_argument("--no-dense", action="store_true", help="Tucker stages only (profiling runs)")
    p.add_argument("--no-dense-rhs", action="store_true", help="skip the dense pass with 8 right-hand sides")
    p.add_argument("--nrhs", type=int, default=None,
                   help="right-hand sides of the multi-RHS section (default: the workload's, else 64; 0: skip)")
    p.add_argument("--mrhs-precs", default="c128,c64,bf16x2,bf16x3",
                   help="precisions of the multi-RHS section (c128, c64, bf16x2, bf16x3)")
    p.add_argument("--no-tune", action="store_true",
                   help="multi-RHS section: default kernel choice instead of the autotuner (profiling runs)")
    p.add_argument("--setup-chunk", type=int, default=128,
                   help="groups per far-field fill + compress chunk when the dense tensor is not kept")
    p.add_argument("--mrhs-steps", type=int, default=10, help="timed passes per multi-RHS precision")
    p.add_argument("--no-svd", action="store_true", help="skip the truncated-SVD comparison")
    p.add_argument("--no-grid", action="store_true", help="skip the box-grid pass")
    p.add_argument("--no-extra", action="store_true",
                   help="skip the other stated configurations (Tucker FP64 pass, gamma = 1e-4, 29 x 58 grid)")
    p.add_argument("--sweep", choices=["gamma", "digits", "box"], default=None,
                   help="measure compression and speedup trends instead of the pass benchmark")
    p.add_argument("--save-factors", default=None, help="write the compressed factors to this file")
    p.add_argument("--load-factors", default=None, help="read the factors from this file instead of compressing")
    return p.parse_args()


def workload(name):
    from synth import workloads as W
    table = {"sphere30": W.SPHERE30, "sphere30g29": W.SPHERE30_G29, "sphere6": W.SPHERE6, "small": W.SMALL,
             "sphere45": W.SPHERE45, "trihedral": W.TRIHEDRAL, "trihedral_small": W.TRIHEDRAL_SMALL}
    for box, wl in W.SPHERE20.items():
        table["sphere20b%g" % box] = wl
    return table[name]


def tucker_stage_bytes(ranks, offsets, n_theta, n_phi, es):
    """Algorithmic bytes of one Tucker stage: every factor and core read once, plus
    the group vectors (x or V: N values) and patterns (F or G: 2 G N_dir values)."""
    nb = np.diff(offsets)
    rt, rp, rb = ranks[..., 0].astype(np.int64), ranks[..., 1].astype(np.int64), ranks[..., 2].astype(np.int64)
    fac = (nb[:, None] * rb + n_theta * rt + n_phi * rp + rt * rp * rb).sum()
    io = int(offsets[-1]) + 2 * (offsets.size - 1) * n_theta * n_phi
    return int(es * (fac + io)), int(es * fac)


def tucker_stage_flops(ranks, offsets, n_theta, n_phi, nrhs):
    """Algorithmic real flops of one Tucker stage for nrhs right-hand sides: 8 per
    complex multiply-add, the beta and core contractions plus the cheaper order of the
    two angular ones."""
    nb = np.diff(offsets)[:, None]
    rt, rp, rb = ranks[..., 0].astype(np.int64), ranks[..., 1].astype(np.int64), ranks[..., 2].astype(np.int64)
    ang = np.minimum(n_theta * rp * (rt + n_phi), rt * n_phi * (rp + n_theta))
    return int(8 * nrhs * (nb * rb + rt * rp * rb + ang).sum())


def kernel_source_sha(name):
    import hashlib
    with open(os.path.join(ROOT, "paper_2103_05822_amd", "csrc", name), "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def measured_traffic(kernel, source, workload_name):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter summary:
    FETCH_SIZE and WRITE_SIZE per dispatch, each scaled by the ratio of known bytes to
    the counter's reading for the calibration copy.  None when the summary is missing,
    covers another workload, or was taken from another version of the kernel's source
    file."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    rec = {}
    for ln in open(TRAFFIC_FILE):
        if ln.startswith("traffic:"):
            kv = dict(t.split("=", 1) for t in ln.split()[1:])
            rec[kv["kernel"]] = kv
    r = rec.get(kernel)
    if r is None or r.get("src_sha") != kernel_source_sha(source) or r.get("workload") != workload_name:
        return None
    return int(float(r["hbm_bytes"]))


def svd_stage_bytes(ranks, offsets, n_theta, n_phi, es):
    """Algorithmic bytes of one truncated-SVD stage: W [N_dir, r_b] and U_b [n_beta, r_b]
    of every tensor read once, plus the group vectors and patterns."""
    nb = np.diff(offsets)
    rb = ranks[..., 2].astype(np.int64)
    fac = (nb[:, None] * rb + n_theta * n_phi * rb).sum()
    io = int(offsets[-1]) + 2 * (offsets.size - 1) * n_theta * n_phi
    return int(es * (fac + io)), int(es * fac)


def dense_stage_bytes(offsets, n_theta, n_phi, es):
    n = int(offsets[-1])
    g = offsets.size - 1
    return int(es * (n * 2 * n_theta * n_phi + n + 2 * g * n_theta * n_phi))


def save_factors(T, h, path):
    """The handle's FP64 factors in the library's own file format."""
    T.fmm_tucker_save(h, path)


def load_factors(T, lay, path):
    h = T.fmm_tucker_load(path)
    if not np.array_equal(T.fmm_tucker_layout(h).offsets, lay.offsets):
        T.fmm_tucker_destroy(h)
        raise SystemExit("factor file %s is for another layout" % path)
    return h


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the aggregation and disaggregation stages have no "
              "cross-GPU exchange in this build (groups would shard with no communication); "
              "run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2103_05822_amd as T
    import synth

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    w = workload(args.workload)
    if args.sweep:
        print(json.dumps(sweep(args, T, torch, synth, w)), flush=True)
        return
    t_setup = time.time()

    # ---------------------------------------------------------------- setup (untimed)
    verts, tris = w.mesh()
    geom = T.fmm_geometry_build(verts, tris, w.origin, w.box, w.boxes_per_axis, w.k, w.n_theta, w.n_phi)
    lay = T.fmm_geometry_layout(geom)
    N, G, nd = lay.n_basis, lay.n_groups, lay.n_dir
    log("geometry: N=%d groups=%d grid=%dx%d" % (N, G, w.n_theta, w.n_phi))
    if args.workload == "sphere45":
        args.no_dense = True   # the dense far-fields of this workload are never materialised
    if args.nrhs is None:
        args.nrhs = w.nrhs if w.nrhs > 1 else 64
    t0 = time.time()
    dense = None
    if not args.no_dense:
        dense = torch.empty((N, 2, w.n_theta, w.n_phi), dtype=torch.complex128, device="cuda")
        T.fmm_farfield_fill(geom, 0, G, dense)
        torch.cuda.synchronize()
    if args.load_factors:
        h = load_factors(T, lay, args.load_factors)
        log("factors loaded from %s (%.1f s)" % (args.load_factors, time.time() - t0))
    else:
        # group chunks: progress shows during long setups; without a dense tensor every
        # chunk's far-fields are filled into one reusable buffer and compressed (streaming)
        h = None
        chunk = args.setup_chunk
        buf = None
        if dense is None:
            rows = max(int(lay.offsets[min(G, g0 + chunk)] - lay.offsets[g0]) for g0 in range(0, G, chunk))
            buf = torch.empty((rows, 2, w.n_theta, w.n_phi), dtype=torch.complex128, device="cuda")
        for g0 in range(0, G, chunk):
            cnt = min(chunk, G - g0)
            rows0 = int(lay.offsets[g0])
            if dense is None:
                T.fmm_farfield_fill(geom, g0, cnt, buf)
                src = buf
            else:
                src = dense[rows0:]
            h = T.fmm_farfield_compress(lay, src, g0, cnt, w.gamma, handle=h)
            log("compress: groups %d..%d done (%.1f s)" % (g0, g0 + cnt - 1, time.time() - t0))
        src = buf = None   # a view of `dense` would keep it alive
    t_compress = time.time() - t0
    ranks = T.fmm_tucker_ranks(h, G)
    if args.save_factors:
        save_factors(T, h, args.save_factors)
        log("factors saved to %s" % args.save_factors)
    log("compress: %.1f s, mean ranks %s" % (t_compress, ranks.reshape(-1, 3).mean(0).round(1)))
    # groups checked against the oracle, and their stored factors (arithmetic-only parity)
    sample = sampled_groups(synth, np.diff(lay.offsets), args.sample_groups)
    stored = {"c64": export_sample(T, h, ranks, sample, lay, T.FMM_C64),
              "c128": export_sample(T, h, ranks, sample, lay, T.FMM_C128)}
    arenas = {}
    for prec in (T.FMM_C64,):
        _, nbytes = T.fmm_tucker_storage_bytes(h, prec)
        arenas[prec] = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        T.fmm_tucker_upload(h, prec, arenas[prec])
    dplan = T.fmm_dense_create(lay)

    x = synth.complex_normal(synth.rng(w.seeds.get("x", 0)), N)
    gin = synth.complex_normal(synth.rng(w.seeds.get("g", 1)), (G, 2, nd))
    x32 = torch.from_numpy(x).to("cuda", torch.complex64)
    g32 = torch.from_numpy(gin).to("cuda", torch.complex64)
    x64 = torch.from_numpy(x).to("cuda")
    g64 = torch.from_numpy(gin).to("cuda")
    F32 = torch.empty((G, 2, nd), dtype=torch.complex64, device="cuda")
    V32 = torch.empty(N, dtype=torch.complex64, device="cuda")
    F64 = torch.empty((G, 2, nd), dtype=torch.complex128, device="cuda")
    V64 = torch.empty(N, dtype=torch.complex128, device="cuda")
    torch.cuda.synchronize()
    t_setup = time.time() - t_setup
    log("setup: %.1f s" % t_setup)

    # the Tucker pass is replayed from a captured graph (one launch for both stages)
    gstream = torch.cuda.Stream()
    with torch.cuda.stream(gstream):
        T.fmm_graph_capture(h, T.FMM_C64, 1, x32, F32, g32, V32, gstream)
    torch.cuda.synchronize()
    stages = [("tucker_pass_f32", lambda: T.fmm_graph_launch(h, torch.cuda.current_stream()))]
    if not args.no_dense:
        stages += [("dense_agg_f64", lambda: T.fmm_dense_aggregate(dplan, T.FMM_C128, dense, 1, x64, F64)),
                   ("dense_disagg_f64", lambda: T.fmm_dense_disaggregate(dplan, T.FMM_C128, dense, 1, g64, V64))]

    # first launch of each stage, alone and before the warm-up: device time and host
    # wall time to completion (the graph's first replay includes its upload)
    first_ms = {}
    for name, fn in stages:
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        tw = time.perf_counter()
        a.record()
        fn()
        b.record()
        torch.cuda.synchronize()
        first_ms[name] = {"gpu": round(a.elapsed_time(b), 4), "wall": round((time.perf_counter() - tw) * 1e3, 4)}

    # ---------------------------------------------------------------- timed region
    for _ in range(args.warmup):
        for _, fn in stages:
            fn()
    torch.cuda.synchronize()
    ev = {name: [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
                 for _ in range(args.steps)] for name, _ in stages}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        for name, fn in stages:
            a, b = ev[name][k]
            a.record()
            fn()
            b.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = {name: float(np.mean([a.elapsed_time(b) for a, b in ev[name]])) for name, _ in stages}

    # stage breakdown of the Tucker path (separate launches), outside the timed steps
    split = [("tucker_agg_f32", lambda: T.fmm_tucker_aggregate(h, T.FMM_C64, 1, x32, F32)),
             ("tucker_disagg_f32", lambda: T.fmm_tucker_disaggregate(h, T.FMM_C64, 1, g32, V32))]
    for name, fn in split:
        fn()
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(10)]
        for a, b in evs:
            a.record()
            fn()
            b.record()
        torch.cuda.synchronize()
        ms[name] = float(np.mean([a.elapsed_time(b) for a, b in evs]))
    log("stage ms: %s" % {k: round(v, 4) for k, v in ms.items()})

    # practical-bandwidth reference and HBM-counter calibration: a plain elementwise
    # copy (dst = src * 1) of 1 GiB, 1 GiB read + 1 GiB written per launch
    csrc = torch.ones(COPY_BYTES // 4, dtype=torch.float32, device="cuda")
    cdst = torch.empty_like(csrc)
    torch.mul(csrc, 1.0, out=cdst)
    cev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(5)]
    for a, b in cev:
        a.record()
        torch.mul(csrc, 1.0, out=cdst)
        b.record()
    torch.cuda.synchronize()
    copy_gbs = 2 * COPY_BYTES / (min(a.elapsed_time(b) for a, b in cev) * 1e-3) / 1e9
    del csrc, cdst

    b_t32, fac32 = tucker_stage_bytes(ranks, lay.offsets, w.n_theta, w.n_phi, 8)
    b_d64 = dense_stage_bytes(lay.offsets, w.n_theta, w.n_phi, 16)
    per_stage_bytes = {"tucker_pass_f32": 2 * b_t32, "tucker_agg_f32": b_t32, "tucker_disagg_f32": b_t32,
                       "dense_agg_f64": b_d64, "dense_disagg_f64": b_d64}
    gbs = {k: per_stage_bytes[k] / (ms[k] * 1e-3) / 1e9 for k in ms}
    tucker_ms = ms["tucker_pass_f32"]
    tucker_gbs = gbs["tucker_pass_f32"]
    dom = "tucker_pass_f32"

    result = {
        "metric": "agg+disagg pass time & GB/s: Tucker FP32 vs dense FP64, 1 GPU, at <=1e-5 rel err",
        "value": round(tucker_gbs, 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall / args.steps * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": w.name, "n_basis": N, "n_groups": G, "grid": [w.n_theta, w.n_phi],
                   "gamma": w.gamma, "nrhs": 1, "tucker_storage": "complex64", "dense_storage": "complex128"},
        "tucker_pass_ms": round(tucker_ms, 4),
        "stage_ms": {k: round(v, 4) for k, v in ms.items()},
        "first_launch_ms": first_ms,
        "stage_GBps": {k: round(v, 1) for k, v in gbs.items()},
        "roofline": {"bound": "hbm", "kernel": "tucker_pass_kernel<float> (+ V zeroing)", "achieved": round(gbs[dom], 1),
                     "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(gbs[dom] / HBM_PEAK_GBS, 4),
                     "traffic": measured_traffic("tucker_pass_kernel<float>", "tucker.hip", w.name),
                     "bytes_per_launch": per_stage_bytes[dom]},
        "copy_GBps": round(copy_gbs, 1),
        "memory_MB": {"tucker_factors_f32": round(fac32 / 2 ** 20, 1),
                      "dense_f64": round(2 * N * nd * 16 / 2 ** 20, 1)},
        "ranks_mean": [round(float(v), 2) for v in ranks.reshape(-1, 3).mean(0)],
        "setup_s": round(t_setup, 2),
        "compress_s": round(t_compress, 2),
        "paper_cpu_context": {"tucker_speedup_agg": 15.2, "tucker_speedup_disagg": 15.8,
                              "memory_reduction": ">87%", "hardware": "Xeon Gold 6142, Matlab 2019b"},
    }
    if not args.no_dense:
        dense_ms = ms["dense_agg_f64"] + ms["dense_disagg_f64"]
        result["dense_pass_ms"] = round(dense_ms, 4)
        result["dense_pass_GBps"] = round(2 * b_d64 / (dense_ms * 1e-3) / 1e9, 1)
        result["speedup_vs_dense"] = {"agg": round(ms["dense_agg_f64"] / ms["tucker_agg_f32"], 2),
                                      "disagg": round(ms["dense_disagg_f64"] / ms["tucker_disagg_f32"], 2),
                                      "pass": round(dense_ms / tucker_ms, 2)}

    # --------------------------------------------- truncated-SVD comparison (Table III)
    svd_out = None
    if not args.no_dense and not args.no_svd:
        result["svd_comparison"], svd_out = svd_comparison(args, T, torch, lay, dense, w, x32, g32,
                                                           tucker_ms, fac32)

    # ------------------------------------------------- box-grid spectra (eq. (3), (5))
    if not args.no_grid:
        result["box_grid"] = box_grid_pass(T, torch, geom, h, lay, w, arenas[T.FMM_C64], x32, g32, F32, V32,
                                           tucker_ms, per_stage_bytes["tucker_pass_f32"])

    # the plain method with 8 right-hand sides: one read of A serves all 8
    if not args.no_dense and not args.no_dense_rhs:
        result["dense_8rhs"] = dense_rhs_block(T, torch, synth, dplan, dense, x64, g64, F64, V64,
                                               result["dense_pass_ms"], b_d64)

    # ------------------------- the other stated configurations of the same sphere
    extra = {}
    if not args.no_dense and not args.no_extra:
        # Tucker FP64 single-RHS pass (the FP64 plain-method comparison of the paper's
        # Table III, on the GPU)
        result["tucker_fp64_pass"], extra["tucker_f64"] = fp64_pass(
            T, torch, h, lay, w, ranks, x64, g64, sample, result.get("dense_pass_ms"))
        # tolerance 1e-4 (Table III's first Tucker row), FP32 pass
        result["gamma_1e-4"], extra["gamma_1e-4_f32"] = gamma_pass(
            args, T, torch, lay, dense, w, 1e-4, x32, g32, sample, result.get("dense_pass_ms"))
    if args.workload == "sphere30" and not args.no_extra and not args.no_dense:
        dense = None
        torch.cuda.empty_cache()
        # the coarser 29 x 58 grid the configuration names, dense FP64 and Tucker FP32
        from synth import workloads as W
        result["grid_29x58"], extra["grid_29x58"] = grid_pass(args, T, torch, synth, W.SPHERE30_G29, verts,
                                                               tris, sample)

    # ------------------------------------------------------------ multi-RHS section
    mr_out = {}
    if args.nrhs > 0:
        dense = None
        torch.cuda.empty_cache()
        result["multi_rhs"], mr_out = multi_rhs(args, T, torch, synth, h, geom, lay, ranks, w, sample)

    # ------------------------------------------------ accuracy + CPU baseline (oracle)
    if not args.no_oracle:
        F32h, V32h = F32.cpu().numpy(), V32.cpu().numpy()
        F64h = V64h = None
        if not args.no_dense:
            F64h, V64h = F64.cpu().numpy(), V64.cpu().numpy()
        result.update(oracle_checks(args, w, verts, tris, lay, x, gin, F32h, V32h, F64h, V64h, sample, stored,
                                    mr_out, svd_out, extra))

    T.fmm_dense_destroy(dplan)
    T.fmm_tucker_destroy(h)
    T.fmm_geometry_destroy(geom)
    print(json.dumps(result), flush=True)


MRHS_PRECS = {"c128": 0, "c64": 1, "bf16x2": 2, "bf16x3": 3}


def sampled_groups(synth, nb, n):
    """Groups checked against the oracle: the largest plus seeded draws (default_rng(4))."""
    big = int(np.argmax(nb))
    draws = [int(g) for g in synth.rng(4).choice(nb.size, size=min(n, nb.size), replace=False) if g != big]
    return sorted([big] + draws[:max(0, n - 1)])


def export_sample(T, h, ranks, sample, lay, prec):
    """Stored factors of the sampled groups as the arena of `prec` holds them, in the
    oracle's per-group form [(core, (U^theta, U^phi, U^beta))] * 2."""
    nb = np.diff(lay.offsets)
    out = {}
    for g in sample:
        pair = []
        for a in range(2):
            c, ut, up, ub = T.fmm_tucker_export(h, g, a, ranks[g, a], lay.n_theta, lay.n_phi, int(nb[g]),
                                                as_stored=prec)
            pair.append((c, (ut, up, ub)))
        out[g] = pair
    return out


def graph_time(torch, T, h, prec, nrhs, x, F, G, V, reps=10):
    """Capture the pass in a graph, replay it (3 untimed, `reps` timed) and return the
    mean ms per replay, HIP events on the graph's stream."""
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        T.fmm_graph_capture(h, prec, nrhs, x, F, G, V, s)
    torch.cuda.synchronize()
    for _ in range(3):
        T.fmm_graph_launch(h, s)
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    for a, b in evs:
        a.record(s)
        T.fmm_graph_launch(h, s)
        b.record(s)
    torch.cuda.synchronize()
    return float(np.mean([a.elapsed_time(b) for a, b in evs]))


def sample_outputs(F, V, sample, offsets):
    return {g: (F[g].cpu().numpy(), V[int(offsets[g]):int(offsets[g + 1])].cpu().numpy()) for g in sample}


def fp64_pass(T, torch, h, lay, w, ranks, x64, g64, sample, dense_ms):
    """Tucker FP64 single-RHS pass (complex128 factors and vectors) on the same handle,
    graph-captured; algorithmic bytes as the FP32 pass with 16-byte elements."""
    G, nd, N = lay.n_groups, lay.n_dir, lay.n_basis
    _, nbytes = T.fmm_tucker_storage_bytes(h, T.FMM_C128)
    ar = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    T.fmm_tucker_upload(h, T.FMM_C128, ar)
    F = torch.empty((G, 2, nd), dtype=torch.complex128, device="cuda")
    V = torch.empty(N, dtype=torch.complex128, device="cuda")
    ms = graph_time(torch, T, h, T.FMM_C128, 1, x64, F, g64, V)
    b_stage, fac = tucker_stage_bytes(ranks, lay.offsets, w.n_theta, w.n_phi, 16)
    gbs = 2 * b_stage / (ms * 1e-3) / 1e9
    rep = {"pass_ms": round(ms, 4), "GBps": round(gbs, 1), "hbm_frac": round(gbs / HBM_PEAK_GBS, 4),
           "factors_MB_f64": round(fac / 2 ** 20, 1)}
    if dense_ms:
        rep["speedup_vs_dense_f64_pass"] = round(dense_ms / ms, 2)
    log("tucker FP64 pass: %s" % rep)
    out = sample_outputs(F, V, sample, lay.offsets)
    del ar
    return rep, out


def dense_rhs_block(T, torch, synth, dplan, dense, x64, g64, F64, V64, dense_ms, stage_bytes, R=8):
    """Dense FP64 pass (eqs. (3), (5)) with R = 8 right-hand sides, whose kernels read
    each far-field element once for all of them.  Column 0 holds the single-RHS inputs,
    so it must reproduce that pass's F and V; the other columns are seeded draws."""
    N, (G, _, nd) = x64.shape[0], g64.shape
    gen = synth.rng(7)
    xr = torch.from_numpy(synth.complex_normal(gen, (N, R))).to("cuda")
    gr = torch.from_numpy(synth.complex_normal(gen, (G, 2, nd, R))).to("cuda")
    xr[:, 0] = x64
    gr[..., 0] = g64
    Fr = torch.empty((G, 2, nd, R), dtype=torch.complex128, device="cuda")
    Vr = torch.empty((N, R), dtype=torch.complex128, device="cuda")

    def run():
        T.fmm_dense_aggregate(dplan, T.FMM_C128, dense, R, xr, Fr)
        T.fmm_dense_disaggregate(dplan, T.FMM_C128, dense, R, gr, Vr)

    run()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(5)]
    for a, b in evs:
        a.record()
        run()
        b.record()
    torch.cuda.synchronize()
    pass_ms = float(np.mean([a.elapsed_time(b) for a, b in evs]))
    rel = lambda u, v: float((u - v).abs().max() / v.abs().max())   # noqa: E731
    vec_bytes = 16 * (R - 1) * 2 * (N + G * 2 * nd)   # the extra columns' x, F, G and V
    out = {"nrhs": R, "pass_ms": round(pass_ms, 4), "ratio_vs_1rhs_pass": round(pass_ms / dense_ms, 3),
           "GBps": round((2 * stage_bytes + vec_bytes) / (pass_ms * 1e-3) / 1e9, 1),
           "column0_max_rel_diff_vs_1rhs": {"F": rel(Fr[..., 0], F64), "V": rel(Vr[:, 0], V64)}}
    log("dense FP64 pass, %d RHS: %s" % (R, out))
    del xr, gr, Fr, Vr
    torch.cuda.empty_cache()
    return out


def gamma_pass(args, T, torch, lay, dense, w, gamma, x32, g32, sample, dense_ms):
    """The same far-fields compressed at another tolerance, FP32 pass (graph-captured).
    Returns the report and (sampled outputs, stored factors of the sample)."""
    G, nd, N = lay.n_groups, lay.n_dir, lay.n_basis
    t0 = time.time()
    h2 = None
    for g0 in range(0, G, args.setup_chunk):
        h2 = T.fmm_farfield_compress(lay, dense[int(lay.offsets[g0]):], g0, min(args.setup_chunk, G - g0), gamma,
                                     handle=h2)
    t_c = time.time() - t0
    try:
        ranks = T.fmm_tucker_ranks(h2, G)
        fb, nbytes = T.fmm_tucker_storage_bytes(h2, T.FMM_C64)
        ar = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        T.fmm_tucker_upload(h2, T.FMM_C64, ar)
        F = torch.empty((G, 2, nd), dtype=torch.complex64, device="cuda")
        V = torch.empty(N, dtype=torch.complex64, device="cuda")
        ms = graph_time(torch, T, h2, T.FMM_C64, 1, x32, F, g32, V)
        b_stage, fac = tucker_stage_bytes(ranks, lay.offsets, w.n_theta, w.n_phi, 8)
        gbs = 2 * b_stage / (ms * 1e-3) / 1e9
        fb64, _ = T.fmm_tucker_storage_bytes(h2, T.FMM_C128)
        rep = {"gamma": gamma, "compress_s": round(t_c, 2), "pass_ms": round(ms, 4), "GBps": round(gbs, 1),
               "hbm_frac": round(gbs / HBM_PEAK_GBS, 4), "factors_MB_f32": round(fb / 2 ** 20, 1),
               "factors_MB_f64": round(fb64 / 2 ** 20, 1),
               "ranks_mean": [round(float(v), 2) for v in ranks.reshape(-1, 3).mean(0)]}
        if dense_ms:
            rep["speedup_vs_dense_f64_pass"] = round(dense_ms / ms, 2)
        log("gamma %g FP32 pass: %s" % (gamma, rep))
        out = (sample_outputs(F, V, sample, lay.offsets), export_sample(T, h2, ranks, sample, lay, T.FMM_C64))
        del ar
        return rep, out
    finally:
        T.fmm_tucker_destroy(h2)


def grid_pass(args, T, torch, synth, wg, verts, tris, sample):
    """The sphere on another angular grid: dense FP64 far-fields filled, compressed,
    Tucker FP32 pass (graph) and dense FP64 stages timed, outputs of the sample kept."""
    geom = T.fmm_geometry_build(verts, tris, wg.origin, wg.box, wg.boxes_per_axis, wg.k, wg.n_theta, wg.n_phi)
    h = None
    dplan = None
    try:
        lay = T.fmm_geometry_layout(geom)
        N, G, nd = lay.n_basis, lay.n_groups, lay.n_dir
        t0 = time.time()
        dense = torch.empty((N, 2, wg.n_theta, wg.n_phi), dtype=torch.complex128, device="cuda")
        T.fmm_farfield_fill(geom, 0, G, dense)
        for g0 in range(0, G, args.setup_chunk):
            h = T.fmm_farfield_compress(lay, dense[int(lay.offsets[g0]):], g0, min(args.setup_chunk, G - g0),
                                        wg.gamma, handle=h)
        t_c = time.time() - t0
        ranks = T.fmm_tucker_ranks(h, G)
        fb, nbytes = T.fmm_tucker_storage_bytes(h, T.FMM_C64)
        ar = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        T.fmm_tucker_upload(h, T.FMM_C64, ar)
        x = synth.complex_normal(synth.rng(wg.seeds.get("x", 0)), N)
        gin = synth.complex_normal(synth.rng(wg.seeds.get("g", 1)), (G, 2, nd))
        x32, g32 = torch.from_numpy(x).to("cuda", torch.complex64), torch.from_numpy(gin).to("cuda", torch.complex64)
        x64, g64 = torch.from_numpy(x).to("cuda"), torch.from_numpy(gin).to("cuda")
        F = torch.empty((G, 2, nd), dtype=torch.complex64, device="cuda")
        V = torch.empty(N, dtype=torch.complex64, device="cuda")
        ms = graph_time(torch, T, h, T.FMM_C64, 1, x32, F, g32, V)
        dplan = T.fmm_dense_create(lay)
        F64 = torch.empty((G, 2, nd), dtype=torch.complex128, device="cuda")
        V64 = torch.empty(N, dtype=torch.complex128, device="cuda")
        dagg = time_ms(torch, lambda: T.fmm_dense_aggregate(dplan, T.FMM_C128, dense, 1, x64, F64), reps=5)
        ddis = time_ms(torch, lambda: T.fmm_dense_disaggregate(dplan, T.FMM_C128, dense, 1, g64, V64), reps=5)
        b_stage, fac = tucker_stage_bytes(ranks, lay.offsets, wg.n_theta, wg.n_phi, 8)
        b_d64 = dense_stage_bytes(lay.offsets, wg.n_theta, wg.n_phi, 16)
        gbs = 2 * b_stage / (ms * 1e-3) / 1e9
        rep = {"workload": wg.name, "grid": [wg.n_theta, wg.n_phi], "compress_s": round(t_c, 2),
               "tucker_pass_ms": round(ms, 4), "tucker_pass_GBps": round(gbs, 1),
               "hbm_frac": round(gbs / HBM_PEAK_GBS, 4),
               "dense_pass_ms": round(dagg + ddis, 4),
               "dense_pass_GBps": round(2 * b_d64 / ((dagg + ddis) * 1e-3) / 1e9, 1),
               "speedup_vs_dense_pass": round((dagg + ddis) / ms, 2),
               "memory_MB": {"tucker_factors_f32": round(fb / 2 ** 20, 1),
                             "dense_f64": round(2 * N * nd * 16 / 2 ** 20, 1)},
               "ranks_mean": [round(float(v), 2) for v in ranks.reshape(-1, 3).mean(0)]}
        log("grid %dx%d: %s" % (wg.n_theta, wg.n_phi, rep))
        out = {"x": x, "gin": gin, "w": wg, "f32": sample_outputs(F, V, sample, lay.offsets),
               "f64_dense": sample_outputs(F64, V64, sample, lay.offsets),
               "stored": export_sample(T, h, ranks, sample, lay, T.FMM_C64)}
        del ar, dense
        return rep, out
    finally:
        if dplan:
            T.fmm_dense_destroy(dplan)
        if h:
            T.fmm_tucker_destroy(h)
        T.fmm_geometry_destroy(geom)

# L of the angular grid (Section II.A: L = 2kR + (2kR)^(1/3) 1.8 d^(2/3), R half the box
# diagonal, rounded, plus one) for the sweep points, by (box edge, digits d).
GRID_ORDER = {(0.5, 3): 13, (1.0, 3): 20, (1.5, 3): 27, (2.0, 3): 33,
              (0.5, 4): 14, (1.0, 4): 22, (1.5, 4): 29, (2.0, 4): 35,
              (0.5, 5): 16, (1.0, 5): 24, (1.5, 5): 31, (2.0, 5): 37,
              (0.5, 6): 17, (1.0, 6): 25, (1.5, 6): 32, (2.0, 6): 39}


def time_ms(torch, fn, reps=5):
    fn()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    for a, b in evs:
        a.record()
        fn()
        b.record()
    torch.cuda.synchronize()
    return float(np.median([a.elapsed_time(b) for a, b in evs]))


def sweep(args, T, torch, synth, w):
    """Trends of Figs. 5-7 / 9-11: per point, far-fields filled and compressed on the
    GPU by both methods at the point's tolerance, FP64 memory (2^20-byte MB as the
    paper's tables) and FP64 stage times, plus the FP32 pass of each method."""
    import math
    if args.sweep == "gamma":
        pts = [(w.box, 5, g) for g in (1e-3, 1e-4, 1e-5, 1e-6, 1e-7)]
    elif args.sweep == "digits":
        pts = [(w.box, d, w.gamma) for d in (3, 4, 5, 6)]
    else:
        pts = [(b, 5, w.gamma) for b in (0.5, 1.0, 1.5, 2.0)]
    verts, tris = w.mesh()
    out = {"sweep": args.sweep, "workload": w.name, "n_basis": w.n_basis, "points": []}
    for box, digits, gamma in pts:
        L = GRID_ORDER[(box, digits)]
        nt, nph = L + 1, 2 * L + 1
        K = int(math.ceil(w.diameter / box - 1e-12))
        t0 = time.time()
        geom = T.fmm_geometry_build(verts, tris, w.origin, box, K, w.k, nt, nph)
        lay = T.fmm_geometry_layout(geom)
        N, G, nd = lay.n_basis, lay.n_groups, lay.n_dir
        dense = torch.empty((N, 2, nt, nph), dtype=torch.complex128, device="cuda")
        T.fmm_farfield_fill(geom, 0, G, dense)
        torch.cuda.synchronize()
        handles = {}
        for name, fn in (("tucker", T.fmm_farfield_compress), ("svd", T.fmm_farfield_compress_svd)):
            h = None
            for g0 in range(0, G, args.setup_chunk):
                h = fn(lay, dense[int(lay.offsets[g0]):], g0, min(args.setup_chunk, G - g0), gamma, handle=h)
            handles[name] = h
            log("sweep point box=%g digits=%d gamma=%g: %s compressed (%.1f s)" % (box, digits, gamma, name,
                                                                                   time.time() - t0))
        rng = synth.rng(w.seeds.get("x", 0))
        x = synth.complex_normal(rng, N)
        gin = synth.complex_normal(rng, (G, 2, nd))
        x64, g64 = torch.from_numpy(x).to("cuda"), torch.from_numpy(gin).to("cuda")
        x32, g32 = x64.to(torch.complex64), g64.to(torch.complex64)
        F64 = torch.empty((G, 2, nd), dtype=torch.complex128, device="cuda")
        V64 = torch.empty(N, dtype=torch.complex128, device="cuda")
        F32, V32 = F64.to(torch.complex64), V64.to(torch.complex64)
        dplan = T.fmm_dense_create(lay)
        pt = {"box": box, "digits": digits, "gamma": gamma, "L": L, "grid": [nt, nph], "n_groups": G,
              "n_avg": round(N / G, 1),
              "dense_MB": round(16 * 2 * N * nd / 2 ** 20, 1),
              "ms": {"dense_agg": time_ms(torch, lambda: T.fmm_dense_aggregate(dplan, T.FMM_C128, dense, 1, x64, F64)),
                     "dense_disagg": time_ms(torch, lambda: T.fmm_dense_disaggregate(dplan, T.FMM_C128, dense, 1,
                                                                                     g64, V64))}}
        T.fmm_dense_destroy(dplan)
        dense = None
        torch.cuda.empty_cache()
        for name, h in handles.items():
            ranks = T.fmm_tucker_ranks(h, G)
            fb, _ = T.fmm_tucker_storage_bytes(h, T.FMM_C128)
            pt[name + "_MB"] = round(fb / 2 ** 20, 1)
            pt[name + "_ranks_mean"] = [round(float(v), 1) for v in ranks.reshape(-1, 3).mean(0)]
            for prec, tag, xx, gg, FF, VV in ((T.FMM_C128, "64", x64, g64, F64, V64),
                                             (T.FMM_C64, "32", x32, g32, F32, V32)):
                _, ab = T.fmm_tucker_storage_bytes(h, prec)
                ar = torch.empty(ab, dtype=torch.uint8, device="cuda")
                T.fmm_tucker_upload(h, prec, ar)
                if prec == T.FMM_C128:
                    pt["ms"][name + "_agg"] = time_ms(torch, lambda: T.fmm_tucker_aggregate(h, prec, 1, xx, FF))
                    pt["ms"][name + "_disagg"] = time_ms(torch, lambda: T.fmm_tucker_disaggregate(h, prec, 1, gg, VV))
                else:
                    pt["ms"][name + "_pass_f32"] = time_ms(torch, lambda: T.fmm_tucker_pass(h, prec, 1, xx, FF, gg, VV))
                if not (bool(torch.isfinite(torch.view_as_real(FF)).all()) and
                        bool(torch.isfinite(torch.view_as_real(VV)).all())):
                    raise SystemExit("sweep point %s: non-finite %s outputs" % (json.dumps(pt), name))
                del ar
            T.fmm_tucker_destroy(h)
        m = pt["ms"]
        for name in handles:
            pt[name + "_compression"] = round(pt["dense_MB"] / pt[name + "_MB"], 2)
            pt[name + "_speedup_agg"] = round(m["dense_agg"] / m[name + "_agg"], 2)
            pt[name + "_speedup_disagg"] = round(m["dense_disagg"] / m[name + "_disagg"], 2)
            pt[name + "_speedup_pass_f32"] = round((m["dense_agg"] + m["dense_disagg"]) / m[name + "_pass_f32"], 2)
        pt["ms"] = {k: round(v, 4) for k, v in m.items()}
        T.fmm_geometry_destroy(geom)
        torch.cuda.empty_cache()
        log("sweep point: %s" % json.dumps(pt))
        out["points"].append(pt)
    return out


def box_grid_pass(T, torch, geom, h, lay, w, ar, x32, g32, F32, V32, tucker_ms, pass_bytes):
    """The FP32 pass with the spectra on the K x K x K box grid: F and G are
    [2][K][K][K][N_dir] tensors, the aggregation also writes zero on the empty boxes.
    Checks that the groups' fibres and V equal the group-compact pass bit for bit, and
    restores the compact layout (uploads C64 again into the same arena)."""
    G, nd = lay.n_groups, lay.n_dir
    K, boxes = T.fmm_geometry_boxes(geom)
    nbox = K ** 3
    T.fmm_tucker_set_box_grid(h, (K, K, K), boxes)
    try:
        _, nbytes = T.fmm_tucker_storage_bytes(h, T.FMM_C64)
        # the header grows by the list of empty-box rows
        gar = ar if nbytes <= ar.numel() else torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        T.fmm_tucker_upload(h, T.FMM_C64, gar)
        bidx = torch.from_numpy(boxes).to("cuda")
        Gg = torch.zeros((2, nbox, nd), dtype=torch.complex64, device="cuda")
        Gg[:, bidx] = g32.transpose(0, 1)          # input construction: each group's G in its box
        Fg = torch.empty((2, nbox, nd), dtype=torch.complex64, device="cuda")
        Vg = torch.empty_like(V32)
        s = torch.cuda.Stream()
        with torch.cuda.stream(s):
            T.fmm_graph_capture(h, T.FMM_C64, 1, x32, Fg, Gg, Vg, s)
        torch.cuda.synchronize()
        for _ in range(3):
            T.fmm_graph_launch(h, s)
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(10)]
        for a, b in evs:
            a.record(s)
            T.fmm_graph_launch(h, s)
            b.record(s)
        torch.cuda.synchronize()
        ms = float(np.mean([a.elapsed_time(b) for a, b in evs]))
        same = bool(torch.equal(Fg[:, bidx].transpose(0, 1), F32) and torch.equal(Vg, V32))
        empty = torch.ones(nbox, dtype=torch.bool, device="cuda")
        empty[bidx] = False
        zeros_ok = bool((Fg[:, empty] == 0).all())
        zero_bytes = 2 * (nbox - G) * nd * 8
        rep = {"boxes": [K, K, K], "n_boxes": nbox, "pass_ms": round(ms, 4),
               "GBps": round((pass_bytes + zero_bytes) / (ms * 1e-3) / 1e9, 1),
               "zero_fill_bytes": zero_bytes, "overhead_vs_compact": round(ms / tucker_ms - 1.0, 4),
               "fibres_and_V_equal_compact": same, "empty_boxes_zero": zeros_ok}
        log("box grid: %s" % rep)
        return rep
    finally:
        T.fmm_tucker_set_box_grid(h, None, None)
        T.fmm_tucker_upload(h, T.FMM_C64, ar)


def svd_comparison(args, T, torch, lay, dense, w, x32, g32, tucker_ms, tucker_fac_bytes):
    """The comparison method: truncated SVD of every aggregation matrix at the same
    gamma (basis mode only), FP32 storage, the same single-RHS pass.  Reports its
    stored bytes and pass time beside the Tucker model's (Table III compares the two
    by memory).  Returns the report and the outputs for the oracle check."""
    G, nd = lay.n_groups, lay.n_dir
    t0 = time.time()
    hs = T.fmm_farfield_compress_svd(lay, dense, 0, G, w.gamma)
    t_c = time.time() - t0
    try:
        rs = T.fmm_tucker_ranks(hs, G)
        fbytes, nbytes = T.fmm_tucker_storage_bytes(hs, T.FMM_C64)
        ar = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        T.fmm_tucker_upload(hs, T.FMM_C64, ar)
        F = torch.empty((G, 2, nd), dtype=torch.complex64, device="cuda")
        V = torch.empty(lay.n_basis, dtype=torch.complex64, device="cuda")
        s = torch.cuda.Stream()
        with torch.cuda.stream(s):
            T.fmm_graph_capture(hs, T.FMM_C64, 1, x32, F, g32, V, s)
        torch.cuda.synchronize()
        for _ in range(3):
            T.fmm_graph_launch(hs, s)
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(10)]
        for a, b in evs:
            a.record(s)
            T.fmm_graph_launch(hs, s)
            b.record(s)
        torch.cuda.synchronize()
        ms = float(np.mean([a.elapsed_time(b) for a, b in evs]))
        b_stage, fac = svd_stage_bytes(rs, lay.offsets, w.n_theta, w.n_phi, 8)
        assert fac == fbytes, (fac, fbytes)
        gbs = 2 * b_stage / (ms * 1e-3) / 1e9
        rep = {"compress_s": round(t_c, 2), "r_beta_mean": round(float(rs[..., 2].mean()), 2),
               "factors_MB_f32": round(fbytes / 2 ** 20, 1),
               "tucker_factors_MB_f32": round(tucker_fac_bytes / 2 ** 20, 1),
               "memory_ratio_svd_over_tucker": round(fbytes / tucker_fac_bytes, 3),
               "pass_ms": round(ms, 4), "pass_GBps": round(gbs, 1),
               "time_ratio_svd_over_tucker": round(ms / tucker_ms, 3)}
        log("svd comparison: %s" % rep)
        return rep, (F.cpu().numpy(), V.cpu().numpy())
    finally:
        T.fmm_tucker_destroy(hs)


def multi_rhs(args, T, torch, synth, h, geom, lay, ranks, w, sample):
    """Multi-RHS pass (aggregation of x [N][R] + disaggregation of G [G][2][N_dir][R])
    per precision: autotuned, captured in a graph, replayed.  x holds R plane-wave
    excitations (eq. (2), directions uniform on the sphere, theta-polarised) computed by
    the library; G holds seeded complex-Gaussian incoming spectra.  Returns the report
    and the sampled outputs for the oracle check."""
    R = args.nrhs
    N, G, nd = lay.n_basis, lay.n_groups, lay.n_dir
    khat, epol = synth.planewaves(synth.rng(w.seeds.get("x", 0) + 200), R)
    gs = synth.complex_normal(synth.rng(w.seeds.get("g", 1) + 100), (G, 2, nd, R))
    dev = {}
    rep = {"nrhs": R, "inputs": "x: %d plane-wave excitations (eq. (2)); G: complex Gaussian" % R,
           "precisions": {}}
    outs = {"khat": khat, "epol": epol, "g": {g: gs[g] for g in sample}}
    s = torch.cuda.Stream()
    for name in [p for p in args.mrhs_precs.split(",") if p]:
        prec = MRHS_PRECS[name]
        dt = torch.complex128 if prec == 0 else torch.complex64
        if dt not in dev:
            dev.clear()   # one dtype's buffers at a time
            torch.cuda.empty_cache()
            xd = torch.empty((N, R), dtype=dt, device="cuda")
            T.fmm_planewave_excitation(geom, khat, epol, T.FMM_C128 if prec == 0 else T.FMM_C64, xd)
            dev[dt] = (xd, torch.from_numpy(gs).to("cuda", dt),
                       torch.empty((G, 2, nd, R), dtype=dt, device="cuda"),
                       torch.empty((N, R), dtype=dt, device="cuda"))
        xd, gd, F, V = dev[dt]
        es = 16 if prec == 0 else 8
        b_stage, fac = tucker_stage_bytes(ranks, lay.offsets, w.n_theta, w.n_phi, es)
        pass_bytes = 2 * (fac + R * (b_stage - fac))
        pass_flops = 2 * tucker_stage_flops(ranks, lay.offsets, w.n_theta, w.n_phi, R)
        _, nbytes = T.fmm_tucker_storage_bytes(h, prec)
        ar = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        T.fmm_tucker_upload(h, prec, ar)
        tuned = None if args.no_tune else T.fmm_tucker_tune(h, prec, R, xd, F, gd, V)
        with torch.cuda.stream(s):
            T.fmm_graph_capture(h, prec, R, xd, F, gd, V, s)
        torch.cuda.synchronize()
        for _ in range(2):
            T.fmm_graph_launch(h, s)
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
               for _ in range(args.mrhs_steps)]
        for a, b in evs:
            a.record(s)
            T.fmm_graph_launch(h, s)
            b.record(s)
        torch.cuda.synchronize()
        ms = float(np.median([a.elapsed_time(b) for a, b in evs]))
        tf = pass_flops / (ms * 1e-3) / 1e12
        gbs = pass_bytes / (ms * 1e-3) / 1e9
        r = {"pass_ms": round(ms, 4), "ms_per_rhs": round(ms / R, 5), "pass_bytes": pass_bytes,
             "pass_flops": pass_flops, "GBps": round(gbs, 1), "TFLOPs": round(tf, 2),
             "hbm_frac": round(gbs / HBM_PEAK_GBS, 4), "tuned": tuned}
        if prec == 0:
            r["fp64_frac"] = round(tf / 78.6, 4)
        elif prec == 1:
            r["mfma_frac_fp32"] = round(tf / 157.3, 4)
        else:
            issued = {2: 3, 3: 6}[prec]
            r["mfma_issued_TFLOPs_bf16"] = round(tf * issued, 1)
            r["mfma_frac_bf16"] = round(tf * issued / 2500.0, 4)
        rep["precisions"][name] = r
        log("multi-RHS %s R=%d: %.3f ms/pass, %.1f GB/s, %.1f TFLOP/s, tuned %s" % (name, R, ms, gbs, tf, tuned))
        outs[name] = sample_outputs(F, V, sample, lay.offsets)
        del ar
    return rep, outs


def oracle_checks(args, w, verts, tris, lay, x, gin, F32h, V32h, F64h, V64h, sample, stored, mr_out=None,
                  svd_out=None, extra=None):
    """Errors of the GPU outputs on the sampled groups against the oracle, and the
    oracle's own throughput.  Two kinds, relative L2 over the sample:
      rel_err_vs_oracle      end to end: against the dense products with the far-fields
                             of eq. (4) (the compression error included);
      arith_err_vs_oracle    arithmetic only: against the oracle's Tucker chain (Fig.
                             2(b) / 3(b)) on the factors as the arena stores them and
                             on the inputs as the path takes them."""
    from oracle import geometry as geo
    from oracle import farfield as ff
    from oracle import hosvd as H
    from oracle import products as pr
    from oracle import excitation as ex
    import synth

    P = geo.Problem(verts, tris, w.origin, w.box, w.boxes_per_axis, w.n_theta, w.n_phi)
    assert np.array_equal(P.offsets, lay.offsets)
    nb = P.group_sizes()
    off = P.offsets
    blocks = {}
    for i, g in enumerate(sample):
        blocks[g] = ff.farfield_group(P, g)
        if (i + 1) % 8 == 0 or i + 1 == len(sample):
            log("oracle: far-fields of %d of %d sampled groups" % (i + 1, len(sample)))
    c64 = lambda a: np.asarray(a).astype(np.complex64).astype(np.complex128)   # noqa: E731

    def err(got_by_g, ref_by_g):
        """(agg, disagg) relative L2 over the sample; entries are (F_g, V_g) pairs."""
        return tuple(float(pr.rel_err(np.concatenate([np.ravel(got_by_g[g][k]) for g in sample]),
                                      np.concatenate([np.ravel(ref_by_g[g][k]) for g in sample])))
                     for k in (0, 1))

    def dense_ref(xx, gg, blk=blocks):
        return {g: (pr.dense_aggregate(blk[g], xx[g]), pr.dense_disaggregate(blk[g], gg[g])) for g in sample}

    def tucker_ref(facs, xx, gg):
        return {g: (pr.tucker_aggregate(facs[g], xx[g]), pr.tucker_disaggregate(facs[g], gg[g])) for g in sample}

    e2e, arith = {}, {}

    def put(table, name, pair):
        table[name + "_agg"], table[name + "_disagg"] = pair

    xg = {g: x[off[g]:off[g + 1]] for g in sample}
    gg = {g: gin[g] for g in sample}
    ref1 = dense_ref(xg, gg)
    got32 = {g: (F32h[g], V32h[off[g]:off[g + 1]]) for g in sample}
    put(e2e, "tucker_f32", err(got32, ref1))
    put(arith, "tucker_f32", err(got32, tucker_ref(stored["c64"], {g: c64(v) for g, v in xg.items()},
                                                   {g: c64(v) for g, v in gg.items()})))
    if F64h is not None:
        put(e2e, "dense_f64", err({g: (F64h[g], V64h[off[g]:off[g + 1]]) for g in sample}, ref1))
    if svd_out is not None:
        put(e2e, "svd_f32", err({g: (svd_out[0][g], svd_out[1][off[g]:off[g + 1]]) for g in sample}, ref1))
    extra = extra or {}
    if "tucker_f64" in extra:
        put(e2e, "tucker_f64", err(extra["tucker_f64"], ref1))
        put(arith, "tucker_f64", err(extra["tucker_f64"], tucker_ref(stored["c128"], xg, gg)))
    if "gamma_1e-4_f32" in extra:
        outs, facs = extra["gamma_1e-4_f32"]
        put(e2e, "gamma_1e-4_f32", err(outs, ref1))
        put(arith, "gamma_1e-4_f32", err(outs, tucker_ref(facs, {g: c64(v) for g, v in xg.items()},
                                                          {g: c64(v) for g, v in gg.items()})))
    if "grid_29x58" in extra:
        o = extra["grid_29x58"]
        wg = o["w"]
        Pg = geo.Problem(verts, tris, wg.origin, wg.box, wg.boxes_per_axis, wg.n_theta, wg.n_phi)
        bg = {g: ff.farfield_group(Pg, g) for g in sample}
        xg2 = {g: o["x"][off[g]:off[g + 1]] for g in sample}
        gg2 = {g: o["gin"][g] for g in sample}
        r2 = dense_ref(xg2, gg2, bg)
        put(e2e, "grid_29x58_tucker_f32", err(o["f32"], r2))
        put(e2e, "grid_29x58_dense_f64", err(o["f64_dense"], r2))
        put(arith, "grid_29x58_tucker_f32", err(o["f32"], tucker_ref(o["stored"], {g: c64(v) for g, v in xg2.items()},
                                                                     {g: c64(v) for g, v in gg2.items()})))
    if mr_out:
        xs = {g: ex.planewave_excitation(P, mr_out["khat"], mr_out["epol"], rows=np.arange(off[g], off[g + 1]))
              for g in sample}
        gs = mr_out["g"]
        rR = dense_ref(xs, gs)
        r64 = tucker_ref(stored["c128"], xs, gs)
        r32 = tucker_ref(stored["c64"], {g: c64(v) for g, v in xs.items()}, gs)
        for name in [k for k in mr_out if k not in ("khat", "epol", "g")]:
            put(e2e, "mrhs_%s" % name, err(mr_out[name], rR))
            put(arith, "mrhs_%s" % name, err(mr_out[name], r64 if name == "c128" else r32))
    out = {"rel_err_vs_oracle": e2e, "arith_err_vs_oracle": arith,
           "rel_err_sample_groups": [int(g) for g in sample]}
    log("errors vs oracle (end to end): %s" % e2e)
    log("errors vs oracle (arithmetic only): %s" % arith)
    if args.cpu_seconds <= 0:
        return out

    # Oracle throughput.  The sampled groups alone (tens of MB) would sit in the host's
    # last-level cache, so the timing sample is a contiguous run of groups whose FP64
    # factors total >= 2 GB, with seeded random factors of the ranks the oracle's own
    # HOSVD gives on the sampled groups (values do not change the arithmetic).
    rk = []
    for g in sample:
        for a in range(2):
            rk.append(H.hosvd(H.tensorize(blocks[g], a), w.gamma)[0].shape)
        log("cpu baseline: oracle HOSVD ranks of group %d: %s" % (g, rk[-2:]))
    rk = np.array(rk)
    rt_m, rp_m = int(round(rk[:, 0].mean())), int(round(rk[:, 1].mean()))
    rb_frac = float(np.mean(rk[:, 2] / np.repeat(nb[sample], 2)))
    frng = synth.rng(5)
    tgroups, nbytes = [], 0
    for g in range(P.n_groups):
        n_b = int(nb[g])
        rb = max(1, min(n_b, int(round(rb_frac * n_b))))
        pair = []
        for a in range(2):
            core, ut, up, ub = synth.synthetic_tucker(frng, w.n_theta, w.n_phi, n_b, rt_m, rp_m, rb)
            pair.append((core, (ut, up, ub)))
            nbytes += 16 * (n_b * rb + w.n_theta * rt_m + w.n_phi * rp_m + rt_m * rp_m * rb + n_b +
                            w.n_theta * w.n_phi)
        tgroups.append((g, pair))
        if nbytes >= 2e9:
            break
    nbytes *= 2   # aggregation and disaggregation each read the factors once

    def timed_passes(budget):
        reps, t0 = 0, time.perf_counter()
        while True:
            for g, pair in tgroups:
                lo, hi = int(P.offsets[g]), int(P.offsets[g + 1])
                pr.tucker_aggregate(pair, x[lo:hi])
                pr.tucker_disaggregate(pair, gin[g])
            reps += 1
            if time.perf_counter() - t0 > budget:
                return reps, (time.perf_counter() - t0) / reps

    reps, dt = timed_passes(args.cpu_seconds)
    try:
        from threadpoolctl import threadpool_info
        cores = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:
        cores = os.cpu_count()
    out["cpu_baseline"] = {"value": round(nbytes / dt / 1e9, 3), "unit": "GB/s", "cores": int(cores),
                           "kind": "oracle",
                           "sample": "FP64 Tucker aggregation+disaggregation over groups 0..%d (%.2f GB of "
                                     "factors, ranks %d/%d/%.2f*n_beta from the oracle's HOSVD of the sampled "
                                     "groups), %d passes in %.1f s" %
                                     (tgroups[-1][0], nbytes / 2 / 1e9, rt_m, rp_m, rb_frac, reps, reps * dt)}
    log("cpu baseline: %s" % out["cpu_baseline"])
    # the same sample on one BLAS thread
    try:
        from threadpoolctl import threadpool_limits
    except ImportError:
        threadpool_limits = None
    if threadpool_limits is not None:
        with threadpool_limits(limits=1):
            reps1, dt1 = timed_passes(args.cpu_seconds / 2)
        out["cpu_baseline_1thread"] = {"value": round(nbytes / dt1 / 1e9, 3), "unit": "GB/s", "cores": 1,
                                       "kind": "oracle", "passes": reps1}
        log("cpu baseline, one thread: %s" % out["cpu_baseline_1thread"])
    out["host_cpu_count"] = os.cpu_count()
    return out


if __name__ == "__main__":
    main()
