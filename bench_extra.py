"""Measurements of the non-headline workloads (each returns one JSON-able dict).

Imported by bench.py only (next to it, outside the library package: the
cpu_baseline and parity legs here run the FP64 oracle).

survey3d_ext: the 3D survey with the extended-precision total time
    (KM_TIME_EXTENDED): both operators' throughput next to the float32 time on
    the same GPU, and each one's sampled parity against the oracle.

survey3d_bf16 / survey3d_f16: the 3D survey with 16-bit trace storage
    (per-trace scale), migrate-only throughput next to float32 on the same GPU,
    and the time of every tile that keeps the samples as 16-bit values in LDS.
line2d_vz: the 2D v(z) adjoint pair (61 440 traces x 2000 samples, image
    1024 x 800 in 32 bins): migrate and demigrate throughput and the float32
    dot-product test.
batch: 64 uneven 2D lines migrated by one persistent hipGraph-captured launch
    against 64 separate launches (same tile shape, chosen by the tuner on the
    largest line), images compared bit for bit.
aa: the 3D survey migrated and demigrated with the anti-alias triangle filter:
    throughput of both operators and a sampled parity against the oracle.
table: the 3D survey migrated and demigrated with curved-ray traveltime
    tables (v = 1500 + 0.5 z, h every 10 m) instead of the RMS double square
    root: throughput of both operators next to the table-gather rate, and with
    amplitude tables (W = A_s A_r).
ltable: the same with laterally varying tables (v0 from 1420 to 1580 m/s
    across the image, curved rays under each node of a 9 x 9 grid at 400 m):
    throughput of both operators next to the table-gather rate.
filter: the rho pre-filter (anti-causal derivative, 65 taps) forward and
    transposed over the 3D survey's 200 000 x 1500 traces: HBM bandwidth
    against 8 TB/s and the FP64 oracle timed on sampled traces.
cig: the offset stack and the common-image-gather moveout of the migrated 3D
    survey image (16 x 256 x 256 x 400): HBM bandwidth of both kernels against
    8 TB/s, and the FP64 oracle timed on a sample of image columns.
"""
from __future__ import annotations

import dataclasses
import os
import time

import numpy as np
import torch

from paper_1204_1225_amd import ops, survey

PEAK_VALU_LANE_OPS = 256 * 64 * 2.4e9  # unpacked VALU issue: 256 CUs x 64 lanes/clk x 2.4 GHz
# L2 read bandwidth: 16 channels x 128 B/clk per XCD, 8 XCDs, 2.4 GHz
PEAK_L2_BYTES = 16 * 128 * 8 * 2.4e9


def host_cpus():
    return len(os.sched_getaffinity(0))


def _time(fn, steps, warmup):
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(steps):
        fn()
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / steps


def _survey16(kind, steps, warmup, dev):
    p = survey.make_survey3d(seed=2, device=dev)
    dp = ops.to_device(p, dev)
    n_ap, _ = ops.count(dp)
    host = dp.data.cpu().numpy()
    bits, sig, _ = survey.quantise(host, kind)
    dq = dp.with_data(torch.from_numpy(bits.view(np.int16)).to(dev), torch.from_numpy(sig).to(dev), kind)
    img = torch.empty(dp.image_shape, device=dev)
    ms32 = _time(lambda: ops.migrate(dp, image=img), steps, warmup)
    ms16 = _time(lambda: ops.migrate(dq, image=img), steps, warmup)
    # the 16-bit staging tiles (samples kept as 16-bit values in LDS), one timed
    # call each after one untimed
    lds16 = {}
    for t in ops.tiles(0, dq):
        if ops.tile_describe(0, t)["lds16"]:
            lds16[t] = _time(lambda: ops.migrate(dq, image=img, tile=t), 1, 1)
    best = min(lds16, key=lds16.get)
    return {"workload": f"survey3d_{kind}", "metric": "G contributions/s (migrate)", "pairs_in_aperture": n_ap,
            "ms_f32": round(ms32, 3), f"ms_{kind}": round(ms16, 3),
            "gcps_f32": round(n_ap / ms32 / 1e6, 3), f"gcps_{kind}": round(n_ap / ms16 / 1e6, 3),
            "trace_bytes_f32": int(host.nbytes), f"trace_bytes_{kind}": int(bits.nbytes + sig.nbytes),
            "lds16_tiles_ms": {str(t): round(v, 3) for t, v in lds16.items()},
            f"ms_{kind}_lds16_best": round(lds16[best], 3), "lds16_best_tile": best}


def _line2d_vz(steps, warmup, dev):
    p = survey.make_line2d_vz()
    dp = ops.to_device(p, dev)
    n_ap, n_eff = ops.count(dp)
    d = torch.from_numpy(survey.random_data(p, 41)).to(dev)
    m = torch.from_numpy(survey.random_image(p, 42)).to(dev)
    img = torch.empty(dp.image_shape, device=dev)
    out = torch.empty((dp.n_traces, dp.n_t), device=dev)
    ms_m = _time(lambda: ops.migrate(dp, data=d, image=img, dtype="f32"), steps, warmup)
    ms_d = _time(lambda: ops.demigrate(dp, m, out=out), steps, warmup)
    lhs = float(ops.dot_f64(img, m))
    rhs = float(ops.dot_f64(d, out))
    return {"workload": "line2d_vz", "metric": "G contributions/s (migrate, demigrate)", "pairs_in_aperture": n_ap,
            "ms_migrate": round(ms_m, 3), "ms_demigrate": round(ms_d, 3),
            "gcps_migrate": round(n_ap / ms_m / 1e6, 3), "gcps_demigrate": round(n_ap / ms_d / 1e6, 3),
            "dot_test_rel": abs(lhs - rhs) / max(abs(lhs), abs(rhs))}


def _batch(steps, warmup, dev):
    shapes = survey.batch_line_shapes(5)
    gen = torch.Generator(device=dev).manual_seed(5)
    dps, t0 = [], time.time()
    for i, sh in enumerate(shapes):
        p = survey.make_batch_line(sh, i)
        dp = ops.to_device(p, dev)
        dps.append(dp.with_data(torch.randn((dp.n_traces, dp.n_t), generator=gen, device=dev)))
    n_ap = sum(ops.count(dp)[0] for dp in dps)
    big = max(range(len(dps)), key=lambda k: dps[k].n_traces * dps[k].nx * dps[k].nz)
    tile, _ = ops.tune(0, dps[big], torch.empty(dps[big].image_shape, device=dev), reps=1)
    gen_s = time.time() - t0
    sep = [torch.empty(dp.image_shape, device=dev) for dp in dps]
    bat = [torch.empty(dp.image_shape, device=dev) for dp in dps]

    def separate():
        for dp, im in zip(dps, sep):
            ops.migrate(dp, image=im, tile=tile)

    ms_sep = _time(separate, steps, warmup)
    tc = time.time()
    b = ops.Batch(dps, bat, tile=tile)
    create_s = time.time() - tc
    ms_bat = _time(b.run, steps, warmup)
    n_items, n_wg = b.info()
    same = all(torch.equal(x, y) for x, y in zip(sep, bat))
    b.close()
    return {"workload": "batch", "metric": "G contributions/s (migrate)", "lines": len(dps),
            "pairs_in_aperture": n_ap, "tile": tile, "ms_separate_launches": round(ms_sep, 3),
            "ms_batched_graph": round(ms_bat, 3), "gcps_separate": round(n_ap / ms_sep / 1e6, 3),
            "gcps_batched": round(n_ap / ms_bat / 1e6, 3), "work_items": n_items, "persistent_workgroups": n_wg,
            "bitwise_equal": bool(same), "create_s": round(create_s, 2), "setup_s": round(gen_s, 1),
            "trace_bytes": int(sum(dp.data.numel() * 4 for dp in dps))}


HBM_PEAK = 8.0e12  # bytes/s


def _cig(steps, warmup, dev, max_lag=12):
    from oracle import cig as ocig

    p = survey.make_survey3d(seed=2, device=dev)
    dp = ops.to_device(p, dev)
    img = ops.migrate(dp)
    hb_np = survey.bin_offsets(p).astype(np.float32)
    hb = torch.from_numpy(hb_np).to(dev)
    nb, ny, nx, nz = img.shape
    stack = torch.empty((ny, nx, nz), device=dev)
    ms_stack = _time(lambda: ops.stack_offsets(img, out=stack), steps, warmup)
    res = {}

    def moveout():
        res["out"] = ops.cig_moveout(img, hb, max_lag=max_lag)

    ms_cig = _time(moveout, steps, warmup)
    n_pts = ny * nx * nz
    bytes_stack = (nb + 1) * n_pts * 4
    bytes_cig = (nb + 1) * n_pts * 4 + 2 * nb * ny * nx * 4 + ny * nx * 4
    fma = ny * nx * nb * (2 * max_lag + 1) * nz
    # oracle on a sample of columns, and the GPU values there
    rng = np.random.default_rng(0)
    n_s = 512
    iy, ix = rng.integers(0, ny, n_s), rng.integers(0, nx, n_s)
    sub = img[:, iy, ix, :].cpu().numpy()[:, :, None, :]
    t0 = time.perf_counter()
    o_stack, o_shift, _, _ = ocig.cig_moveout(sub, hb_np.astype(np.float64), max_lag)
    t_cpu = time.perf_counter() - t0
    g_shift = res["out"][1][:, iy, ix].cpu().numpy()
    C = ocig.correlations(sub, max_lag)
    Cs = np.sort(C, axis=-1)
    clear = ((Cs[..., -1] - Cs[..., -2]) > 1e-9 * (np.abs(C).max(axis=-1) + 1e-300))[:, :, 0]
    err = float(np.abs(g_shift - o_shift[:, :, 0])[clear].max())
    return {"workload": "cig", "metric": "HBM GB/s (offset stack; CIG moveout)", "image": [nb, ny, nx, nz],
            "max_lag": max_lag, "ms_stack": round(ms_stack, 4), "ms_moveout": round(ms_cig, 4),
            "roofline_stack": {"bound": "hbm", "achieved": round(bytes_stack / ms_stack / 1e6, 1),
                               "peak": HBM_PEAK / 1e9, "unit": "GB/s",
                               "frac": round(bytes_stack / ms_stack * 1e3 / HBM_PEAK, 4)},
            "roofline_moveout": {"bound": "hbm", "achieved": round(bytes_cig / ms_cig / 1e6, 1),
                                 "peak": HBM_PEAK / 1e9, "unit": "GB/s",
                                 "frac": round(bytes_cig / ms_cig * 1e3 / HBM_PEAK, 4),
                                 "fp64_fma_tflops": round(2 * fma / ms_cig / 1e9, 3)},
            "cpu_baseline": {"value": round(n_s / t_cpu, 1), "unit": "columns/s", "cores": 1, "kind": "oracle",
                             "sample": f"moveout of {n_s} random columns x {nb} bins x {nz} depths, lag +-{max_lag}"},
            "gpu_columns_per_s": round(ny * nx / ms_cig * 1e3, 1),
            "parity_sample_max_shift_err": err, "parity_sample_clear_frac": round(float(clear.mean()), 4),
            "host_cpus": host_cpus()}


def _filter(steps, warmup, dev):
    from oracle import trace_filter as otf

    p = survey.make_survey3d(seed=2, device=dev)
    dp = ops.to_device(p, dev)
    taps_np, c = survey.rho_filter_taps(p.dt, 1.0, half_len=32)
    taps = torch.from_numpy(taps_np).to(dev)
    x = dp.data
    y = torch.empty_like(x)
    ms_f = _time(lambda: ops.trace_filter(x, taps, c, out=y), steps, warmup)
    z = torch.empty_like(x)
    ms_a = _time(lambda: ops.trace_filter(y, taps, c, adjoint=True, out=z), steps, warmup)
    nbytes = 2 * x.numel() * 4
    fma = x.numel() * taps.numel()
    rng = np.random.default_rng(0)
    idx = np.sort(rng.choice(x.shape[0], 512, replace=False))
    sample = x[idx].cpu().numpy()
    t0 = time.perf_counter()
    ref = otf.forward(sample, taps_np, c)
    t_cpu = time.perf_counter() - t0
    got = y[idx].cpu().numpy()
    err = float(np.abs(got - ref).max() / (np.abs(ref).max() + 1e-30))
    return {"workload": "filter", "metric": "HBM GB/s (rho pre-filter, forward; transpose)",
            "traces": list(x.shape), "taps": int(taps.numel()), "ms_forward": round(ms_f, 4),
            "ms_adjoint": round(ms_a, 4),
            "roofline": {"bound": "hbm", "achieved": round(nbytes / ms_f / 1e6, 1), "peak": HBM_PEAK / 1e9,
                         "unit": "GB/s", "frac": round(nbytes / ms_f * 1e3 / HBM_PEAK, 4),
                         "fp32_fma_tflops": round(2 * fma / ms_f / 1e9, 3)},
            "cpu_baseline": {"value": round(512 / t_cpu, 1), "unit": "traces/s", "cores": 1, "kind": "oracle",
                             "sample": "forward filter of 512 random traces x 1500 samples, 65 taps"},
            "gpu_traces_per_s": round(x.shape[0] / ms_f * 1e3, 1), "parity_sample_max_rel_err": err}


def _table(steps, warmup, dev):
    p = survey.make_survey3d(seed=2, device=dev)
    pt = survey.with_curved_ray_table(p, dh=10.0)
    dp = ops.to_device(pt, dev)
    n_ap, _ = ops.count(dp, aperture_only=True)
    img = torch.empty(dp.image_shape, device=dev)
    out = torch.empty((dp.n_traces, dp.n_t), device=dev)
    ms_m = _time(lambda: ops.migrate(dp, image=img), steps, warmup)
    ms_d = _time(lambda: ops.demigrate(dp, img, out=out), steps, warmup)
    # the same with amplitude tables (W = A_s A_r: 4 more table reads per pair)
    da = ops.to_device(survey.with_curved_ray_table(p, dh=10.0, amplitude=True), dev)
    ms_ma = _time(lambda: ops.migrate(da, image=img), steps, warmup)
    ms_da = _time(lambda: ops.demigrate(da, img, out=out), steps, warmup)
    # Two resources per pair once the legs are hoisted.  The table gathers:
    # 4 float32 values (16 bytes: two rows of each leg at the lane's depth), read
    # through the L2 (the tables are 565 KB, resident in every XCD's 4 MB L2).
    # The VALU: per leg 2 widenings + 1 float64 FMA (6), sum + scale + 2 clamps
    # (4), index, fraction and its narrowing (3), row address, interpolation (2)
    # and accumulate (1) = 17 full-rate lane-ops.
    c_k = 17
    table_bytes = 16
    dom = max(ms_m, ms_d)
    gather = n_ap * table_bytes / (dom * 1e-3)
    valu = n_ap * c_k / (dom * 1e-3)
    return {"workload": "table", "metric": "G contributions/s (migrate, demigrate; curved-ray tables)",
            "pairs_in_aperture": n_ap, "table_shape": list(pt.ttab.shape),
            "ms_migrate": round(ms_m, 3), "ms_demigrate": round(ms_d, 3),
            "gcps_migrate": round(n_ap / ms_m / 1e6, 3), "gcps_demigrate": round(n_ap / ms_d / 1e6, 3),
            "step_gcps": round(2 * n_ap / (ms_m + ms_d) / 1e6, 3),
            "amplitudes": {"ms_migrate": round(ms_ma, 3), "ms_demigrate": round(ms_da, 3),
                           "step_gcps": round(2 * n_ap / (ms_ma + ms_da) / 1e6, 3), "bytes_per_pair": 32},
            "roofline": {"bound": "l2_gather", "achieved": round(gather / 1e12, 3),
                         "peak": round(PEAK_L2_BYTES / 1e12, 3), "unit": "TB/s",
                         "frac": round(gather / PEAK_L2_BYTES, 4), "bytes_per_pair": table_bytes,
                         "kernel": "migrate" if ms_m >= ms_d else "demigrate",
                         "co_bound": {"resource": "VALU", "ops_per_pair": c_k, "achieved": round(valu / 1e12, 3),
                                      "peak": round(PEAK_VALU_LANE_OPS / 1e12, 3), "unit": "T lane-ops/s",
                                      "frac": round(valu / PEAK_VALU_LANE_OPS, 4)}}}


def _ltable(steps, warmup, dev):
    p = survey.make_survey3d(seed=2, device=dev)
    pl = survey.with_survey3d_lateral_tables(p, dh=10.0)
    dp = ops.to_device(pl, dev)
    n_ap, _ = ops.count(dp, aperture_only=True)
    img = torch.empty(dp.image_shape, device=dev)
    out = torch.empty((dp.n_traces, dp.n_t), device=dev)
    ms_m = _time(lambda: ops.migrate(dp, image=img), steps, warmup)
    ms_d = _time(lambda: ops.demigrate(dp, img, out=out), steps, warmup)
    # Per pair 16 float32 table reads (64 bytes: two rows of each of the four
    # nodes around the column, per leg), through the L2 (the 81 node tables
    # are 45 MB in all; a workgroup's depth chunk touches four nodes' rows).
    # VALU: per node and leg one float32 difference, two widenings and one
    # float64 FMA (16 per leg), the x and y steps (3 float64 differences and 3
    # FMAs per leg), then sum + scale + 2 clamps (4), index, fraction and its
    # narrowing (3), row address, interpolation (2), accumulate (1) = 54.
    c_k = 54
    table_bytes = 64
    dom = max(ms_m, ms_d)
    gather = n_ap * table_bytes / (dom * 1e-3)
    valu = n_ap * c_k / (dom * 1e-3)
    return {"workload": "ltable", "metric": "G contributions/s (migrate, demigrate; laterally varying tables)",
            "pairs_in_aperture": n_ap, "table_shape": list(pl.ttab.shape), "node_grid": list(pl.tgrid),
            "ms_migrate": round(ms_m, 3), "ms_demigrate": round(ms_d, 3),
            "gcps_migrate": round(n_ap / ms_m / 1e6, 3), "gcps_demigrate": round(n_ap / ms_d / 1e6, 3),
            "step_gcps": round(2 * n_ap / (ms_m + ms_d) / 1e6, 3),
            "roofline": {"bound": "l2_gather", "achieved": round(gather / 1e12, 3),
                         "peak": round(PEAK_L2_BYTES / 1e12, 3), "unit": "TB/s",
                         "frac": round(gather / PEAK_L2_BYTES, 4), "bytes_per_pair": table_bytes,
                         "kernel": "migrate" if ms_m >= ms_d else "demigrate",
                         "co_bound": {"resource": "VALU", "ops_per_pair": c_k, "achieved": round(valu / 1e12, 3),
                                      "peak": round(PEAK_VALU_LANE_OPS / 1e12, 3), "unit": "T lane-ops/s",
                                      "frac": round(valu / PEAK_VALU_LANE_OPS, 4)}}}


def _aa(steps, warmup, dev):
    """The 3D survey with the anti-alias triangle filter (dip over the 12.5 m
    image spacing in x and y, half-widths up to 8 samples)."""
    from oracle import migrate_points

    p = survey.make_survey3d(seed=2, device=dev)
    pa = dataclasses.replace(p, aa=(12.5, 12.5, 8))
    dp = ops.to_device(pa, dev)
    n_ap, _ = ops.count(dp, aperture_only=True)
    img = torch.empty(dp.image_shape, device=dev)
    out = torch.empty((dp.n_traces, dp.n_t), device=dev)
    ms_m = _time(lambda: ops.migrate(dp, image=img), steps, warmup)
    ms_d = _time(lambda: ops.demigrate(dp, img, out=out), steps, warmup)
    # full-rate lane-ops per pair: the square-root pair (10 plus 2 square roots;
    # its weight 1 / (a_s a_r) is the square of the product of the dip's two leg
    # reciprocals) and the filter: the dip (12: two legs' x and y slopes, the
    # weighted sum, clamp, floor and fraction, plus 2 reciprocals), the blend
    # weights (5), addresses (3), four float64 second differences (8), blend and
    # interpolation with widening and narrowing (8), less the plain
    # interpolation (1): 45 + 4 transcendentals
    t_fma, t_sqrt, t_rcp = ops.probe_issue(0), ops.probe_issue(1), ops.probe_issue(2)
    r = 0.5 * (t_sqrt + t_rcp) / t_fma
    c_k = 45 + 4 * r
    peak = PEAK_VALU_LANE_OPS
    dom = max(ms_m, ms_d)
    # sampled parity of the migrated image against the FP64 oracle
    rng = np.random.default_rng(0)
    host = dataclasses.replace(pa, data=dp.data.cpu().numpy())
    pts = np.stack([rng.integers(0, pa.n_bins, 64), rng.integers(0, len(pa.y), 64),
                    rng.integers(0, len(pa.x), 64), rng.integers(0, len(pa.z), 64)], 1).astype(np.int32)
    t0 = time.perf_counter()
    ref = migrate_points(host, pts)
    t_cpu = time.perf_counter() - t0
    got = img[pts[:, 0], pts[:, 1], pts[:, 2], pts[:, 3]].cpu().numpy().astype(np.float64)
    err = float(np.linalg.norm(got - ref) / max(np.linalg.norm(ref), 1e-300))
    from oracle import threads as oracle_threads
    return {"workload": "aa", "metric": "G contributions/s (migrate, demigrate; anti-alias triangle filter)",
            "pairs_in_aperture": n_ap, "aa": list(pa.aa),
            "ms_migrate": round(ms_m, 3), "ms_demigrate": round(ms_d, 3),
            "gcps_migrate": round(n_ap / ms_m / 1e6, 3), "gcps_demigrate": round(n_ap / ms_d / 1e6, 3),
            "step_gcps": round(2 * n_ap / (ms_m + ms_d) / 1e6, 3),
            "roofline": {"bound": "alu", "achieved": round(n_ap * c_k / (dom * 1e-3) / 1e12, 3),
                         "peak": round(peak / 1e12, 3), "unit": "T lane-ops/s",
                         "frac": round(n_ap * c_k / (dom * 1e-3) / peak, 4), "ops_per_pair": round(c_k, 3),
                         "kernel": "migrate" if ms_m >= ms_d else "demigrate"},
            "cpu_baseline": {"value": round(64 / t_cpu, 2), "unit": "image points/s", "cores": oracle_threads(),
                             "host_cpus": host_cpus(), "kind": "oracle",
                             "sample": "64 random image points against all traces of their bins"},
            "gpu_image_points_per_s": round(pa.n_bins * len(pa.y) * len(pa.x) * len(pa.z) / ms_m * 1e3, 1),
            "parity_sample_rel_l2": err}


def _ext(steps, warmup, dev):
    """The 3D survey with the extended-precision total time against the float32
    time: both operators, and 300 sampled image points of each against the
    oracle."""
    from oracle import migrate_points

    p = survey.make_survey3d(seed=2, device=dev)
    dp32 = ops.to_device(p, dev)
    dpx = dp32.with_precision("extended")
    n_ap, _ = ops.count(dp32)
    img = torch.empty(dp32.image_shape, device=dev)
    out = torch.empty((dp32.n_traces, dp32.n_t), device=dev)
    rng = np.random.default_rng(5)
    pts = np.stack([rng.integers(0, p.n_bins, 300), rng.integers(0, 256, 300), rng.integers(0, 256, 300),
                    rng.integers(0, 400, 300)], 1).astype(np.int32)
    host = dataclasses.replace(p, data=dp32.data.cpu().numpy())
    ref = migrate_points(host, pts)
    res = {}
    for name, dp in [("fp32", dp32), ("extended", dpx)]:
        ms_m = _time(lambda: ops.migrate(dp, image=img), steps, warmup)
        got = img[pts[:, 0], pts[:, 1], pts[:, 2], pts[:, 3]].double().cpu().numpy()
        ms_d = _time(lambda: ops.demigrate(dp, img, out=out), steps, warmup)
        res[name] = {"ms_migrate": round(ms_m, 3), "ms_demigrate": round(ms_d, 3),
                     "gcps_migrate": round(n_ap / ms_m / 1e6, 3), "gcps_demigrate": round(n_ap / ms_d / 1e6, 3),
                     "step_gcps": round(2 * n_ap / (ms_m + ms_d) / 1e6, 3),
                     "parity_sample_rel_l2": float(np.linalg.norm(got - ref) / np.linalg.norm(ref))}
    return {"workload": "survey3d_ext", "metric": "G contributions/s (migrate + adjoint), float32 vs extended time",
            "pairs_in_aperture": n_ap, **res}


def run(workload, steps, warmup, dev):
    if workload == "survey3d_ext":
        return _ext(steps, warmup, dev)
    if workload == "aa":
        return _aa(steps, warmup, dev)
    if workload == "table":
        return _table(steps, warmup, dev)
    if workload == "ltable":
        return _ltable(steps, warmup, dev)
    if workload == "filter":
        return _filter(steps, warmup, dev)
    if workload == "cig":
        return _cig(steps, warmup, dev)
    if workload in ("survey3d_bf16", "survey3d_f16"):
        return _survey16(workload.split("_")[1], steps, warmup, dev)
    if workload == "line2d_vz":
        return _line2d_vz(steps, warmup, dev)
    if workload == "batch":
        return _batch(steps, warmup, dev)
    raise ValueError(workload)
