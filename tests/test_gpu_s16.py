"""GPU parity of the 16-bit staging migrate kernels (tile levels 4 and 5:
KM_BF16 / KM_F16 traces staged in LDS as their 16-bit storage, widened and
scaled per sample read) against the FP64 oracle on the dequantised samples,
on every compiled shape: square-root times with both weights and t_first != 0,
curved-ray tables, lateral tables with amplitudes, and sampled points of the
full 3D survey in bfloat16; the staged-window edge cases (strided rows, one-
and two-sample records, 20000-sample records, whole-record fallback, short
records under a deep image).  With unit scales they give the float-staging
tiles' bits; a tuned 16-bit staging tile leaves the batched calls working."""
import dataclasses
import os

import numpy as np
import pytest
import torch

from paper_1204_1225_amd import survey

pytestmark = pytest.mark.gpu

CASES = [  # seed, traces, samples, nx, ny, nz, bins, t_first, weight
    (121, 160, 420, 19, 3, 70, 3, 0.0, survey.WEIGHT_COSCOS),
    (122, 120, 380, 13, 4, 45, 2, 0.04, survey.WEIGHT_UNIT),
    (123, 90, 333, 9, 5, 129, 2, -0.02, survey.WEIGHT_COSCOS),
]
KINDS = ["bf16", "f16"]


@pytest.fixture(scope="module")
def ops():
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    from paper_1204_1225_amd import _lib, ops

    _lib.load()
    return ops


def rel_l2(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / max(np.linalg.norm(b), 1e-300))


def s16_tiles(ops, dp):
    t = [x for x in ops.tiles(0, dp) if ops.tile_describe(0, x)["lds16"]]
    assert len(t) == 2 * ops.tile_count(0)
    return t


def problem(case):
    seed, n, nt, nx, ny, nz, nb, tf, w = case
    return survey.make_random(seed, n_traces=n, n_t=nt, nx=nx, ny=ny, nz=nz, n_bins=nb, dz=10.0, t_first=tf,
                              weight=w)


def check_every_s16_tile(ops, oracle_lib, p, kind, what):
    dp = ops.to_device(p, dtype=kind)
    _, _, deq = survey.quantise(p.data, kind)
    ref = oracle_lib.migrate(p, deq)
    worst = 0.0
    for tile in s16_tiles(ops, dp):
        e = rel_l2(ops.migrate(dp, tile=tile).cpu().numpy(), ref)
        worst = max(worst, e)
        assert e <= 1e-5, (what, kind, tile, e)
    print(f"{what} {kind}: worst rel L2 of the 16-bit staging tiles {worst:.3e}")


@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("case", CASES, ids=lambda c: f"seed{c[0]}")
def test_s16_sqrt_times_every_shape(ops, oracle_lib, case, kind):
    check_every_s16_tile(ops, oracle_lib, problem(case), kind, "square-root")


@pytest.mark.parametrize("kind", KINDS)
def test_s16_tables_every_shape(ops, oracle_lib, kind):
    p = problem(CASES[1])
    check_every_s16_tile(ops, oracle_lib, survey.with_curved_ray_table(p, dh=7.5), kind, "table")
    check_every_s16_tile(ops, oracle_lib, survey.with_curved_ray_table(p, dh=7.5, amplitude=True), kind,
                         "table amplitudes")
    pl = survey.with_lateral_tables(p, survey.lateral_v0(1500.0, 0.3, -0.2, 1000.0, 2000.0), 0.5, 960.0, 1970.0,
                                    60.0, 40.0, 3, 3, dh=7.5, amplitude=True)
    check_every_s16_tile(ops, oracle_lib, pl, kind, "lateral amplitudes")


@pytest.mark.parametrize("kind", KINDS)
def test_s16_unit_scales_give_the_float_staging_bits(ops, kind):
    # With scale 1 the widened samples are the staged floats, the scale factor
    # multiplies by 1 and the interpolation is the same FMA: bit for bit.
    # A NULL scale (no scale array) means 1 on both kinds of tile.
    for p in (problem(CASES[0]), survey.with_curved_ray_table(problem(CASES[2]), dh=7.5)):
        dp = ops.to_device(p, dtype=kind)
        dn = dp.with_data(dp.data, None, kind)
        dp = dp.with_data(dp.data, torch.ones_like(dp.scale), kind)
        for sh in range(ops.tile_count(0)):
            for lv_f, lv_s in ((0, 4), (3, 5)):
                a = ops.migrate(dp, tile=sh + 64 * lv_f)
                b = ops.migrate(dp, tile=sh + 64 * lv_s)
                assert torch.equal(a, b), (sh, lv_s)
                assert torch.equal(a, ops.migrate(dn, tile=sh + 64 * lv_f)), (sh, lv_f)
                assert torch.equal(b, ops.migrate(dn, tile=sh + 64 * lv_s)), (sh, lv_s)


def test_s16_survey3d_sampled(ops, oracle_lib):
    # The full survey in bfloat16 on both 16-bit staging levels of the
    # benchmark's migrate shape: 200 sampled image points against the oracle on
    # the dequantised samples.
    p = survey.make_survey3d(seed=2, device="cuda")
    dp = ops.to_device(p, "cuda", dtype="bf16")
    bits = dp.data.cpu().numpy().view(np.uint16)
    deq = (bits.astype(np.uint32) << 16).view(np.float32).astype(np.float64)
    deq *= dp.scale.cpu().numpy().astype(np.float64)[:, None]
    host = dataclasses.replace(p, data=deq)
    rng = np.random.default_rng(7)
    pts = np.stack([rng.integers(0, p.n_bins, 200), rng.integers(0, 256, 200), rng.integers(0, 256, 200),
                    rng.integers(0, 400, 200)], 1).astype(np.int32)
    ref = oracle_lib.migrate_points(host, pts)
    for lv in (4, 5):
        img = ops.migrate(dp, tile=2 + 64 * lv)
        got = img[pts[:, 0], pts[:, 1], pts[:, 2], pts[:, 3]].double().cpu().numpy()
        e = rel_l2(got, ref)
        print(f"survey bf16 level {lv}: sampled rel L2 {e:.3e}")
        assert e <= 1e-5, lv
        del img


def test_tuned_s16_tile_leaves_batches_working(ops, oracle_lib, tmp_path):
    # A tuned 16-bit staging tile is used by single calls; the batched calls of
    # the same class take its float-staging level instead.
    from paper_1204_1225_amd import _lib

    os.environ["KM_TUNE_CACHE"] = str(tmp_path / "tune.json")
    try:
        p = problem(CASES[0])
        dp = ops.to_device(p, dtype="bf16")
        lib = _lib.load()
        tile = 2 + 64 * 5
        assert lib.km_tune_record(0, _lib.KM_BF16, ops.KIND_DSR, 0, dp.nz, dp.n_t, tile, 1.0) == _lib.KM_OK
        assert ops.tune_lookup(0, dp) == tile
        assert torch.equal(ops.migrate(dp), ops.migrate(dp, tile=tile))
        imgs = [torch.zeros(dp.image_shape, device="cuda")]
        ops.Batch([dp], imgs).run()
        torch.cuda.synchronize()
        assert torch.equal(imgs[0], ops.migrate(dp, tile=2 + 64 * 3))
    finally:
        del os.environ["KM_TUNE_CACHE"]


def check_s16(ops, oracle_lib, p, kind, what, tol=1e-5, data=None, scale=None):
    """Every 16-bit staging tile against the oracle on the dequantised samples."""
    dp = ops.to_device(p, dtype=kind)
    _, _, deq = survey.quantise(p.data, kind)
    ref = oracle_lib.migrate(p, deq)
    for tile in s16_tiles(ops, dp):
        img = ops.migrate(dp, tile=tile, data=data, dtype=kind if data is not None else None,
                          scale=scale).cpu().numpy()
        e = rel_l2(img, ref)
        assert e <= tol, (what, kind, tile, e)
    return ref


@pytest.mark.parametrize("kind", KINDS)
def test_s16_edges(ops, oracle_lib, kind):
    # strided 16-bit rows (stride 256 for 200 samples)
    p = survey.make_random(124, n_traces=80, n_t=200, nx=10, ny=3, nz=50, n_bins=2, dz=10.0)
    dp = ops.to_device(p, dtype=kind)
    wide = torch.zeros((p.n_traces, 256), dtype=torch.int16, device="cuda")
    wide[:, :200] = dp.data
    check_s16(ops, oracle_lib, p, kind, "strided", data=wide[:, :200], scale=dp.scale)
    # one- and two-sample records
    for nt in (1, 2):
        r = survey.make_random(125 + nt, n_traces=50, n_t=nt, nx=6, ny=1, nz=30, n_bins=1, dz=2.0, spread=0.0)
        r.data[:] = 1.0
        check_s16(ops, oracle_lib, r, kind, f"n_t = {nt}")
    # 20000-sample records: few staged traces per block
    q = survey.make_random(127, n_traces=12, n_t=20000, nx=8, ny=1, nz=40, n_bins=1, dz=50.0, dt=0.001)
    check_s16(ops, oracle_lib, q, kind, "long record")
    check_s16(ops, oracle_lib, survey.with_curved_ray_table(q, dh=25.0), kind, "long record, table")


@pytest.mark.parametrize("kind", KINDS)
def test_s16_staged_window_edges(ops, oracle_lib, kind):
    # s2 < 0 on some depths: whole-record windows; a short record under a deep
    # image: most times past the record end
    p = survey.make_random(128, n_traces=300, n_t=500, nx=24, ny=3, nz=90, n_bins=2, dz=10.0, spread=400.0)
    s2 = p.s2.copy()
    s2[30:60] *= -0.01
    ref = check_s16(ops, oracle_lib, dataclasses.replace(p, s2=s2), kind, "s2 < 0")
    assert np.count_nonzero(ref[:, :, :, 30:60]) > 0
    r = survey.make_random(129, n_traces=200, n_t=60, nx=20, ny=2, nz=200, n_bins=3, dz=10.0)
    ref = check_s16(ops, oracle_lib, r, kind, "short record")
    assert np.count_nonzero(ref) > 0 and np.all(ref[:, :, :, 150:] == 0)
