"""GPU parity of the table-traveltime path (kirchhoff_migrate_table /
kirchhoff_demigrate_table, curved rays of v(z) = v0 + k z) against the FP64
oracle's table path: ragged random cases on every tile, t_first != 0, the
float32 dot-product test, the curved-ray diffractor line, and sampled points of
the full 3D survey in the launch configuration of the benchmark."""
import dataclasses

import numpy as np
import pytest
import torch

from paper_1204_1225_amd import survey

pytestmark = pytest.mark.gpu

CASES = [  # seed, traces, samples, nx, ny, nz, bins, t_first
    (71, 130, 400, 19, 1, 70, 3, 0.0),
    (72, 90, 350, 11, 5, 45, 2, 0.0),
    (73, 60, 500, 7, 3, 33, 2, 0.05),
    (74, 150, 300, 17, 1, 129, 4, -0.02),
]


@pytest.fixture(scope="module")
def ops():
    from paper_1204_1225_amd import _lib, ops

    _lib.load()
    return ops


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def table_problem(case):
    seed, n, nt, nx, ny, nz, nb, tf = case
    p = survey.make_random(seed, n_traces=n, n_t=nt, nx=nx, ny=ny, nz=nz, n_bins=nb, dz=10.0, t_first=tf)
    return survey.with_curved_ray_table(p, dh=7.5)


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"seed{c[0]}")
def test_table_migrate_parity_all_tiles(ops, oracle_lib, case):
    p = table_problem(case)
    ref = oracle_lib.migrate(p)
    dp = ops.to_device(p)
    for tile in range(ops.tile_count(0)):
        img = ops.migrate(dp, tile=tile).cpu().numpy()
        assert rel_l2(img, ref) <= 1e-5, tile


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"seed{c[0]}")
def test_table_demigrate_parity_all_tiles(ops, oracle_lib, case):
    # Band-limited images meet the float32 bar with float32 legs; an image that
    # is white in depth changes by O(1) per sample, so the float32 rounding of
    # the leg lengths alone gives about 1e-5 with float32 legs (the white-noise
    # bound of the double-square-root path, 5e-5, applies there), and the
    # extended legs meet 1e-5.
    p = table_problem(case)
    for make, prec, tol in [(survey.bandlimited_image, "fp32", 1e-5), (survey.random_image, "extended", 1e-5),
                            (survey.random_image, "fp32", 5e-5)]:
        dp = ops.to_device(p, prec=prec)
        m = make(p, case[0] + 1)
        ref = oracle_lib.demigrate(p, m)
        mt = torch.from_numpy(m).cuda()
        for tile in range(ops.tile_count(1)):
            d = ops.demigrate(dp, mt, tile=tile).cpu().numpy()
            assert rel_l2(d, ref) <= tol, (make.__name__, prec, tile)


def test_table_dot_product(ops):
    p = table_problem(CASES[0])
    dp = ops.to_device(p)
    d = torch.from_numpy(survey.random_data(p, 41)).cuda()
    m = torch.from_numpy(survey.random_image(p, 42)).cuda()
    lhs = float(ops.dot_f64(ops.migrate(dp, data=d, dtype="f32"), m))
    rhs = float(ops.dot_f64(d, ops.demigrate(dp, m)))
    scale = float(torch.linalg.norm(ops.migrate(dp, data=d, dtype="f32"))) * float(torch.linalg.norm(m))
    assert abs(lhs - rhs) <= 1e-8 * scale


def test_table_curved_diffractor(ops, oracle_lib):
    from tests.test_oracle_table import diffractor_line

    p = survey.with_curved_ray_table(diffractor_line(), dh=2.0)
    ref = oracle_lib.migrate(p)
    img = ops.migrate(ops.to_device(p)).cpu().numpy()
    assert rel_l2(img, ref) <= 1e-5


def test_table_survey3d_sampled(ops, oracle_lib):
    # Full survey with curved-ray tables, in the benchmark's launch
    # configuration: 200 sampled image points and 16 sampled trace samples of
    # the adjoint (of the migrated image) against the oracle.  The adjoint of
    # a migrated image adds, per output sample, pairs whose leg lengths round
    # differently in float32: 2e-5 with float32 legs, 1e-5 with extended legs.
    p = survey.make_survey3d(seed=2, device="cuda")
    pt = survey.with_curved_ray_table(p, dh=10.0)
    rng = np.random.default_rng(5)
    pts = np.stack([rng.integers(0, p.n_bins, 200), rng.integers(0, 256, 200), rng.integers(0, 256, 200),
                    rng.integers(0, 400, 200)], 1).astype(np.int32)
    smp = np.stack([rng.integers(0, p.n_traces, 16), rng.integers(0, p.n_t, 16)], 1)
    host = None
    for prec, tol_d in [("fp32", 2e-5), ("extended", 1e-5)]:
        dp = ops.to_device(pt, "cuda", prec=prec)
        if host is None:
            host = dataclasses_replace_data(pt, dp.data.cpu().numpy())
            ref = oracle_lib.migrate_points(host, pts)
        img = ops.migrate(dp)
        got = img[pts[:, 0], pts[:, 1], pts[:, 2], pts[:, 3]].double().cpu().numpy()
        assert rel_l2(got, ref) <= 1e-5, prec
        m = img.clone()
        out = ops.demigrate(dp, m)
        ref_d = oracle_lib.demigrate_samples(host, m.cpu().numpy(), smp)
        got_d = out[smp[:, 0], smp[:, 1]].double().cpu().numpy()
        print(f"table survey {prec}: adjoint sample rel L2 {rel_l2(got_d, ref_d):.3e}")
        assert rel_l2(got_d, ref_d) <= tol_d, prec


def dataclasses_replace_data(p, data):
    import dataclasses

    return dataclasses.replace(p, data=data)


def test_table_not_increasing_in_h_falls_back(ops, oracle_lib):
    # A table whose rows dip at some offsets and depths (times that fall with
    # h) still matches the oracle on every tile: migrate stages whole records
    # for tables and derives no window from the time's growth with h.
    p = table_problem(CASES[1])
    t = p.ttab.copy()
    t[3:6, 10:30] -= 0.02  # rows 3..5 fall below row 2 on these depths
    q = dataclasses.replace(p, ttab=t)
    assert np.any(np.diff(t, axis=0) < 0)
    ref = oracle_lib.migrate(q)
    dp = ops.to_device(q)
    for tile in range(ops.tile_count(0)):
        img = ops.migrate(dp, tile=tile).cpu().numpy()
        assert rel_l2(img, ref) <= 1e-5, tile


@pytest.mark.parametrize("case", CASES[1:3], ids=lambda c: f"seed{c[0]}")
def test_table_amplitudes_all_tiles(ops, oracle_lib, case):
    # W = A_s A_r from curved-ray amplitude tables (t0 / T^2 per leg)
    seed, n, nt, nx, ny, nz, nb, tf = case
    p = survey.make_random(seed, n_traces=n, n_t=nt, nx=nx, ny=ny, nz=nz, n_bins=nb, dz=10.0, t_first=tf)
    p = survey.with_curved_ray_table(p, dh=7.5, amplitude=True)
    ref = oracle_lib.migrate(p)
    m = survey.bandlimited_image(p, seed + 3)
    ref_d = oracle_lib.demigrate(p, m)
    mt = torch.from_numpy(m).cuda()
    for prec in ("fp32", "extended"):
        dp = ops.to_device(p, prec=prec)
        for tile in range(ops.tile_count(0)):
            e = rel_l2(ops.migrate(dp, tile=tile).cpu().numpy(), ref)
            assert e <= 1e-5, (prec, tile, e)
        for tile in range(ops.tile_count(1)):
            e = rel_l2(ops.demigrate(dp, mt, tile=tile).cpu().numpy(), ref_d)
            assert e <= 1e-5, (prec, tile, e)


def test_table_unit_amplitudes_are_bitwise_unit_weight(ops):
    p = table_problem(CASES[0])
    q = dataclasses.replace(p, tamp=np.ones_like(p.ttab))
    d0, d1 = ops.to_device(p), ops.to_device(q)
    m = torch.from_numpy(survey.random_image(p, 5)).cuda()
    for tile in range(ops.tile_count(0)):
        assert torch.equal(ops.migrate(d0, tile=tile), ops.migrate(d1, tile=tile)), tile
    for tile in range(ops.tile_count(1)):
        a, b = ops.demigrate(d0, m, tile=tile), ops.demigrate(d1, m, tile=tile)
        assert rel_l2(a.cpu().numpy(), b.cpu().numpy()) <= 1e-7, tile
