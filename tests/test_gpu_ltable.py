"""GPU parity of the laterally varying table path (kirchhoff_migrate_ltable /
kirchhoff_demigrate_ltable: one curved-ray table per node of a coarse lateral
grid, trilinear over image x, y and h) against the FP64 oracle's lateral
path: ragged random cases on every tile (node grids covering the image,
clamped at its edges, a single node row for a 2D line), band-limited and
white inputs in both time precisions, t_first != 0, equal node tables against
the laterally invariant kernels, the dot-product test, and sampled points of
the full 3D survey in the launch configuration of the benchmark."""
import dataclasses

import numpy as np
import pytest
import torch

from paper_1204_1225_amd import survey

pytestmark = pytest.mark.gpu

# seed, traces, samples, nx, ny, nz, bins, t_first, node grid (gx0, gy0, gdx, gdy, n_gx, n_gy)
CASES = [
    (81, 130, 400, 19, 1, 70, 3, 0.0, (880.0, 0.0, 60.0, 1.0, 5, 1)),
    (82, 90, 350, 11, 5, 45, 2, 0.0, (930.0, 1960.0, 35.0, 25.0, 5, 4)),
    (83, 60, 500, 7, 3, 33, 2, 0.05, (1000.0, 1990.0, 20.0, 40.0, 2, 2)),
    (84, 150, 300, 17, 1, 129, 4, -0.02, (800.0, 0.0, 150.0, 1.0, 4, 1)),
]


@pytest.fixture(scope="module")
def ops():
    from paper_1204_1225_amd import _lib, ops

    _lib.load()
    return ops


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def ltable_problem(case, data="bandlimited"):
    seed, n, nt, nx, ny, nz, nb, tf, (gx0, gy0, gdx, gdy, n_gx, n_gy) = case
    p = survey.make_random(seed, n_traces=n, n_t=nt, nx=nx, ny=ny, nz=nz, n_bins=nb, dz=10.0, t_first=tf,
                           data=data)
    v0_at = survey.lateral_v0(1500.0, 0.4, -0.3, 1000.0, 2000.0 if ny > 1 else 0.0)
    return survey.with_lateral_tables(p, v0_at, 0.5, gx0, gy0, gdx, gdy, n_gx, n_gy, dh=7.5)


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"seed{c[0]}")
def test_ltable_migrate_parity_all_tiles(ops, oracle_lib, case):
    p = ltable_problem(case)
    ref = oracle_lib.migrate(p)
    for prec in ("fp32", "extended"):
        dp = ops.to_device(p, prec=prec)
        for tile in range(ops.tile_count(0)):
            img = ops.migrate(dp, tile=tile).cpu().numpy()
            e = rel_l2(img, ref)
            assert e <= 1e-5, (prec, tile, e)


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"seed{c[0]}")
def test_ltable_demigrate_parity_all_tiles(ops, oracle_lib, case):
    # as the invariant tables: band-limited images meet 1e-5 with float32
    # legs, white images 1e-5 with extended legs and 5e-5 with float32 legs
    p = ltable_problem(case, data=None)
    for make, prec, tol in [(survey.bandlimited_image, "fp32", 1e-5), (survey.random_image, "extended", 1e-5),
                            (survey.random_image, "fp32", 5e-5)]:
        dp = ops.to_device(p, prec=prec)
        m = make(p, case[0] + 1)
        ref = oracle_lib.demigrate(p, m)
        mt = torch.from_numpy(m).cuda()
        for tile in range(ops.tile_count(1)):
            d = ops.demigrate(dp, mt, tile=tile).cpu().numpy()
            e = rel_l2(d, ref)
            assert e <= tol, (make.__name__, prec, tile, e)


@pytest.mark.parametrize("case", CASES[1:3], ids=lambda c: f"seed{c[0]}")
def test_ltable_white_extended(ops, oracle_lib, case):
    p = ltable_problem(case, data="normal")
    dp = ops.to_device(p, prec="extended")
    ref = oracle_lib.migrate(p)
    for tile in range(ops.tile_count(0)):
        e = rel_l2(ops.migrate(dp, tile=tile).cpu().numpy(), ref)
        print(f"lateral white seed{case[0]} migrate tile{tile}: {e:.3e}")
        assert e <= 1e-5, tile


def test_ltable_equal_nodes_match_invariant_kernels_bitwise(ops):
    # every node holding the same table: the lateral kernels add exact zeros
    # to the invariant kernels' times, so both give the same bits on one tile
    case = CASES[1]
    seed, n, nt, nx, ny, nz, nb, tf, _ = case
    p = survey.make_random(seed, n_traces=n, n_t=nt, nx=nx, ny=ny, nz=nz, n_bins=nb, dz=10.0, t_first=tf)
    pt = survey.with_curved_ray_table(p, dh=7.5)
    pl = dataclasses.replace(pt, ttab=np.broadcast_to(pt.ttab, (4, 5) + pt.ttab.shape).copy(),
                             tgrid=(930.0, 1960.0, 35.0, 25.0))
    for prec in ("fp32", "extended"):
        dt_, dl = ops.to_device(pt, prec=prec), ops.to_device(pl, prec=prec)
        m = torch.from_numpy(survey.random_image(pt, 7)).cuda()
        for tile in (0, 2):
            assert torch.equal(ops.migrate(dt_, tile=tile), ops.migrate(dl, tile=tile)), (prec, tile)
        for tile in (1, 3):
            a, b = ops.demigrate(dt_, m, tile=tile), ops.demigrate(dl, m, tile=tile)
            # the float64 LDS atomics add in no fixed order: equal to the
            # summation rounding
            assert rel_l2(a.cpu().numpy(), b.cpu().numpy()) <= 1e-7, (prec, tile)


def test_ltable_dot_product(ops):
    p = ltable_problem(CASES[1])
    dp = ops.to_device(p)
    d = torch.from_numpy(survey.random_data(p, 43)).cuda()
    m = torch.from_numpy(survey.random_image(p, 44)).cuda()
    md = ops.migrate(dp, data=d, dtype="f32")
    lhs = float(ops.dot_f64(md, m))
    rhs = float(ops.dot_f64(d, ops.demigrate(dp, m)))
    scale = float(torch.linalg.norm(md)) * float(torch.linalg.norm(m))
    assert abs(lhs - rhs) <= 1e-8 * scale


def test_ltable_survey3d_sampled(ops, oracle_lib):
    # The full 3D survey with its laterally varying tables (9 x 9 nodes, 400 m),
    # in the benchmark's launch configuration: 200 sampled image points and 16
    # sampled adjoint samples against the oracle (tolerances as the invariant
    # tables').
    p = survey.make_survey3d(seed=2, device="cuda")
    pl = survey.with_survey3d_lateral_tables(p, dh=10.0)
    rng = np.random.default_rng(6)
    pts = np.stack([rng.integers(0, p.n_bins, 200), rng.integers(0, 256, 200), rng.integers(0, 256, 200),
                    rng.integers(0, 400, 200)], 1).astype(np.int32)
    smp = np.stack([rng.integers(0, p.n_traces, 16), rng.integers(0, p.n_t, 16)], 1)
    host = None
    for prec, tol_d in [("fp32", 2e-5), ("extended", 1e-5)]:
        dp = ops.to_device(pl, "cuda", prec=prec)
        if host is None:
            host = dataclasses.replace(pl, data=dp.data.cpu().numpy())
            ref = oracle_lib.migrate_points(host, pts)
        img = ops.migrate(dp)
        got = img[pts[:, 0], pts[:, 1], pts[:, 2], pts[:, 3]].double().cpu().numpy()
        e = rel_l2(got, ref)
        print(f"lateral survey {prec}: migrate sample rel L2 {e:.3e}")
        assert e <= 1e-5, prec
        out = ops.demigrate(dp, img)
        ref_d = oracle_lib.demigrate_samples(host, img.cpu().numpy(), smp)
        got_d = out[smp[:, 0], smp[:, 1]].double().cpu().numpy()
        e = rel_l2(got_d, ref_d)
        print(f"lateral survey {prec}: adjoint sample rel L2 {e:.3e}")
        assert e <= tol_d, prec


@pytest.mark.parametrize("case", [CASES[1], CASES[3]], ids=lambda c: f"seed{c[0]}")
def test_ltable_amplitudes_all_tiles(ops, oracle_lib, case):
    # W = A_s A_r from each node's curved-ray amplitude table, interpolated
    # over (x, y, h) as the times are
    seed, n, nt, nx, ny, nz, nb, tf, (gx0, gy0, gdx, gdy, n_gx, n_gy) = case
    p = survey.make_random(seed, n_traces=n, n_t=nt, nx=nx, ny=ny, nz=nz, n_bins=nb, dz=10.0, t_first=tf)
    v0_at = survey.lateral_v0(1500.0, 0.4, -0.3, 1000.0, 2000.0 if ny > 1 else 0.0)
    p = survey.with_lateral_tables(p, v0_at, 0.5, gx0, gy0, gdx, gdy, n_gx, n_gy, dh=7.5, amplitude=True)
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
