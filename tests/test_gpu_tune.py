"""The autotuner on the GPU: every tile (compiled shape x runtime level) of
both operators matches the FP64 oracle; km_tune picks one, later calls with
tile = -1 use it (bit-identical to passing it), and a fresh process reading
the persisted cache (KM_TUNE_CACHE) gets the same tile for the same class."""
import os
import subprocess
import sys

import numpy as np
import pytest
import torch

from paper_1204_1225_amd import survey

pytestmark = pytest.mark.gpu
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def ops():
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    from paper_1204_1225_amd import _lib, ops

    _lib.load()
    return ops


def rel_l2(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / max(np.linalg.norm(b), 1e-300))


@pytest.mark.parametrize("prec,tol", [("extended", 1e-5), ("fp32", 5e-5)])
def test_every_tile_level_matches_oracle(ops, oracle_lib, prec, tol):
    # 90 depths: one partial depth chunk for the 8-slot shapes; extended time
    # at 1e-5 (its errors are near 1e-7, so a wrong tile stands out), float32
    # time at its derived bound
    p = survey.make_random(61, n_traces=180, n_t=420, nx=19, ny=4, nz=90, n_bins=3, dz=10.0)
    dp = ops.to_device(p, prec=prec)
    ref = oracle_lib.migrate(p)
    m = survey.bandlimited_image(p, 62)
    ref_d = oracle_lib.demigrate(p, m)
    mt = torch.from_numpy(m).cuda()
    worst = 0.0
    for tile in ops.tiles(0, dp):
        e = rel_l2(ops.migrate(dp, tile=tile).cpu().numpy(), ref)
        worst = max(worst, e)
        assert e <= tol, tile
    for tile in ops.tiles(1):
        e = rel_l2(ops.demigrate(dp, mt, tile=tile).cpu().numpy(), ref_d)
        worst = max(worst, e)
        assert e <= tol, tile
    print(f"{prec}: {len(ops.tiles(0, dp))} migrate and {len(ops.tiles(1))} demigrate tiles, "
          f"worst rel L2 {worst:.3e}")
    assert len(ops.tiles(0, dp)) > ops.tile_count(0) and len(ops.tiles(1)) > ops.tile_count(1)
    assert len(ops.tiles(0)) > len(ops.tiles(0, dp))  # the 16-bit staging levels need 16-bit traces


@pytest.mark.parametrize("kind", ["plain", "table", "ltable"])
def test_tune_pick_persist_reload(ops, oracle_lib, tmp_path, kind):
    path = str(tmp_path / "tune.json")
    os.environ["KM_TUNE_CACHE"] = path
    try:
        p = survey.make_random(63, n_traces=150, n_t=380, nx=17, ny=3, nz=70, n_bins=2, dz=10.0)
        if kind == "table":
            p = survey.with_curved_ray_table(p, dh=7.5)
        if kind == "ltable":
            p = survey.with_lateral_tables(p, survey.lateral_v0(1500.0, 0.3, -0.2, 1000.0, 2000.0), 0.5, 960.0,
                                           1970.0, 60.0, 40.0, 3, 3, dh=7.5, amplitude=True)
        # the extended time keeps the oracle check at 1e-5 on this geometry
        # (the float32 time's adjoint sits near 1.1e-5 here)
        dp = ops.to_device(p, prec="extended")
        img = torch.empty(dp.image_shape, device="cuda")
        t0, ms0 = ops.tune(0, dp, img, reps=1)
        m = torch.from_numpy(survey.bandlimited_image(p, 64)).cuda()
        out = torch.empty((dp.n_traces, dp.n_t), device="cuda")
        t1, ms1 = ops.tune(1, dp, m, traces_out=out, reps=1)
        print(f"{kind}: tuned migrate tile {t0} ({ms0:.3f} ms), demigrate tile {t1} ({ms1:.3f} ms)")
        assert ops.tune_lookup(0, dp) == t0 and ops.tune_lookup(1, dp) == t1
        # tile -1 takes the tuned tile: the same bits as passing it (the
        # adjoint's float64 atomics add in no fixed order: to an ulp or so)
        assert torch.equal(ops.migrate(dp), ops.migrate(dp, tile=t0))
        a, b = ops.demigrate(dp, m), ops.demigrate(dp, m, tile=t1)
        assert float((a - b).abs().max()) <= 2.0 ** -22 * float(a.abs().max())
        assert rel_l2(ops.migrate(dp).cpu().numpy(), oracle_lib.migrate(p)) <= 1e-5
        assert rel_l2(ops.demigrate(dp, m).cpu().numpy(), oracle_lib.demigrate(p, m.cpu().numpy())) <= 1e-5
        # a fresh process reads the file and finds the same tiles for the class
        kind_id = {"plain": 0, "table": 1, "ltable": 3}[kind]
        code = (f"import sys; sys.path.insert(0, {ROOT!r})\n"
                "from paper_1204_1225_amd import _lib\n"
                "lib = _lib.load()\n"
                f"print(lib.km_tune_lookup(0, 0, {kind_id}, 1, {dp.nz}, {dp.n_t}), "
                f"lib.km_tune_lookup(1, 0, {kind_id}, 1, {dp.nz}, {dp.n_t}))\n")
        r = subprocess.run([sys.executable, "-c", code], env=dict(os.environ), capture_output=True, text=True,
                           timeout=120)
        assert r.returncode == 0, r.stderr
        assert r.stdout.split()[-2:] == [str(t0), str(t1)]
    finally:
        os.environ.pop("KM_TUNE_CACHE", None)


def test_tune_covers_16bit_staging_for_16bit_traces(ops, oracle_lib, tmp_path):
    # km_tune on bf16 traces with float32 time searches the 16-bit staging
    # levels too; the tile it records is used by tile = -1 and matches the
    # oracle on the dequantised samples.
    os.environ["KM_TUNE_CACHE"] = str(tmp_path / "tune.json")
    try:
        p = survey.make_random(65, n_traces=150, n_t=380, nx=17, ny=3, nz=70, n_bins=2, dz=10.0)
        dp = ops.to_device(p, dtype="bf16")
        assert len(ops.tiles(0, dp)) == ops.tile_count(0) * ops.tile_levels(0)
        _, _, deq = survey.quantise(p.data, "bf16")
        img = torch.empty(dp.image_shape, device="cuda")
        t0, ms0 = ops.tune(0, dp, img, reps=1)
        print(f"bf16: tuned migrate tile {t0} ({ms0:.3f} ms), {ops.tile_describe(0, t0)}")
        assert ops.tune_lookup(0, dp) == t0
        assert torch.equal(ops.migrate(dp), ops.migrate(dp, tile=t0))
        assert rel_l2(ops.migrate(dp).cpu().numpy(), oracle_lib.migrate(p, deq)) <= 1e-5
    finally:
        os.environ.pop("KM_TUNE_CACHE", None)
