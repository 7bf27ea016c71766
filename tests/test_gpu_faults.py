"""Error paths and repeatability on the GPU.

Injected launch failures (KM_FAULT_INJECT=launch): the operators report
KM_E_HIP with a message, run nothing and leave their outputs untouched, and
the next call without injection works and gives the usual result.  Repeat
runs: migrate is bitwise repeatable (every accumulator belongs to one lane);
demigrate adds float64 LDS atomics in no fixed order, so two runs agree to
the float32 rounding of the float64 sums."""
import numpy as np
import pytest
import torch

from paper_1204_1225_amd import survey

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ops():
    from paper_1204_1225_amd import _lib, ops

    _lib.load()
    return ops


@pytest.fixture(scope="module")
def problem(ops):
    p = survey.make_random(95, n_traces=160, n_t=400, nx=13, ny=4, nz=60, n_bins=2, dz=10.0)
    return p, ops.to_device(p)


def test_injected_launch_failure_leaves_outputs(ops, problem, monkeypatch):
    from paper_1204_1225_amd._lib import KM_E_HIP, KirchhoffError

    p, dp = problem
    ref_img = ops.migrate(dp)
    m = torch.from_numpy(survey.bandlimited_image(p, 96)).cuda()
    ref_d = ops.demigrate(dp, m)
    img = torch.full(dp.image_shape, float("nan"), device="cuda")
    out = torch.full((dp.n_traces, dp.n_t), float("nan"), device="cuda")
    monkeypatch.setenv("KM_FAULT_INJECT", "launch")
    with pytest.raises(KirchhoffError) as e1:
        ops.migrate(dp, image=img)
    with pytest.raises(KirchhoffError) as e2:
        ops.demigrate(dp, m, out=out)
    with pytest.raises(KirchhoffError) as e3:
        ops.dot_f64(m, m)
    torch.cuda.synchronize()
    assert e1.value.status == e2.value.status == e3.value.status == KM_E_HIP
    assert "injected" in str(e1.value)
    assert torch.isnan(img).all() and torch.isnan(out).all()
    monkeypatch.delenv("KM_FAULT_INJECT")
    assert torch.equal(ops.migrate(dp, image=img), ref_img)
    d = ops.demigrate(dp, m, out=out)
    assert float(torch.linalg.norm(d - ref_d) / torch.linalg.norm(ref_d)) <= 1e-7


def test_injected_failure_in_batch_run(ops, problem, monkeypatch):
    from paper_1204_1225_amd._lib import KM_E_HIP, KirchhoffError

    p, dp = problem
    img = torch.full(dp.image_shape, float("nan"), device="cuda")
    b = ops.Batch([dp], [img], tile=2)
    try:
        monkeypatch.setenv("KM_FAULT_INJECT", "launch")
        with pytest.raises(KirchhoffError) as e:
            b.run()
        torch.cuda.synchronize()
        assert e.value.status == KM_E_HIP and torch.isnan(img).all()
        monkeypatch.delenv("KM_FAULT_INJECT")
        b.run()
        torch.cuda.synchronize()
        assert torch.equal(img, ops.migrate(dp, tile=2))
    finally:
        b.close()


def test_repeat_runs(ops, problem):
    p, dp = problem
    for tile in range(ops.tile_count(0)):
        assert torch.equal(ops.migrate(dp, tile=tile), ops.migrate(dp, tile=tile)), tile
    m = torch.from_numpy(survey.random_image(p, 97)).cuda()
    for tile in range(ops.tile_count(1)):
        a, b = ops.demigrate(dp, m, tile=tile), ops.demigrate(dp, m, tile=tile)
        diff = (a - b).abs()
        # float64 sums in another order, rounded to float32: at most an ulp or so of each sample
        assert float(diff.max()) <= 2.0 ** -22 * float(a.abs().max()), tile
