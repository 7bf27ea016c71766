"""Pins of the offset-stack / moveout oracle (oracle/cig.py).

Nothing re-types the oracle's formulas: the stack is checked against the
migration of all traces in a single bin (Eq. (1) without the offset split),
the moveout measure against gathers whose displacements are known by
construction, and the whole chain (migration + measure) against the closed
form of the depth at which a constant-velocity migration with the wrong
velocity images a flat reflector (Introduction: reflector positioning across
offset images measures the velocity error).
"""
import numpy as np
import pytest

from oracle import cig
from paper_1204_1225_amd import survey


def test_stack_is_single_bin_migration(oracle_lib):
    p = survey.make_random(91, n_traces=120, n_t=250, nx=9, ny=3, nz=40, n_bins=4, dz=10.0, spread=300)
    img = oracle_lib.migrate(p)
    one = survey.dataclasses.replace(p, bin=np.zeros_like(p.bin), n_bins=1)
    ref = oracle_lib.migrate(one)[0]
    got = cig.stack(img)
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()


def gaussian_gathers(taus, nz=120, z0=60.0, sigma=4.0, ny=1, nx=1):
    z = np.arange(nz, dtype=np.float64)
    img = np.zeros((len(taus), ny, nx, nz))
    for b, t in enumerate(taus):
        img[b, :, :, :] = np.exp(-0.5 * ((z - z0 - t) / sigma) ** 2)
    return img


def test_identical_gathers_have_zero_shift():
    img = gaussian_gathers([0.0] * 6, nz=100, z0=47.3)
    _, shift, peak, curv = cig.cig_moveout(img, offsets=np.arange(6) * 100.0, max_lag=8)
    assert np.abs(shift).max() < 1e-12
    assert (peak > 0).all()
    assert np.abs(curv).max() < 1e-18


@pytest.mark.parametrize("taus", [[-1.6, -0.7, 0.0, 0.7, 1.6], [-3.0, -1.0, 1.0, 3.0], [-2.0, 2.0]])
def test_displaced_wavelets_are_recovered(taus):
    # The stack is symmetric about z0 when the displacements are, so bin b's
    # shift against it is its own displacement tau_b.
    img = gaussian_gathers(taus)
    _, shift, _, _ = cig.cig_moveout(img, offsets=np.zeros(len(taus)), max_lag=10)
    assert np.abs(shift[:, 0, 0] - np.asarray(taus)).max() < 0.05
    # integer lags of the unrefined maximum
    C = cig.correlations(img, 10)
    assert list(np.argmax(C[:, 0, 0], axis=1) - 10) == [int(np.rint(t)) for t in taus]


def test_curvature_of_parabolic_moveout():
    h = np.array([0.0, 200.0, 400.0, 600.0, 800.0])
    kappa = -4.0e-6  # samples per m^2
    taus = kappa * h ** 2  # the stack reference moves every bin alike; the slope is unaffected
    img = gaussian_gathers(list(taus), sigma=5.0)
    _, shift, _, curv = cig.cig_moveout(img, offsets=h, max_lag=10)
    assert curv[0, 0] == pytest.approx(kappa, rel=0.05)


def test_window_and_lag_limit():
    # A second event outside the window must not pull the measure; a lag at
    # the limit is reported unrefined.
    img = gaussian_gathers([0.0, 0.0], nz=200, z0=50.0)
    img[1, 0, 0, :] += gaussian_gathers([0.0], nz=200, z0=150.0)[0, 0, 0] * 3.0
    _, shift, _, _ = cig.cig_moveout(img, offsets=[0.0, 1.0], max_lag=5, z_lo=20, z_hi=90)
    assert np.abs(shift).max() < 1e-9
    far = gaussian_gathers([0.0, 9.0], nz=120, z0=60.0)
    _, shift, _, _ = cig.cig_moveout(far, offsets=[0.0, 1.0], max_lag=3)
    assert shift[1, 0, 0] == 3.0


@pytest.mark.parametrize("v_mig", [2000.0, 1900.0, 2100.0])
def test_flat_reflector_moveout(oracle_lib, v_mig):
    p = survey.make_flat_line(v_true=2000.0, v_mig=v_mig, z_reflector=800.0)
    img = oracle_lib.migrate(p)
    hb = survey.bin_offsets(p)
    z_lo, z_hi = 120, 190  # 605 .. 950 m
    _, shift, peak, curv = cig.cig_moveout(img, offsets=hb, max_lag=12, z_lo=z_lo, z_hi=z_hi)
    zb = np.array([cig.flat_reflector_depth(800.0, h, 2000.0, v_mig) for h in hb])
    dz = 5.0
    expect = (zb - zb[0]) / dz
    got = shift[:, 0, :] - shift[0:1, 0, :]
    assert (peak > 0).all()
    assert np.abs(got - expect[:, None]).max() < 0.1, (got.mean(1), expect)
    if v_mig == 2000.0:
        assert np.abs(curv).max() < 2e-7
    elif v_mig < 2000.0:
        assert (curv < -1e-6).all()
    else:
        assert (curv > 1e-6).all()
