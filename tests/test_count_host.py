"""The library's exact host pair counter (km_count_contributions_host, Eq. (2))
against the FP64 oracle's counts: integer equality on ragged random problems
(with and without t_first, records too short for every pair), the 2D
constant-velocity line, exact-time record-end cases, an aperture table that is
not monotone in depth, and every thread count.  Host code only: no GPU."""
import dataclasses

import numpy as np
import pytest

from paper_1204_1225_amd import ops, survey

RAGGED = [
    # seed, n_traces, n_t, nx, ny, nz, n_bins, t_first
    (21, 301, 257, 13, 7, 37, 4, 0.0),
    (22, 97, 600, 70, 1, 300, 3, 0.0),
    (23, 64, 131, 5, 5, 16, 2, 0.05),
    (24, 33, 90, 1, 1, 1, 1, 0.0),
    (25, 120, 250, 17, 3, 90, 3, -0.02),  # short record: many pairs past its end
    (26, 200, 150, 9, 9, 50, 5, 0.2),     # t_first late: pairs before the record start
]


@pytest.mark.parametrize("case", RAGGED, ids=lambda c: f"seed{c[0]}")
def test_host_count_equals_oracle(oracle_lib, case):
    seed, n, nt, nx, ny, nz, nb, tf = case
    p = survey.make_random(seed, n_traces=n, n_t=nt, nx=nx, ny=ny, nz=nz, n_bins=nb, dz=10.0, t_first=tf,
                           data=None)
    assert ops.count_host(p) == oracle_lib.count(p)


def test_host_count_short_records_differ():
    for seed, nt, tf in [(25, 250, -0.02), (26, 150, 0.2)]:
        p = survey.make_random(seed, n_traces=120, n_t=nt, nx=17, ny=3, nz=90, n_bins=3, dz=10.0, t_first=tf,
                               data=None)
        na, ne = ops.count_host(p)
        assert 0.1 * na < ne < 0.9 * na


def test_host_count_line2d(oracle_lib):
    p = survey.make_line2d(1)
    assert ops.count_host(p) == oracle_lib.count(p)


def test_host_count_threads_agree():
    p = survey.make_random(22, n_traces=97, n_t=600, nx=70, ny=1, nz=300, n_bins=3, dz=10.0, data=None)
    ref = ops.count_host(p, n_threads=1)
    for n in (2, 3, 8, 0):
        assert ops.count_host(p, n_threads=n) == ref


def test_host_count_exact_record_ends(oracle_lib):
    # zero-offset trace over depths 512 + k m, v = 1024 m/s, dt = 1/256 s:
    # u = 256 + k/2 - t_first/dt exactly (k = 0..15)
    from tests.test_oracle_pins import exact_time_problem

    for n_t, tf, eff in [(260, 0.0, 8), (261, 0.0, 10), (256, 0.0, 0), (1000, 258.0 / 256.0, 13)]:
        p = exact_time_problem(n_t, tf)
        assert ops.count_host(p) == oracle_lib.count(p) == (16, eff)


def test_host_count_non_monotone_aperture(oracle_lib):
    p = survey.make_random(27, n_traces=80, n_t=200, nx=11, ny=4, nz=60, n_bins=2, dz=10.0, data=None)
    r2 = p.r2.copy()
    r2[20:30] = r2[20:30][::-1] * 0.5  # a dip in the aperture with depth
    q = dataclasses.replace(p, r2=r2)
    assert np.any(np.diff(r2) < 0)
    assert ops.count_host(q) == oracle_lib.count(q)


def test_host_count_empty_and_errors():
    from paper_1204_1225_amd._lib import KM_E_INVALID, KirchhoffError

    p = survey.make_random(28, n_traces=10, n_t=50, nx=3, ny=1, nz=5, n_bins=1, dz=10.0, data=None)
    assert ops.count_host(dataclasses.replace(p, n_bins=0)) == (0, 0)
    with pytest.raises(KirchhoffError) as e:
        ops.count_host(dataclasses.replace(p, dt=0.0))
    assert e.value.status == KM_E_INVALID
