"""GPU parity of the trace pre-filter (km_trace_filter) against the FP64
oracle (oracle/trace_filter.py), its adjoint identity, and the rho-filtered
migration of the flat-reflector line against the oracle chain."""
import numpy as np
import pytest
import torch

from oracle import trace_filter as tf
from paper_1204_1225_amd import survey

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ops():
    from paper_1204_1225_amd import _lib, ops

    _lib.load()
    return ops


CASES = [(7, 300, 65, 32), (3, 1500, 65, 32), (5, 37, 9, 0), (4, 50, 9, 8), (2, 10, 40, 17), (1, 1, 1, 0),
         (3, 700, 257, 100), (6, 2001, 33, 16)]


@pytest.mark.parametrize("n,ns,K,c", CASES)
@pytest.mark.parametrize("adjoint", [False, True])
def test_filter_parity(ops, n, ns, K, c, adjoint):
    rng = np.random.default_rng(n * 1000 + ns + K)
    x = rng.standard_normal((n, ns)).astype(np.float32)
    h = rng.standard_normal(K).astype(np.float32)
    got = ops.trace_filter(torch.from_numpy(x).cuda(), torch.from_numpy(h).cuda(), c, adjoint=adjoint).cpu().numpy()
    ref = (tf.adjoint if adjoint else tf.forward)(x, h, c)
    scale = np.abs(h).sum() * np.abs(x).max()
    assert np.abs(got - ref).max() <= 1e-6 * scale


def test_filter_strided_and_in_place(ops):
    rng = np.random.default_rng(5)
    base = torch.from_numpy(rng.standard_normal((9, 520)).astype(np.float32)).cuda()
    x = base[:, 7:507]  # stride 520, 500 samples
    taps, c = survey.rho_filter_taps(0.004, 0.5)
    h = torch.from_numpy(taps).cuda()
    ref = tf.forward(x.cpu().numpy(), taps, c)
    got = ops.trace_filter(x, h, c).cpu().numpy()
    assert np.abs(got - ref).max() <= 1e-6 * np.abs(ref).max() * 10
    y = x.clone()
    ops.trace_filter(y, h, c, out=y)
    assert torch.equal(y.cpu(), torch.from_numpy(got))


def test_filter_dot_product(ops):
    rng = np.random.default_rng(11)
    taps, c = survey.rho_filter_taps(0.004, 0.5)
    h = torch.from_numpy(taps).cuda()
    x = torch.from_numpy(rng.standard_normal((64, 1500)).astype(np.float32)).cuda()
    y = torch.from_numpy(rng.standard_normal((64, 1500)).astype(np.float32)).cuda()
    lhs = float(ops.dot_f64(ops.trace_filter(x, h, c), y))
    rhs = float(ops.dot_f64(x, ops.trace_filter(y, h, c, adjoint=True)))
    assert abs(lhs - rhs) <= 1e-6 * max(abs(lhs), abs(rhs))


def test_rho_filtered_migration(ops, oracle_lib):
    p = survey.make_flat_line()
    taps, c = survey.rho_filter_taps(p.dt, 0.5)
    dp = ops.to_device(p)
    d = ops.trace_filter(dp.data, torch.from_numpy(taps).cuda(), c)
    img = ops.migrate(dp, data=d).cpu().numpy().astype(np.float64)
    ref = oracle_lib.migrate(p, data=tf.forward(p.data, taps, c))
    assert np.linalg.norm(img - ref) <= 1e-5 * np.linalg.norm(ref)
