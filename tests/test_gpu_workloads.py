"""GPU checks at the workloads' full sizes, in the launch configurations the
benchmark uses: sampled image points and trace samples against the FP64
oracle (which evaluates them one by one), the adjoint pair, 16-bit storage
and the batched launch.  Each test prints what it measures."""
import time

import numpy as np
import pytest
import torch

from paper_1204_1225_amd import survey

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ops():
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    from paper_1204_1225_amd import _lib, ops

    _lib.load()
    return ops


def rel_l2(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.fixture(scope="module")
def survey3d(ops):
    t = time.time()
    p = survey.make_survey3d(seed=2, device="cuda")
    dp = ops.to_device(p, "cuda")
    torch.cuda.synchronize()
    print(f"survey3d generated in {time.time() - t:.1f} s")
    return p, dp


def _sample_points(p, n, seed):
    rng = np.random.default_rng(seed)
    return np.stack([rng.integers(0, p.n_bins, n), rng.integers(0, p.ny, n), rng.integers(0, p.nx, n),
                     rng.integers(0, p.nz, n)], 1).astype(np.int32)


def test_survey3d_sampled_parity(ops, oracle_lib, survey3d):
    p, dp = survey3d
    img = ops.migrate(dp)
    pts = _sample_points(p, 400, 7)
    host = dp.data.cpu().numpy()
    ref = oracle_lib.migrate_points(p, pts, data=host)
    got = img[tuple(torch.from_numpy(pts.T.astype(np.int64)).cuda())].double().cpu().numpy()
    e = rel_l2(got, ref)
    print(f"survey3d migrate, 400 sampled points: rel L2 {e:.3e}")
    assert e <= 1e-5
    # adjoint at sampled trace samples, input = the migrated image
    out = ops.demigrate(dp, img)
    rng = np.random.default_rng(8)
    smp = np.stack([rng.integers(0, p.n_traces, 24), rng.integers(200, p.n_t - 1, 24)], 1)
    ref_d = oracle_lib.demigrate_samples(p, img.cpu().numpy(), smp)
    got_d = out[smp[:, 0], smp[:, 1]].double().cpu().numpy()
    e_d = rel_l2(got_d, ref_d)
    print(f"survey3d demigrate, 24 sampled samples: rel L2 {e_d:.3e}")
    assert e_d <= 1e-5


# The 16-bit storage configuration's oracle sub-volume: columns ix, iy in
# [96, 160), depths [150, 250), every offset bin (65 536 columns x 100 depths).
C3_IX = (96, 160)
C3_IZ = (150, 250)


@pytest.fixture(scope="module")
def c3_subvolume(oracle_lib, survey3d):
    p, dp = survey3d
    host = dp.data.cpu().numpy()
    cols = np.array([(b, iy, ix) for b in range(p.n_bins) for iy in range(*C3_IX) for ix in range(*C3_IX)],
                    np.int32)
    t = time.time()
    ref_o = oracle_lib.migrate_window(p, cols, *C3_IZ, data=host)
    print(f"oracle on the 64 x 64 x 100 sub-volume, 16 bins (original samples): {time.time() - t:.1f} s")
    return host, cols, ref_o


def _subvolume(img):
    nb = img.shape[0]
    w = C3_IX[1] - C3_IX[0]
    return img[:, C3_IX[0]:C3_IX[1], C3_IX[0]:C3_IX[1], C3_IZ[0]:C3_IZ[1]].reshape(nb * w * w, -1)


@pytest.mark.parametrize("kind", ["bf16", "f16"])
def test_survey3d_16bit(ops, oracle_lib, survey3d, c3_subvolume, kind):
    # Whole sub-volume, all bins: the kernel against the oracle on the
    # dequantised samples (the kernel's own error: 1e-5), and the storage error
    # against the oracle on the original samples (reported; quantisation-bound).
    p, dp = survey3d
    host, cols, ref_o = c3_subvolume
    bits, sig, deq = survey.quantise(host, kind)
    dq = dp.with_data(torch.from_numpy(bits.view(np.int16)).cuda(), torch.from_numpy(sig).cuda(), kind)
    g16 = _subvolume(ops.migrate(dq)).double().cpu().numpy()
    g32 = _subvolume(ops.migrate(dp)).double().cpu().numpy()
    t = time.time()
    ref_q = oracle_lib.migrate_window(p, cols, *C3_IZ, data=deq)
    e_kernel = rel_l2(g16, ref_q)
    e_store = rel_l2(g16, ref_o)
    e_f32 = rel_l2(g32, ref_o)
    print(f"{kind}, 64 x 64 x 100 x 16 bins: vs oracle(dequantised) {e_kernel:.3e}; vs oracle(original) "
          f"{e_store:.3e}; f32 vs oracle {e_f32:.3e} (oracle {time.time() - t:.1f} s)")
    assert e_kernel <= 1e-5
    assert e_f32 <= 1e-5
    assert e_store <= (1e-2 if kind == "bf16" else 1e-3)


@pytest.fixture(scope="module")
def line2d_vz(ops):
    p = survey.make_line2d_vz()
    return p, ops.to_device(p, "cuda")


def test_line2d_vz_dot_product(ops, line2d_vz):
    p, dp = line2d_vz
    d = torch.from_numpy(survey.random_data(p, 41)).cuda()
    m = torch.from_numpy(survey.random_image(p, 42)).cuda()
    Md = ops.migrate(dp, data=d, dtype="f32")
    Mtm = ops.demigrate(dp, m)
    lhs = float(ops.dot_f64(Md, m))
    rhs = float(ops.dot_f64(d, Mtm))
    e = abs(lhs - rhs) / max(abs(lhs), abs(rhs))
    en = abs(lhs - rhs) / (float(ops.dot_f64(Md, Md)) ** 0.5 * float(ops.dot_f64(m, m)) ** 0.5)
    print(f"line2d_vz dot test: <Md,m> {lhs:.12e} <d,M^T m> {rhs:.12e} rel {e:.3e} (|a-b|/(|Md||m|) {en:.3e})")
    assert e < 1e-6


def test_line2d_vz_fd_and_lsm(ops, line2d_vz):
    from paper_1204_1225_amd import autograd, lsm

    p, dp = line2d_vz
    rng = np.random.default_rng(4)
    m_true = torch.zeros(p.image_shape, device="cuda")
    for _ in range(50):
        m_true[:, 0, rng.integers(100, p.nx - 100), rng.integers(100, p.nz - 50)] = 1.0
    d_obs = ops.demigrate(dp, m_true)
    m = torch.zeros(p.image_shape, device="cuda", requires_grad=True)

    def J(mm):
        r = autograd.demigrate(mm, dp) - d_obs
        return 0.5 * ops.dot_f64(r.contiguous(), r.contiguous())

    # gradient at m = 0.3 m_true (J is quadratic: central differences are exact up to rounding)
    m0 = (0.3 * m_true).requires_grad_(True)
    r0 = autograd.demigrate(m0, dp) - d_obs
    (0.5 * (r0.double() ** 2).sum()).backward()
    g = m0.grad.double()
    worst = 0.0
    for k in range(16):
        delta = torch.from_numpy(np.random.default_rng(43 + k).standard_normal(p.image_shape).astype(np.float32)).cuda()
        eps = 0.1 * float(m0.detach().norm()) / float(delta.norm())
        with torch.no_grad():
            fd = (float(J(m0 + eps * delta)) - float(J(m0 - eps * delta))) / (2 * eps)
        an = float((g * delta.double()).sum())
        worst = max(worst, abs(fd - an) / abs(an))
    print(f"line2d_vz finite differences, 16 perturbations: worst rel error {worst:.3e}")
    assert worst < 1e-4
    res = lsm.lsm(dp, d_obs, n_iter=10)
    J0, J10 = res.objective[0], res.objective[-1]
    print(f"line2d_vz LSM 10 steps: J {J0:.6e} -> {J10:.6e} (reduction {J10 / J0:.4f})")
    assert all(res.objective[k + 1] <= res.objective[k] for k in range(10))
    for k in range(10):  # exact line search on a quadratic: decrease = |g|^4 / (2 |Lg|^2)
        dec = res.objective[k] - res.objective[k + 1]
        assert abs(dec - res.predicted_decrease[k]) <= 1e-3 * res.objective[0]
    assert J10 < J0


def test_batch_matches_single_launches(ops, oracle_lib):
    # a reduced uneven batch (8 lines with the batch's shape distribution scaled down)
    shapes = [(max(16, s[0] // 8), max(48, s[1] // 4), s[2] // 2, max(64, s[3] // 8), s[4] // 2)
              for s in survey.batch_line_shapes(5)[:8]]
    probs, dps = [], []
    for i, sh in enumerate(shapes):
        p = survey.make_batch_line(sh, i)
        rng = np.random.default_rng(100 + i)
        p.data = survey.bandlimited_noise(rng, p.n_traces, p.n_t, p.dt)
        probs.append(p)
        dps.append(ops.to_device(p, "cuda"))
    imgs = [torch.full(dp.image_shape, float("nan"), device="cuda") for dp in dps]
    b = ops.Batch(dps, imgs, tile=0)
    b.run()
    torch.cuda.synchronize()
    n_items, n_wg = b.info()
    print(f"batch of {len(dps)} lines: {n_items} work items on {n_wg} persistent workgroups")
    for k in range(2):  # graph replays agree with single launches, replay after replay
        for dp, img in zip(dps, imgs):
            ref = ops.migrate(dp, tile=0)
            assert torch.equal(img, ref)
        b.run()
        torch.cuda.synchronize()
    for i in (0, 3):
        e = rel_l2(imgs[i].cpu().numpy(), oracle_lib.migrate(probs[i]))
        print(f"batch line {i} vs oracle: rel L2 {e:.3e}")
        assert e <= 1e-5
    b.close()


def test_batch_seed5_full(ops, oracle_lib):
    # The uneven 64-line batch of seed 5 at full size (about 36 GB of traces),
    # with both time precisions: every image of the persistent, graph-captured
    # launch equals the single launch of its line bit for bit, and the 4
    # smallest lines, which carry 3 point diffractors each (the others N(0, 1)
    # samples), match the oracle: 1e-5 with the extended time; with the float32
    # time the derived bound 5e-5 (records up to 2427 samples, where an ulp of u
    # is up to 2.4e-4 samples; the deepest line measured 1.06e-5).
    shapes = survey.batch_line_shapes(5)
    work = [s[0] * s[1] * s[3] * s[4] for s in shapes]
    small = [int(i) for i in np.argsort(work)[:4]]
    gen = torch.Generator(device="cuda").manual_seed(5)
    dps, lines = [], {}
    t = time.time()
    for i, sh in enumerate(shapes):
        p = survey.make_batch_line(sh, i)
        dp = ops.to_device(p, "cuda")
        if i in small:
            survey.with_diffractors(p, 50 + i, device="cuda")
            lines[i] = p
            dp = dp.with_data(torch.from_numpy(p.data).cuda())
        else:
            dp = dp.with_data(torch.randn((dp.n_traces, dp.n_t), generator=gen, device="cuda"))
        dps.append(dp)
    torch.cuda.synchronize()
    print(f"seed-5 batch generated in {time.time() - t:.1f} s")
    refs = {i: oracle_lib.migrate(lines[i]) for i in small}
    tile = 2
    imgs = [torch.full(dp.image_shape, float("nan"), device="cuda") for dp in dps]
    for prec, tol in [("extended", 1e-5), ("fp32", 5e-5)]:
        dpp = [dp.with_precision(prec) for dp in dps]
        b = ops.Batch(dpp, imgs, tile=tile)
        b.run()
        torch.cuda.synchronize()
        n_items, n_wg = b.info()
        for dp, img in zip(dpp, imgs):
            assert torch.equal(img, ops.migrate(dp, tile=tile))
        print(f"{prec}: 64 lines, {n_items} work items on {n_wg} workgroups, all equal to single launches")
        for i in small:
            e = rel_l2(imgs[i].cpu().numpy(), refs[i])
            print(f"{prec}: diffractor line {i} {shapes[i]}: rel L2 vs oracle {e:.3e}")
            assert e <= tol, (prec, i)
        b.close()
