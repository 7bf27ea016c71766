"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every entry point include/kirchhoff.h declares, and rejects bad arguments on
the host before launching anything."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "kirchhoff.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s*((?:km|kirchhoff)_[A-Za-z0-9_]+)\s*\(", src,
                       flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    from paper_1204_1225_amd import _lib

    if not os.path.exists(_lib.LIB_PATH):
        from paper_1204_1225_amd import build

        build.build(verbose=False)
    return _lib.load()


def test_exports_every_declared_symbol(lib):
    from paper_1204_1225_amd import _lib

    names = declared_functions()
    assert len(names) >= 18
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(_lib.SIGNATURES), "binding and header disagree"


def test_abi_version_and_limits(lib):
    from paper_1204_1225_amd import _lib

    assert lib.km_abi_version() == _lib.ABI_VERSION == 4
    assert lib.km_max_samples() >= 20000
    assert lib.km_tile_count(0) >= 2 and lib.km_tile_count(1) >= 2
    assert lib.km_tile_count(7) == 0


def test_tile_describe(lib):
    from paper_1204_1225_amd import _lib

    info = _lib.KmTileInfo()
    assert lib.km_tile_describe(0, 0, ctypes.byref(info)) == _lib.KM_OK
    assert info.waves >= 1 and info.depth_slots >= 1 and info.lds_budget > 0
    assert lib.km_tile_describe(0, 99, ctypes.byref(info)) == _lib.KM_E_INVALID
    assert b"out of range" in lib.km_last_error()


def _args(_lib, **over):
    t = _lib.KmTraces(n_traces=4, n_samples=10, dtype=_lib.KM_F32, trace_stride=10, t_first=0.0, dt=0.004,
                      data=ctypes.c_void_p(0x1000), scale=None, src=ctypes.c_void_p(0x1000),
                      rec=ctypes.c_void_p(0x1000), bin=ctypes.c_void_p(0x1000))
    g = _lib.KmGrid(nx=2, ny=1, nz=3, n_bins=1, x=ctypes.c_void_p(0x1000), y=ctypes.c_void_p(0x1000))
    tt = _lib.KmTraveltime(t0sq=ctypes.c_void_p(0x1000), s2=ctypes.c_void_p(0x1000), r2=ctypes.c_void_p(0x1000))
    w = _lib.KmWeight(kind=1)
    for k, v in over.items():
        obj, field = k.split("__")
        setattr({"t": t, "g": g, "tt": tt, "w": w}[obj], field, v)
    return t, g, tt, w


@pytest.mark.parametrize("over,status,msg", [
    ({"t__dt": 0.0}, 1, b"dt"),
    ({"t__n_traces": -1}, 1, b"n_traces"),
    ({"t__trace_stride": 5}, 1, b"trace_stride"),
    ({"t__dtype": 9}, 1, b"dtype"),
    ({"t__data": None}, 1, b"data"),
    ({"t__scale": ctypes.c_void_p(0x1000)}, 1, b"scale"),
    ({"t__n_samples": 10 ** 6, "t__trace_stride": 10 ** 6}, 2, b"km_max_samples"),
    ({"w__kind": 5}, 1, b"weight"),
    ({"tt__time_precision": 7}, 1, b"time precision"),
    ({"g__x": None}, 1, b"x and y"),
    ({"tt__r2": None}, 1, b"r2"),
    ({"g__nx": -3}, 1, b"negative"),
    ({"t__src": ctypes.c_void_p(0x1002)}, 1, b"aligned"),
])
def test_migrate_rejects_bad_arguments(lib, over, status, msg):
    from paper_1204_1225_amd import _lib

    t, g, tt, w = _args(_lib, **over)
    st = lib.kirchhoff_migrate(ctypes.byref(t), ctypes.byref(g), ctypes.byref(tt), ctypes.byref(w),
                               ctypes.c_void_p(0x1000), 0, -1, None)
    assert st == status
    assert msg in lib.km_last_error()


def test_demigrate_rejects_16bit_output_and_null_image(lib):
    from paper_1204_1225_amd import _lib

    t, g, tt, w = _args(_lib, t__dtype=_lib.KM_BF16)
    st = lib.kirchhoff_demigrate(ctypes.c_void_p(0x1000), ctypes.byref(g), ctypes.byref(tt), ctypes.byref(w),
                                 ctypes.byref(t), 0, -1, None)
    assert st == _lib.KM_E_UNSUPPORTED
    t, g, tt, w = _args(_lib)
    st = lib.kirchhoff_demigrate(None, ctypes.byref(g), ctypes.byref(tt), ctypes.byref(w), ctypes.byref(t), 0, -1,
                                 None)
    assert st == _lib.KM_E_INVALID


def test_null_struct_and_bad_tile(lib):
    from paper_1204_1225_amd import _lib

    t, g, tt, w = _args(_lib)
    assert lib.kirchhoff_migrate(None, ctypes.byref(g), ctypes.byref(tt), ctypes.byref(w), ctypes.c_void_p(0x1000), 0,
                                 -1, None) == _lib.KM_E_INVALID
    assert lib.kirchhoff_migrate(ctypes.byref(t), ctypes.byref(g), ctypes.byref(tt), ctypes.byref(w),
                                 ctypes.c_void_p(0x1000), 0, 42, None) == _lib.KM_E_INVALID
    assert b"tile" in lib.km_last_error()


def test_reductions_reject_bad_arguments(lib):
    from paper_1204_1225_amd import _lib

    assert lib.km_dot_f64(None, None, -1, ctypes.c_void_p(0x1000), None) == _lib.KM_E_INVALID
    assert lib.km_dot_f64(None, None, 5, ctypes.c_void_p(0x1000), None) == _lib.KM_E_INVALID
    assert lib.km_axpby(float("nan"), ctypes.c_void_p(0x1000), 1.0, ctypes.c_void_p(0x1000), 4, None) == \
        _lib.KM_E_INVALID
    h = ctypes.c_void_p()
    assert lib.km_batch_create(None, 0, 0, -1, None, ctypes.byref(h)) == _lib.KM_E_INVALID
    assert lib.km_batch_create(None, 1, 2, -1, None, ctypes.byref(h)) == _lib.KM_E_INVALID
    assert lib.km_batch_create(None, 1, 1, -1, None, ctypes.byref(h)) == _lib.KM_E_UNSUPPORTED
    assert b"not built" in lib.km_last_error()
    assert lib.km_batch_run(None, None) == _lib.KM_E_INVALID


def test_tune_cache_roundtrip(lib):
    from paper_1204_1225_amd import _lib

    # class key: (arch, op, dtype, kind, precision, nz / 128, n_samples / 512)
    assert lib.km_tune_lookup(0, 0, 0, 0, 4000, 7000) == -1
    assert lib.km_tune_record(0, 0, 0, 0, 4000, 7000, 1, 3.5) == _lib.KM_OK
    assert lib.km_tune_lookup(0, 0, 0, 0, 4000, 7000) == 1
    assert lib.km_tune_lookup(0, 0, 0, 0, 4010, 7100) == 1  # same class
    assert lib.km_tune_lookup(0, 0, 1, 0, 4000, 7000) == -1  # table times: another class
    assert lib.km_tune_lookup(0, 0, 0, 1, 4000, 7000) == -1  # extended time: another class
    assert lib.km_tune_record(0, 0, 0, 0, 4000, 7000, 99, 1.0) == _lib.KM_E_INVALID
    assert lib.km_tune_record(0, 0, 7, 0, 4000, 7000, 1, 1.0) == _lib.KM_E_INVALID
    assert lib.km_tune_record(1, 0, 0, 0, 4000, 7000, 1 + 64 * 3, 1.0) == _lib.KM_OK  # 16 waves x 8 slots x 3 quads


def test_tiles_encode_shape_and_level(lib):
    from paper_1204_1225_amd import _lib

    info = _lib.KmTileInfo()
    assert (lib.km_tile_levels(0), lib.km_tile_levels(1)) == (6, 4)
    for op in (0, 1):
        for sh in range(lib.km_tile_count(op)):
            assert lib.km_tile_describe(op, sh, ctypes.byref(info)) == _lib.KM_OK
            assert (info.shape, info.level, info.lds16) == (sh, 0, 0)
    # migrate levels scale the trace block's budget (at most 160 KiB); levels
    # 4 and 5 stage 16-bit traces with budgets 1 and 2
    assert lib.km_tile_describe(0, 2, ctypes.byref(info)) == _lib.KM_OK
    base = info.lds_budget
    assert lib.km_tile_describe(0, 2 + 64, ctypes.byref(info)) == _lib.KM_OK and info.lds_budget == base // 2
    assert lib.km_tile_describe(0, 2 + 192, ctypes.byref(info)) == _lib.KM_OK and info.lds_budget == 2 * base
    assert info.lds16 == 0
    assert lib.km_tile_describe(0, 2 + 256, ctypes.byref(info)) == _lib.KM_OK
    assert (info.lds_budget, info.lds16, info.level) == (base, 1, 4)
    assert lib.km_tile_describe(0, 2 + 320, ctypes.byref(info)) == _lib.KM_OK
    assert (info.lds_budget, info.lds16) == (2 * base, 1)
    assert lib.km_tile_describe(0, 2 + 384, ctypes.byref(info)) == _lib.KM_E_INVALID
    assert lib.km_tile_describe(1, 3 + 256, ctypes.byref(info)) == _lib.KM_E_INVALID
    # demigrate levels pick the trace quads per workgroup, up to the shape's
    assert lib.km_tile_describe(1, 3 + 64, ctypes.byref(info)) == _lib.KM_OK and info.trace_quads == 1
    assert lib.km_tile_describe(1, 3 + 128, ctypes.byref(info)) == _lib.KM_E_INVALID  # one-quad shape


def test_tune_cache_persists_across_processes(tmp_path):
    # KM_TUNE_CACHE: a record written by one process is read by the next
    # (host calls only: no GPU; the class key then carries arch "unknown").
    import json
    import os
    import subprocess
    import sys

    path = tmp_path / "tune.json"
    code = ("import sys; sys.path.insert(0, {root!r})\n"
            "from paper_1204_1225_amd import _lib\n"
            "lib = _lib.load()\n"
            "{body}\n")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    env = dict(os.environ, KM_TUNE_CACHE=str(path), HIP_VISIBLE_DEVICES="")
    write = "assert lib.km_tune_record(1, 0, 2, 0, 900, 3000, 3, 12.5) == 0\n" \
            "assert lib.km_tune_record(0, 1, 0, 1, 300, 1500, 2 + 64, 7.25) == 0"
    subprocess.run([sys.executable, "-c", code.format(root=root, body=write)], env=env, check=True)
    doc = json.loads(path.read_text())
    assert doc["format"] == "km_tune_cache" and len(doc["entries"]) == 2
    e = {(x["op"], x["kind"]): x for x in doc["entries"]}
    assert e[(1, 2)]["tile"] == 3 and e[(1, 2)]["nz_bucket"] == 8 and e[(1, 2)]["nt_bucket"] == 6
    assert e[(0, 0)]["tile"] == 66 and e[(0, 0)]["precision"] == 1 and e[(0, 0)]["dtype"] == 1
    read = "assert lib.km_tune_lookup(1, 0, 2, 0, 900, 3000) == 3\n" \
           "assert lib.km_tune_lookup(0, 1, 0, 1, 300, 1500) == 66\n" \
           "assert lib.km_tune_lookup(0, 0, 0, 1, 300, 1500) == -1"
    subprocess.run([sys.executable, "-c", code.format(root=root, body=read)], env=env, check=True)


def test_stack_and_moveout_reject_bad_arguments(lib):
    from paper_1204_1225_amd import _lib

    p = ctypes.c_void_p(0x1000)
    assert lib.km_stack_offsets(p, 0, 10, p, None) == _lib.KM_E_INVALID
    assert lib.km_stack_offsets(p, 2, -1, p, None) == _lib.KM_E_INVALID
    assert lib.km_stack_offsets(None, 2, 10, p, None) == _lib.KM_E_INVALID
    assert lib.km_stack_offsets(ctypes.c_void_p(0x1002), 2, 10, p, None) == _lib.KM_E_INVALID
    assert lib.km_stack_offsets(None, 2, 0, None, None) == _lib.KM_OK  # nothing to do
    g = _lib.KmGrid(nx=4, ny=2, nz=50, n_bins=3, x=None, y=None)
    gp = ctypes.byref(g)
    cases = [
        ((p, gp, p, -1, 0, 50, None, p, None, None), _lib.KM_E_INVALID, b"max_lag"),
        ((p, gp, p, 300, 0, 50, None, p, None, None), _lib.KM_E_UNSUPPORTED, b"max_lag"),
        ((p, gp, p, 4, 10, 10, None, p, None, None), _lib.KM_E_INVALID, b"window"),
        ((p, gp, p, 4, 0, 51, None, p, None, None), _lib.KM_E_INVALID, b"window"),
        ((None, gp, p, 4, 0, 50, None, p, None, None), _lib.KM_E_INVALID, b"non-NULL"),
        ((p, gp, p, 4, 0, 50, None, None, None, None), _lib.KM_E_INVALID, b"non-NULL"),
        ((p, gp, None, 4, 0, 50, None, p, None, p), _lib.KM_E_INVALID, b"offsets"),
        ((p, gp, p, 4, 0, 50, ctypes.c_void_p(0x1001), p, None, None), _lib.KM_E_INVALID, b"misaligned"),
    ]
    for args, status, msg in cases:
        assert lib.km_cig_moveout(*args, None) == status, args
        assert msg in lib.km_last_error()
    big = _lib.KmGrid(nx=4, ny=2, nz=20000, n_bins=16, x=None, y=None)
    assert lib.km_cig_moveout(p, ctypes.byref(big), p, 4, 0, 100, None, p, None, None, None) == \
        _lib.KM_E_UNSUPPORTED
    assert b"LDS" in lib.km_last_error()


def test_trace_filter_rejects_bad_arguments(lib):
    from paper_1204_1225_amd import _lib

    p = ctypes.c_void_p(0x1000)
    q = ctypes.c_void_p(0x10000000)  # far enough from p that the buffers do not overlap
    cases = [
        ((p, 10, q, 10, -1, 10, p, 3, 1, 0), _lib.KM_E_INVALID, b"negative"),
        ((p, 10, q, 10, 4, 10, p, 0, 0, 0), _lib.KM_E_INVALID, b"n_taps"),
        ((p, 10, q, 10, 4, 10, p, 2000, 0, 0), _lib.KM_E_UNSUPPORTED, b"n_taps"),
        ((p, 10, q, 10, 4, 10, p, 3, 3, 0), _lib.KM_E_INVALID, b"center"),
        ((p, 10, q, 10, 4, 10, p, 3, -1, 0), _lib.KM_E_INVALID, b"center"),
        ((p, 5, q, 10, 4, 10, p, 3, 1, 0), _lib.KM_E_INVALID, b"stride"),
        ((None, 10, q, 10, 4, 10, p, 3, 1, 0), _lib.KM_E_INVALID, b"NULL"),
        ((p, 10, ctypes.c_void_p(0x1010), 10, 4, 10, p, 3, 1, 0), _lib.KM_E_INVALID, b"overlap"),
        ((p, 40000, q, 40000, 4, 40000, p, 1024, 1, 0), _lib.KM_E_UNSUPPORTED, b"LDS"),
    ]
    for args, status, msg in cases:
        assert lib.km_trace_filter(*args, None) == status, args
        assert msg in lib.km_last_error()
    assert lib.km_trace_filter(None, 10, None, 10, 0, 10, None, 3, 1, 0, None) == _lib.KM_OK


def test_table_entry_points_reject_bad_tables(lib):
    from paper_1204_1225_amd import _lib

    t, g, tt, w = _args(_lib)
    p = ctypes.c_void_p(0x1000)
    for tab, msg in [(None, b"NULL"), (_lib.KmTtable(n_h=1, dh=10.0, t=p, r2=p), b"n_h"),
                     (_lib.KmTtable(n_h=4, dh=0.0, t=p, r2=p), b"dh"),
                     (_lib.KmTtable(n_h=4, dh=float("inf"), t=p, r2=p), b"dh"),
                     (_lib.KmTtable(n_h=4, dh=10.0, t=None, r2=p), b"non-NULL"),
                     (_lib.KmTtable(n_h=4, dh=10.0, t=ctypes.c_void_p(0x1002), r2=p), b"misaligned"),
                     (_lib.KmTtable(n_h=4, dh=10.0, t=p, r2=p, amp=ctypes.c_void_p(0x1001)), b"misaligned")]:
        ref = ctypes.byref(tab) if tab is not None else None
        assert lib.kirchhoff_migrate_table(ctypes.byref(t), ctypes.byref(g), ref, p, 0, -1, None) == _lib.KM_E_INVALID
        assert msg in lib.km_last_error()
        assert lib.kirchhoff_demigrate_table(p, ctypes.byref(g), ref, ctypes.byref(t), 0, -1, None) == \
            _lib.KM_E_INVALID
    big = _lib.KmTtable(n_h=1 << 30, dh=1.0, t=p, r2=p)
    assert lib.kirchhoff_migrate_table(ctypes.byref(t), ctypes.byref(g), ctypes.byref(big), p, 0, -1, None) == \
        _lib.KM_E_UNSUPPORTED


def test_ltable_entry_points_reject_bad_tables(lib):
    from paper_1204_1225_amd import _lib

    t, g, tt, w = _args(_lib)
    p = ctypes.c_void_p(0x1000)

    def lt(**over):
        f = dict(n_h=4, dh=10.0, n_gx=3, n_gy=2, gx0=0.0, gy0=0.0, gdx=100.0, gdy=100.0, t=p, r2=p)
        f.update(over)
        return _lib.KmLtable(**f)

    for tab, msg in [(None, b"NULL"), (lt(n_gx=0), b"n_gx and n_gy"), (lt(n_gy=-1), b"n_gx and n_gy"),
                     (lt(gx0=float("nan")), b"gx0 and gy0"), (lt(gy0=float("inf")), b"gx0 and gy0"),
                     (lt(gdx=0.0), b"gdx"), (lt(gdy=-5.0), b"gdx"), (lt(gdx=float("inf")), b"gdx"),
                     (lt(n_h=1), b"n_h"), (lt(dh=0.0), b"dh"), (lt(t=None), b"non-NULL"),
                     (lt(r2=ctypes.c_void_p(0x1002)), b"misaligned"), (lt(amp=ctypes.c_void_p(0x1003)), b"misaligned")]:
        ref = ctypes.byref(tab) if tab is not None else None
        assert lib.kirchhoff_migrate_ltable(ctypes.byref(t), ctypes.byref(g), ref, p, 0, -1, None) == \
            _lib.KM_E_INVALID
        assert msg in lib.km_last_error()
        assert lib.kirchhoff_demigrate_ltable(p, ctypes.byref(g), ref, ctypes.byref(t), 0, -1, None) == \
            _lib.KM_E_INVALID
        assert msg in lib.km_last_error()
    # the tuner validates the table the same way (before any launch)
    assert lib.km_tune_ltable(0, ctypes.byref(t), ctypes.byref(g), None, p, 1, None, None, None) == _lib.KM_E_INVALID
    assert lib.km_tune_ltable(0, ctypes.byref(t), ctypes.byref(g), ctypes.byref(lt(gdx=0.0)), p, 1, None, None,
                              None) == _lib.KM_E_INVALID
    assert b"gdx" in lib.km_last_error()
    # the spacing of an axis with one node is not read
    one = lt(n_gx=1, n_gy=1, gdx=0.0, gdy=float("nan"), n_h=1)
    assert lib.kirchhoff_migrate_ltable(ctypes.byref(t), ctypes.byref(g), ctypes.byref(one), p, 0, -1, None) == \
        _lib.KM_E_INVALID
    assert b"n_h" in lib.km_last_error()
    big = lt(n_gx=1 << 12, n_gy=1 << 12, n_h=64)
    assert lib.kirchhoff_migrate_ltable(ctypes.byref(t), ctypes.byref(g), ctypes.byref(big), p, 0, -1, None) == \
        _lib.KM_E_UNSUPPORTED


def test_antialias_entry_points_reject_bad_options(lib):
    from paper_1204_1225_amd import _lib

    t, g, tt, w = _args(_lib)
    p = ctypes.c_void_p(0x1000)
    for aa, msg in [(None, b"NULL"), (_lib.KmAntialias(dx=-1.0, dy=0.0, max_half=4), b"dx and dy"),
                    (_lib.KmAntialias(dx=10.0, dy=float("inf"), max_half=4), b"dx and dy"),
                    (_lib.KmAntialias(dx=10.0, dy=float("nan"), max_half=4), b"dx and dy"),
                    (_lib.KmAntialias(dx=10.0, dy=10.0, max_half=0), b"max_half"),
                    (_lib.KmAntialias(dx=10.0, dy=10.0, max_half=33), b"max_half")]:
        ref = ctypes.byref(aa) if aa is not None else None
        assert lib.kirchhoff_migrate_aa(ctypes.byref(t), ctypes.byref(g), ctypes.byref(tt), ctypes.byref(w), ref, p,
                                        0, -1, None) == _lib.KM_E_INVALID
        assert msg in lib.km_last_error()
        assert lib.kirchhoff_demigrate_aa(p, ctypes.byref(g), ctypes.byref(tt), ctypes.byref(w), ref,
                                          ctypes.byref(t), 0, -1, None) == _lib.KM_E_INVALID
        assert msg in lib.km_last_error()
    # the ordinary argument checks still apply
    ok = _lib.KmAntialias(dx=10.0, dy=10.0, max_half=8)
    t2, g2, tt2, w2 = _args(_lib, t__dt=0.0)
    assert lib.kirchhoff_migrate_aa(ctypes.byref(t2), ctypes.byref(g2), ctypes.byref(tt2), ctypes.byref(w2),
                                    ctypes.byref(ok), p, 0, -1, None) == _lib.KM_E_INVALID
    assert b"dt" in lib.km_last_error()


def test_plain_only_calls_reject_table_and_antialias_problems():
    # count (with n_effective) and Batch evaluate the plain square-root
    # operator; a table-traveltime or anti-aliased problem must raise instead
    # of silently running it (checked before any library call: no GPU needed).
    import dataclasses

    import torch

    from paper_1204_1225_amd import _lib, ops

    z = torch.zeros(4)
    base = ops.DeviceProblem(device=torch.device("cpu"), n_t=10, dt=0.004, t_first=0.0, n_bins=1, weight=1,
                             src=torch.zeros(2, 2), rec=torch.zeros(2, 2), bin=torch.zeros(2, dtype=torch.int32),
                             x=torch.zeros(3), y=torch.zeros(1), t0sq=z, s2=z, r2=z)
    for dp in [dataclasses.replace(base, ttab=torch.zeros(2, 4), tdh=1.0),
               dataclasses.replace(base, aa=(12.5, 12.5, 4))]:
        with pytest.raises(_lib.KirchhoffError) as e1:
            ops.count(dp)
        with pytest.raises(_lib.KirchhoffError) as e3:
            ops.Batch([dp], [torch.zeros(dp.image_shape)])
        assert e1.value.status == e3.value.status == _lib.KM_E_UNSUPPORTED


def test_batch_static_rejects_what_does_not_fit(lib):
    # The allocation-free batch checks its work list against the static scratch
    # before any HIP call (host validation only; the pointers are never used):
    # 4096 x 1024 columns in tiles of 128, 16 bins, one depth chunk is 524 288
    # work items, more than the scratch holds.
    from paper_1204_1225_amd import _lib

    t, g, tt, w = _args(_lib)
    g.nx, g.ny, g.nz, g.n_bins = 4096, 1024, 16, 16
    pr = (_lib.KmProblem * 1)()
    pr[0] = _lib.KmProblem(traces=t, grid=g, tt=tt, weight=w, image=ctypes.c_void_p(0x1000))
    assert lib.km_batch_migrate_static(pr, 1, 2, None) == _lib.KM_E_UNSUPPORTED
    assert b"scratch" in lib.km_last_error()
    big = (_lib.KmProblem * 4097)()
    g.nx, g.ny, g.nz, g.n_bins = 2, 1, 3, 1
    for k in range(4097):
        big[k] = _lib.KmProblem(traces=t, grid=g, tt=tt, weight=w, image=ctypes.c_void_p(0x1000))
    assert lib.km_batch_migrate_static(big, 4097, 2, None) == _lib.KM_E_UNSUPPORTED
    assert lib.km_batch_migrate_static(None, 0, -1, None) == _lib.KM_E_INVALID


def test_injected_launch_failure_is_reported(lib, monkeypatch):
    # KM_FAULT_INJECT=launch: a valid call reaches its launch and reports
    # KM_E_HIP with a message instead of launching (host only: the pointers
    # are never dereferenced, no GPU is touched); without it validation errors
    # still come first.
    from paper_1204_1225_amd import _lib

    t, g, tt, w = _args(_lib)
    p = ctypes.c_void_p(0x1000)
    monkeypatch.setenv("KM_FAULT_INJECT", "launch")
    assert lib.kirchhoff_migrate(ctypes.byref(t), ctypes.byref(g), ctypes.byref(tt), ctypes.byref(w), p, 0, 2,
                                 None) == _lib.KM_E_HIP
    assert b"migrate launch" in lib.km_last_error() and b"injected" in lib.km_last_error()
    assert lib.kirchhoff_demigrate(p, ctypes.byref(g), ctypes.byref(tt), ctypes.byref(w), ctypes.byref(t), 0, 3,
                                   None) == _lib.KM_E_HIP
    assert b"demigrate launch" in lib.km_last_error()
    assert lib.km_dot_f64(p, p, 16, p, None) == _lib.KM_E_HIP
    assert lib.km_axpby(1.0, p, 1.0, p, 16, None) == _lib.KM_E_HIP
    t_bad, g2, tt2, w2 = _args(_lib, t__dt=0.0)
    assert lib.kirchhoff_migrate(ctypes.byref(t_bad), ctypes.byref(g2), ctypes.byref(tt2), ctypes.byref(w2), p, 0,
                                 2, None) == _lib.KM_E_INVALID
    monkeypatch.setenv("KM_FAULT_INJECT", "other")
    assert lib.kirchhoff_migrate(ctypes.byref(t_bad), ctypes.byref(g2), ctypes.byref(tt2), ctypes.byref(w2), p, 0,
                                 2, None) == _lib.KM_E_INVALID


def test_16bit_staging_tiles_need_16bit_float32_time_plain_problems(lib, monkeypatch):
    # Host validation only (the pointers are never used): migrate levels 4 and
    # 5 take KM_BF16 / KM_F16 traces with float32 time and no anti-alias
    # filter; the batched calls refuse them.  With KM_FAULT_INJECT=launch a
    # valid call reaches its launch (KM_E_HIP) without touching a GPU.
    from paper_1204_1225_amd import _lib

    p = ctypes.c_void_p(0x1000)
    for tile in (2 + 256, 0 + 320):
        t, g, tt, w = _args(_lib)
        st = lib.kirchhoff_migrate(ctypes.byref(t), ctypes.byref(g), ctypes.byref(tt), ctypes.byref(w), p, 0, tile,
                                   None)
        assert st == _lib.KM_E_UNSUPPORTED and b"16-bit" in lib.km_last_error()
        t, g, tt, w = _args(_lib, t__dtype=_lib.KM_BF16, t__scale=p, tt__time_precision=_lib.KM_TIME_EXTENDED)
        st = lib.kirchhoff_migrate(ctypes.byref(t), ctypes.byref(g), ctypes.byref(tt), ctypes.byref(w), p, 0, tile,
                                   None)
        assert st == _lib.KM_E_UNSUPPORTED and b"16-bit" in lib.km_last_error()
        t, g, tt, w = _args(_lib, t__dtype=_lib.KM_F16, t__scale=p)
        aa = _lib.KmAntialias(dx=10.0, dy=10.0, max_half=2)
        st = lib.kirchhoff_migrate_aa(ctypes.byref(t), ctypes.byref(g), ctypes.byref(tt), ctypes.byref(w),
                                      ctypes.byref(aa), p, 0, tile, None)
        assert st == _lib.KM_E_UNSUPPORTED and b"16-bit" in lib.km_last_error()
        pr = (_lib.KmProblem * 1)()
        pr[0] = _lib.KmProblem(traces=t, grid=g, tt=tt, weight=w, image=p)
        assert lib.km_batch_migrate_static(pr, 1, tile, None) == _lib.KM_E_UNSUPPORTED
        assert b"not batched" in lib.km_last_error()
        monkeypatch.setenv("KM_FAULT_INJECT", "launch")
        st = lib.kirchhoff_migrate(ctypes.byref(t), ctypes.byref(g), ctypes.byref(tt), ctypes.byref(w), p, 0, tile,
                                   None)
        assert st == _lib.KM_E_HIP and b"injected" in lib.km_last_error()
        monkeypatch.delenv("KM_FAULT_INJECT")


def test_tuned_tiles_must_apply_to_their_class(lib, tmp_path):
    # km_tune_record refuses a 16-bit staging tile for a class that cannot run
    # it; a cache file holding one (written by hand here) is ignored by calls
    # with tile = -1, which take the default and reach their launch (host only:
    # KM_FAULT_INJECT=launch reports KM_E_HIP instead of launching).
    import json
    import subprocess
    import sys

    from paper_1204_1225_amd import _lib

    assert lib.km_tune_record(0, _lib.KM_F32, 0, 0, 3, 10, 2 + 256, 1.0) == _lib.KM_E_INVALID
    assert b"16-bit" in lib.km_last_error()
    assert lib.km_tune_record(0, _lib.KM_BF16, 0, 1, 3, 10, 2 + 256, 1.0) == _lib.KM_E_INVALID
    assert lib.km_tune_record(0, _lib.KM_BF16, 2, 0, 3, 10, 2 + 256, 1.0) == _lib.KM_E_INVALID
    code = (f"import ctypes, json, sys; sys.path.insert(0, {ROOT!r})\n"
            "from paper_1204_1225_amd import _lib\n"
            "from tests.test_abi import _args\n"
            "lib = _lib.load()\n"
            "t, g, tt, w = _args(_lib)\n"
            "p = ctypes.c_void_p(0x1000)\n"
            "print(lib.km_tune_lookup(0, 0, 0, 0, 3, 10), lib.kirchhoff_migrate(ctypes.byref(t), ctypes.byref(g), "
            "ctypes.byref(tt), ctypes.byref(w), p, 0, -1, None), lib.km_last_error().decode())\n")
    path = tmp_path / "tune.json"
    path.write_text(json.dumps({"format": "km_tune_cache", "version": 1, "entries": [
        {"arch": "unknown", "op": 0, "dtype": 0, "kind": 0, "precision": 0, "nz_bucket": 1, "nt_bucket": 1,
         "tile": 2 + 256, "ms": 1.0}]}))
    env = dict(os.environ, KM_TUNE_CACHE=str(path), KM_FAULT_INJECT="launch", HIP_VISIBLE_DEVICES="")
    r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    looked, status, msg = r.stdout.split(maxsplit=2)
    assert int(looked) == 2 + 256 and int(status) == _lib.KM_E_HIP and "injected" in msg
