"""FP64 CPU oracle for Kirchhoff prestack migration (Eq. (1), Section 3).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
benchmark's CPU-baseline leg, never by the GPU library or its binding.  The
arithmetic lives in kirchhoff_oracle.c (plain C, FP64, OpenMP over image
columns or traces); this module only loads it and passes numpy arrays.

Every function takes a problem object with the attributes of a survey
problem (src, rec, bin, n_t, dt, t_first, x, y, t0sq, s2, r2, weight,
n_bins, and optionally a one-way traveltime table ttab [n_h][nz] with
spacing tdh, which replaces the t0sq / s2 form, or with tgrid = (gx0, gy0,
gdx, gdy) a laterally varying table ttab [n_gy][n_gx][n_h][nz] on the node
grid (gx0 + i gdx, gy0 + j gdy), with optionally tamp, one-way amplitudes of
the same layout (W = A_s A_r instead of 1), and optionally aa = (dx, dy, max
half-width) for the anti-alias triangle filter) and, where samples are
needed, a float64 data array [n_traces, n_t] (default: the problem's own data
widened to float64).

Parity status: all functions are pinned by the CPU tests (closed forms,
invariants, adjoint identity, focusing); none is unpinned.  The pair counts
(count, count_columns) are pinned by hand counts of the 45-degree cone, per
column and in total, by exact-time cases that put u exactly at -1 and N_t and
strictly inside (-1, 0) and (N_t - 1, N_t), and by the identity between the
per-column and the total counts.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "kirchhoff_oracle.c")
# KM_ORACLE_LIBRARY names another build of the oracle (its sanitizer build)
_LIB = os.environ.get("KM_ORACLE_LIBRARY") or os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile liboracle.so with gcc (-O2, -ffp-contract=off, OpenMP, no fast-math)."""
    if force or not os.path.exists(_LIB):
        cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-Wall",
               "-shared", "-fPIC", _SRC, "-o", _LIB + ".tmp", "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


def build_sanitized(out: str) -> str:
    """The oracle with AddressSanitizer and UndefinedBehaviorSanitizer checks
    (clang, the same arithmetic flags); load it into a process that preloads
    clang's shared AddressSanitizer runtime."""
    cmd = ["/opt/rocm/llvm/bin/clang", "-O1", "-g", "-std=c11", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-shared-libasan",
           "-fno-omit-frame-pointer", "-shared", "-fPIC", _SRC, "-o", out, "-lm"]
    subprocess.run(cmd, check=True)
    return out


class _Problem(ctypes.Structure):
    _fields_ = [
        ("n_traces", ctypes.c_int64), ("n_t", ctypes.c_int32),
        ("t_first", ctypes.c_double), ("dt", ctypes.c_double),
        ("data", ctypes.c_void_p), ("src", ctypes.c_void_p), ("rec", ctypes.c_void_p),
        ("bin", ctypes.c_void_p),
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32), ("n_bins", ctypes.c_int32),
        ("x", ctypes.c_void_p), ("y", ctypes.c_void_p),
        ("t0sq", ctypes.c_void_p), ("s2", ctypes.c_void_p), ("r2", ctypes.c_void_p),
        ("weight", ctypes.c_int32),
        ("n_h", ctypes.c_int32), ("dh", ctypes.c_double), ("ttab", ctypes.c_void_p),
        ("aa_dx", ctypes.c_double), ("aa_dy", ctypes.c_double), ("aa_max", ctypes.c_int32),
        ("n_gx", ctypes.c_int32), ("n_gy", ctypes.c_int32), ("gx0", ctypes.c_double), ("gy0", ctypes.c_double),
        ("gdx", ctypes.c_double), ("gdy", ctypes.c_double), ("tamp", ctypes.c_void_p),
    ]


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = ctypes.CDLL(_LIB)
        P = ctypes.POINTER(_Problem)
        vp, i64 = ctypes.c_void_p, ctypes.c_int64
        lib.oracle_migrate.argtypes = [P, vp]
        lib.oracle_migrate_columns.argtypes = [P, i64, vp, vp]
        lib.oracle_migrate_points.argtypes = [P, i64, vp, vp]
        lib.oracle_migrate_window.argtypes = [P, i64, vp, ctypes.c_int32, ctypes.c_int32, vp]
        lib.oracle_demigrate.argtypes = [P, vp, vp]
        lib.oracle_demigrate_samples.argtypes = [P, vp, i64, vp, vp]
        lib.oracle_count.argtypes = [P, ctypes.POINTER(i64), ctypes.POINTER(i64)]
        lib.oracle_count_columns.argtypes = [P, i64, vp, vp]
        lib.oracle_threads.argtypes = []
        _lib = lib
    return _lib


def _arr(a, dtype):
    return np.ascontiguousarray(np.asarray(a), dtype=dtype)


class _Bound:
    """ctypes view of a problem; keeps the numpy buffers alive."""

    def __init__(self, p, data=None, need_data=True):
        self.keep = {
            "src": _arr(p.src, np.float32), "rec": _arr(p.rec, np.float32), "bin": _arr(p.bin, np.int32),
            "x": _arr(p.x, np.float32), "y": _arr(p.y, np.float32),
            "t0sq": _arr(p.t0sq, np.float64), "s2": _arr(p.s2, np.float64), "r2": _arr(p.r2, np.float32),
        }
        if data is None and need_data:
            data = p.data
        if data is not None:
            data = np.asarray(data)
            if hasattr(data, "detach"):
                data = data.detach().cpu().numpy()
            self.keep["data"] = _arr(data, np.float64)
            assert self.keep["data"].shape == (self.keep["src"].shape[0], int(p.n_t))
        ttab = getattr(p, "ttab", None)
        tgrid = getattr(p, "tgrid", None)
        n_gx = n_gy = 0
        if ttab is not None:
            self.keep["ttab"] = t = _arr(ttab, np.float32)
            if tgrid is not None:
                assert t.ndim == 4, "a laterally varying table is [n_gy][n_gx][n_h][nz]"
                n_gy, n_gx = t.shape[0], t.shape[1]
            else:
                assert t.ndim == 2
            assert t.shape[-1] == self.keep["t0sq"].shape[0]
        k = self.keep
        self.s = _Problem(
            n_traces=k["src"].shape[0], n_t=int(p.n_t), t_first=float(p.t_first), dt=float(p.dt),
            data=k["data"].ctypes.data if "data" in k else None,
            src=k["src"].ctypes.data, rec=k["rec"].ctypes.data, bin=k["bin"].ctypes.data,
            nx=k["x"].shape[0], ny=k["y"].shape[0], nz=k["t0sq"].shape[0], n_bins=int(p.n_bins),
            x=k["x"].ctypes.data, y=k["y"].ctypes.data, t0sq=k["t0sq"].ctypes.data, s2=k["s2"].ctypes.data,
            r2=k["r2"].ctypes.data, weight=int(p.weight),
            n_h=k["ttab"].shape[-2] if "ttab" in k else 0, dh=float(getattr(p, "tdh", 0.0) or 0.0),
            ttab=k["ttab"].ctypes.data if "ttab" in k else None)
        tamp = getattr(p, "tamp", None)
        if tamp is not None:
            self.keep["tamp"] = _arr(tamp, np.float32)
            assert ttab is not None and self.keep["tamp"].shape == self.keep["ttab"].shape
            self.s.tamp = self.keep["tamp"].ctypes.data
        if n_gx:
            self.s.n_gx, self.s.n_gy = n_gx, n_gy
            self.s.gx0, self.s.gy0, self.s.gdx, self.s.gdy = (float(v) for v in tgrid)
        aa = getattr(p, "aa", None)  # (dx, dy, max half-width) or None
        if aa is not None:
            self.s.aa_dx, self.s.aa_dy, self.s.aa_max = float(aa[0]), float(aa[1]), int(aa[2])
        assert k["s2"].shape[0] == self.s.nz and k["r2"].shape[0] == self.s.nz

    @property
    def ref(self):
        return ctypes.byref(self.s)


def _image_shape(p):
    return (int(p.n_bins), len(p.y), len(p.x), len(p.t0sq))


def migrate(p, data=None) -> np.ndarray:
    """Full image [n_bins, ny, nx, nz] in FP64."""
    b = _Bound(p, data)
    out = np.zeros(_image_shape(p), dtype=np.float64)
    if _load().oracle_migrate(b.ref, out.ctypes.data) != 0:
        raise ValueError("oracle_migrate rejected the problem")
    return out


def migrate_columns(p, cols, data=None) -> np.ndarray:
    """Image columns cols[k] = (bin, iy, ix) -> [len(cols), nz] in FP64."""
    b = _Bound(p, data)
    cols = _arr(cols, np.int32).reshape(-1, 3)
    out = np.zeros((cols.shape[0], len(p.t0sq)), dtype=np.float64)
    if _load().oracle_migrate_columns(b.ref, cols.shape[0], cols.ctypes.data, out.ctypes.data) != 0:
        raise ValueError("oracle_migrate_columns rejected the problem")
    return out


def migrate_window(p, cols, z_lo, z_hi, data=None) -> np.ndarray:
    """Depths z_lo .. z_hi - 1 of image columns cols[k] = (bin, iy, ix) ->
    [len(cols), z_hi - z_lo] in FP64 (a sub-volume)."""
    b = _Bound(p, data)
    cols = _arr(cols, np.int32).reshape(-1, 3)
    out = np.zeros((cols.shape[0], int(z_hi) - int(z_lo)), dtype=np.float64)
    if _load().oracle_migrate_window(b.ref, cols.shape[0], cols.ctypes.data, int(z_lo), int(z_hi),
                                     out.ctypes.data) != 0:
        raise ValueError("oracle_migrate_window rejected the problem")
    return out


def migrate_points(p, pts, data=None) -> np.ndarray:
    """Image points pts[k] = (bin, iy, ix, iz) -> values in FP64."""
    b = _Bound(p, data)
    pts = _arr(pts, np.int32).reshape(-1, 4)
    out = np.zeros(pts.shape[0], dtype=np.float64)
    if _load().oracle_migrate_points(b.ref, pts.shape[0], pts.ctypes.data, out.ctypes.data) != 0:
        raise ValueError("oracle_migrate_points rejected the problem")
    return out


def demigrate(p, image) -> np.ndarray:
    """Adjoint: traces [n_traces, n_t] in FP64 from an image [n_bins, ny, nx, nz]."""
    b = _Bound(p, need_data=False)
    img = _arr(image, np.float64)
    assert img.shape == _image_shape(p)
    out = np.zeros((b.s.n_traces, int(p.n_t)), dtype=np.float64)
    if _load().oracle_demigrate(b.ref, img.ctypes.data, out.ctypes.data) != 0:
        raise ValueError("oracle_demigrate rejected the problem")
    return out


def demigrate_samples(p, image, samples) -> np.ndarray:
    """Adjoint at samples[k] = (trace, sample index) -> values in FP64."""
    b = _Bound(p, need_data=False)
    img = _arr(image, np.float64)
    assert img.shape == _image_shape(p)
    smp = _arr(samples, np.int64).reshape(-1, 2)
    out = np.zeros(smp.shape[0], dtype=np.float64)
    if _load().oracle_demigrate_samples(b.ref, img.ctypes.data, smp.shape[0], smp.ctypes.data,
                                        out.ctypes.data) != 0:
        raise ValueError("oracle_demigrate_samples rejected the problem")
    return out


def count(p):
    """(n_aperture, n_effective) pair counts of Eq. (2)."""
    b = _Bound(p, need_data=False)
    na, ne = ctypes.c_int64(0), ctypes.c_int64(0)
    if _load().oracle_count(b.ref, ctypes.byref(na), ctypes.byref(ne)) != 0:
        raise ValueError("oracle_count rejected the problem")
    return int(na.value), int(ne.value)


def count_columns(p, cols):
    """(n_aperture, n_effective) over image columns cols[k] = (bin, iy, ix)."""
    b = _Bound(p, need_data=False)
    cols = _arr(cols, np.int32).reshape(-1, 3)
    out = np.zeros(2, dtype=np.int64)
    if _load().oracle_count_columns(b.ref, cols.shape[0], cols.ctypes.data, out.ctypes.data) != 0:
        raise ValueError("oracle_count_columns rejected the problem")
    return int(out[0]), int(out[1])


def threads() -> int:
    """OpenMP threads the oracle's parallel loops use."""
    return int(_load().oracle_threads())
